/* bipqn.h -- C ABI of the MI355X (gfx950) mobility-product and PQN/Bi-PQN library.
 *
 * The operations follow the statement of the problem in Rummel, Jensen, Becker,
 * Corona, "A Bifidelity Proximal Quasi-Newton Method for Dense Rigid Body
 * Suspension Collision Resolution":
 *   - the rigid-body mobility product U = M F (Sec. 2, eq. (mobility); Fig. 1),
 *     computed by a second-kind boundary integral solve with GMRES inside;
 *   - the LCP 0 <= A x + b  perp  x >= 0 with A = D^T M D and
 *     b = Phi/dt + D^T U_nc (Sec. 3, eq. (LCP), eq. (defAandb)), solved by
 *     BB-PGD (eq. (spectralStepSize)), Mono-PQN (Alg. 1) or Bi-PQN (Alg. 4);
 *   - one forward-Euler step of the linearised DVI (Sec. 3, eq. (dvi)).
 *
 * Conventions (all entry points):
 *   - Every function returns pqn_status; PQN_OK = 0. A negative status means
 *     nothing was written to the outputs; pqn_last_error() then returns a
 *     message (thread-local, valid until the next call on the same thread).
 *     PQN_WARN_NOT_CONVERGED means outputs were written but an iteration cap
 *     was hit; the stats structure says which.
 *   - Pointers without a _dev suffix in the function name are HOST pointers
 *     owned by the caller; the library copies in and out and returns after
 *     the work has finished. _dev functions take DEVICE pointers on the
 *     context's device and return after the work has finished on the
 *     context's stream.
 *   - Forces/velocities are particle-major [M][6]: (Fx,Fy,Fz,Tx,Ty,Tz) and
 *     (Ux,Uy,Uz,Wx,Wy,Wz), the layout of the paper's vectors F and U (Sec. 2).
 *   - Surface fields are SoA [3][N] (all x components, then y, then z), node
 *     index t = sphere*n + theta_row*n_phi + phi_col, n = n_theta*n_phi,
 *     theta rows in ascending cos(theta).
 *   - A context is not thread-safe; use one context per host thread/stream.
 */
#ifndef BIPQN_H
#define BIPQN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pqn_ctx pqn_ctx;

typedef enum {
  PQN_OK = 0,
  PQN_WARN_NOT_CONVERGED = 1,
  PQN_ERR_INVALID = -1, /* bad argument or size */
  PQN_ERR_DEVICE = -2,  /* HIP runtime error */
  PQN_ERR_OOM = -3,     /* device allocation failed */
  PQN_ERR_NUMERIC = -4, /* NaN/Inf encountered */
  PQN_ERR_STATE = -5,   /* call not valid in the context's state */
  PQN_ERR_INDEFINITE = -6 /* pqn_step: the contact LCP met p.Ap <= 0 (A = D^T M D not positive
                             definite) and did not converge; the configuration is unchanged */
} pqn_status;

typedef enum { PQN_FP64 = 0, PQN_MIXED = 1 } pqn_precision;
/* PQN_BI_REC: recursive Bi-PQN over three fidelities (the generalisation sketched in
 * Sec. 7): every Bi-PQN subproblem is solved by Bi-PQN one fidelity down, the lowest by
 * Mono-PQN. Needs both low-fidelity levels of the context. */
typedef enum { PQN_BBPGD = 0, PQN_MONO = 1, PQN_BI = 2, PQN_BI_REC = 3 } pqn_solver;
/* PQN_LOFI2: the second, coarsest low fidelity (n_theta_lo2 / gmres_tol_lo2). */
typedef enum { PQN_HIFI = 0, PQN_LOFI = 1, PQN_LOFI2 = 2 } pqn_fidelity;

/* Context description; copied by pqn_create. Zero fields take the defaults
 * given in brackets. */
typedef struct {
  int32_t n_particles;      /* M spheres (> 0) */
  double radius;            /* sphere radius a [1] */
  double mu;                /* viscosity [1] */
  int32_t n_theta, n_phi;   /* high-fidelity grid: Gauss-Legendre x trapezoid; p = n_theta - 1 */
  int32_t n_theta_lo, n_phi_lo; /* low-fidelity grid; 0 = none (Bi-PQN then unavailable) */
  double gmres_tol;         /* relative residual of each high-fidelity BIE solve [1e-8] */
  double gmres_tol_lo;      /* same, low fidelity [1e-8] */
  int32_t gmres_restart;    /* Krylov restart length [50] */
  int32_t gmres_max_iter;   /* iteration cap per solve [500] */
  double near_gap;          /* sphere pairs with gap < near_gap use the near rule [0.5 a] */
  int32_t near_up;          /* upsampling factor of the near rule [2] */
  double slip_speed;        /* Janus slip magnitude s [1] */
  int32_t precision;        /* pqn_precision of the far-field pair sums [PQN_FP64] */
  int32_t refine_sweeps;    /* mixed precision: outer refinement sweeps with an FP64 residual [0];
                               a system still above tolerance after them gets one FP64 correction
                               solve (counted in pqn_mvp_stats.fp64_fallback) */
  int32_t targets_per_thread; /* far FP32 kernel: 1 or 2 targets per thread, 256 threads per block [2] */
  int32_t far_chunks;       /* far kernels: source-sphere chunks (grid y); 0 = automatic */
  int32_t far_split;        /* far FP32 kernel: 1 = 64 targets per block, its four waves split each
                               chunk's sources and add their sums in LDS (targets_per_thread ignored) */
  int32_t device;           /* HIP device ordinal [0] */
  void* stream;             /* hipStream_t to run on; NULL = the library creates one */
  int32_t profile;          /* 1 = time every far pair-sum launch (and the other operator stages) with
                               HIP events; work then stays on one stream (side_stream ignored) */
  int32_t use_graphs;       /* 1 = replay each GMRES iteration of a single linear system from a
                               captured hipGraph (one per Arnoldi index; ignored when profile = 1) */
  int32_t warm_start;       /* 1 = the slip-driven solve (U_nc, also inside pqn_step) starts GMRES
                               from the previous slip solve's density instead of 0 */
  int32_t n_theta_lo2, n_phi_lo2; /* second low-fidelity grid (PQN_LOFI2); 0 = none (PQN_BI_REC
                               then unavailable). Needs the first low-fidelity grid. */
  double gmres_tol_lo2;     /* relative residual of each PQN_LOFI2 solve [1e-8] */
  /* Device memory provider (e.g. the PyTorch caching allocator), both or neither; NULL =
   * hipMalloc / hipFree. Every device buffer of the context is obtained through dev_alloc
   * (bytes, alloc_user), at create and when a call needs larger buffers, and returned
   * through dev_free(ptr, alloc_user) after the context's stream has been synchronised
   * (or at pqn_destroy). Blocks must be usable on the context's stream; dev_alloc returns
   * NULL on failure (the call then fails with PQN_ERR_OOM). The callbacks are invoked on
   * the calling thread during calls on this context only. */
  void* (*dev_alloc)(size_t bytes, void* user);
  void (*dev_free)(void* ptr, void* user);
  void* alloc_user;
  int32_t side_stream;      /* 1 = the coefficient / self-interaction GEMMs, near tiles and rigid
                               moments of an operator application run on a second stream of the
                               library, concurrently with the far pair sum (same results) */
  double near_close_gap;    /* near pairs with gap < near_close_gap use the finer factor
                               near_close_up [0 = none]: a gap the near_up grid does not resolve
                               can make the pair's discrete mobility, and the contact LCP
                               matrix, indefinite */
  int32_t near_close_up;    /* upsampling factor of those close pairs [3] */
  int32_t far_coarse_lo;    /* first low fidelity: far sphere pairs summed from a coarse source grid of
                               far_coarse_lo x 2 far_coarse_lo nodes carrying the density truncated to
                               degree far_coarse_lo - 1 (its multipoles to that degree); self and near
                               terms keep the level's grid. Sec. 5.1 lowers the order of the surface
                               representation for its low fidelity; with n_theta_lo = n_theta this lowers
                               it for the far field only. 0 = the node rule; else 2..n_theta_lo */
  int32_t far_coarse_lo2;   /* the same for the second low fidelity (2..n_theta_lo2) */
  int32_t precond;          /* right-preconditioned GMRES (Sec. 2 calls for preconditioned Krylov
                               solves without fixing one): for sphere i with near partners j,
                               (P v)_i = inv(S_i) (v_i - sum_j A_ij inv(D) v_j),
                               S_i = D - sum_j A_ij inv(D) A_ji, D the single-sphere block and A_ij
                               the near blocks. The near blocks act through the L = n_theta^2
                               harmonic coefficients of a density, so inv(S_i) is inv(D) plus a
                               rank-3L term; applied as inv(D) v (FP64) plus one block-sparse
                               product with 3n x 3L blocks in FP16 (each scaled by its largest
                               magnitude). Same solution and stopping rule (true residual), fewer
                               iterations. The set-up (pqn_mvp_stats.t_precond_ms) is per
                               configuration and fidelity: 1 = built when a configuration is solved
                               a second time (its first solve is plain), 2 = built at the first
                               solve; 0 = plain GMRES. Device memory about (2 n_near + 3 M) 3n 3L
                               + (n_near + 4 M) (3L)^2 doubles during the set-up, (M + n_near) 3n 3L FP16
                               values after it. In a batch context each suspension has its own (built at
                               the same points; its GMRES iterations then run eagerly, not from
                               captured graphs) [0] */
  int32_t precond_coarse;   /* with precond: 1 = two levels. A coarse correction on every sphere's
                               harmonics of degree <= 2 (27 unknowns per sphere) is applied before
                               the near-patch preconditioner P_f: z1 = Z inv(E) R v,
                               z = z1 + P_f (v - A~ z1), E = R A~ Z, R the projection on those
                               harmonics, Z their synthesis, A~ the operator with its far pairs
                               summed on coarse source grids (6 x 12 nodes for
                               far pairs whose centres are closer than 3.5
                               radii, 3 x 6 for the others):
                               the far field's smooth low modes, which the near patches cannot
                               reach, are solved for directly. Built with the rest of the
                               preconditioner; inv(E) by Newton-Schulz, stored in FP32 (about
                               4 (27 M)^2 doubles kept, whose Newton-Schulz GEMMs cost about
                               14 (27 M)^3 flop from the block diagonal's inverse, fewer from the
                               previous configuration's inverse, the start where it is close, as
                               after a time step; n_theta >= 3, at most 512 nodes per
                               sphere, at most 1024 spheres). Not for batch contexts
                               (PQN_ERR_INVALID) [0] */
} pqn_config_desc;

typedef struct {
  int32_t gmres_iters;      /* Krylov iterations (all sweeps) */
  int32_t matvecs;          /* BIE operator applications */
  int32_t refine_sweeps;    /* FP64-residual refinement sweeps done */
  int32_t converged;        /* 1 if the last residual met the tolerance */
  double rel_residual;      /* final relative residual (GMRES estimate, or FP64 residual after refinement) */
  double t_total_ms;        /* wall time of the call */
  double t_far_ms;          /* summed far pair-sum kernel time (profile = 1) */
  int32_t n_far;            /* far pair-sum launches */
  int32_t graph_launches;   /* GMRES iterations replayed from captured graphs (use_graphs = 1) */
  int32_t fp64_fallback;    /* mixed precision with refine_sweeps > 0: systems whose FP64 residual was
                               still above tolerance after the sweeps and were finished by an FP64
                               correction solve */
  /* profile = 1: summed HIP-event times of the other operator stages (one stream) */
  double t_near_ms;         /* near tiles */
  double t_gemm_ms;         /* harmonic coefficients, self interaction and upsampling GEMMs */
  double t_local_ms;        /* packing, rigid moments and the final combination */
  double t_arnoldi_ms;      /* CGS2 dot products and vector updates of GMRES */
  double t_precond_ms;      /* precond = 1: wall time of preconditioner set-ups in this call */
  int32_t precond_fallback; /* precond = 1: spheres whose Schur complement inverse did not converge
                               in those set-ups (they use inv(D)) */
  int32_t precond_applies;  /* precond = 1: applications of the preconditioner (one per group of
                               densities per GMRES iteration, one per system per cycle end) */
  double t_precond_apply_ms; /* profile = 1: summed HIP-event time of those applications */
  double t_far_by_k_ms[6];  /* profile = 1: far pair-sum time of the launches with k + 1 densities
                               (single-suspension contexts; the lockstep solves' tail launches
                               have fewer densities than the call) */
  int32_t n_far_by_k[6];    /* those launches' counts */
  int32_t precond_coarse_steps; /* precond_coarse = 1: Newton-Schulz steps of the coarse inverse in
                                   the set-ups of this call */
  int32_t precond_coarse_warm;  /* those set-ups that started from the previous configuration's
                                   coarse inverse */
} pqn_mvp_stats;

typedef struct {
  int32_t k_max;            /* outer iteration cap [100] */
  int32_t k_max_inner;      /* Bi-PQN: low-fidelity products per subproblem / initial solve [50] */
  int32_t j_max;            /* semi-smooth Newton steps per prox (Alg. 3) [50] */
  double kkt_tol_abs;       /* ||min(x, Ax+b)||_2 tolerance, eq. (kkt-error) [1e-8] */
  double kkt_tol_rel;       /* relative change tolerance, eq. (kkt-error) [1e-8] */
  double ssn_tol;           /* semi-smooth Newton stop: step <= ssn_tol * max(1, |(a, a~)|) [1e-14] */
  int32_t printed_metric;   /* initial quasi-Newton metric of the Mono-PQN solves (Alg. 1, and Alg. 4's
                               subproblems): 0 = H0 = I for the first step, then B0 = sigma I with
                               sigma = p.Ap/p.p of that step (invariant to the units of A) [0];
                               1 = H0 = I throughout, Alg. 1 as printed */
  int32_t recycle;          /* 1 = every mobility solve of an LCP product starts GMRES from the best
                               combination of the earlier products' solutions of the same call (per
                               fidelity, at most 32 kept; the Krylov reuse Sec. 7 names as future
                               work): x0 = Q (W^T r) with W = A Q orthonormal, so the initial
                               residual costs no operator application. Same stopping rule as a cold
                               solve. Ignored in mixed precision with refine_sweeps > 0 [0] */
} pqn_lcp_opts;

typedef struct {
  int32_t iters;            /* outer iterations */
  int32_t mvp_hi;           /* high-fidelity LCP products A[.] (each one BIE solve) */
  int32_t mvp_lo;           /* low-fidelity LCP products (Bi-PQN) */
  double emvp;              /* mvp_hi + mvp_lo * t_lo/t_hi (E-MVPs, Sec. 6) */
  double lo_hi_cost_ratio;  /* measured t_lo/t_hi of this call */
  double kkt_abs;           /* final absolute KKT error */
  int32_t converged;
  int32_t ssn_steps;        /* semi-smooth Newton steps in total */
  double t_total_ms;
  int32_t gmres_iters;      /* Krylov iterations over all products */
  int32_t model_rejected;   /* Bi-PQN: 1 if a low-fidelity solve met non-positive curvature or no
                               descent and the solve finished as Mono-PQN on A */
  int32_t mvp_lo2;          /* PQN_BI_REC: products at the second low fidelity (each one BIE solve) */
  double lo2_hi_cost_ratio; /* measured t_lo2/t_hi of this call; emvp adds mvp_lo2 * this ratio */
  double kkt_rel;           /* relative change of the last two KKT errors (0 before two iterates) */
  int32_t nonpos_curvature; /* steps on A (the final phase of the solve) whose direction p had
                               p.Ap <= 0, i.e. A is not positive definite along p; the step then
                               takes eta = 1 and resets the quasi-Newton memory (Alg. 2 edge case).
                               Positive definiteness of A is the method's assumption (Sec. 3); a
                               near-contact pair below the surface grid's resolution can break it */
} pqn_lcp_stats;

typedef struct {
  int32_t n_contacts;       /* |A| of eq. (collisional-set) */
  int32_t n_active;         /* contacts with x > 0 */
  pqn_lcp_stats lcp;
  int32_t gmres_iters_nc;   /* Krylov iterations of the U_nc solve */
  double t_total_ms;
  /* wall time of each stage of the step (the stream is synchronised between stages) */
  double t_contacts_ms;     /* contact search, eq. (collisional-set) */
  double t_nc_ms;           /* slip-driven solve U_nc */
  double t_lcp_ms;          /* b = Phi/dt + D^T U_nc and the LCP solve */
  double t_update_ms;       /* Euler update of centres and axes, new pair classes and near lists */
} pqn_step_stats;

/* Create a context for M spheres (centers [M][3], janus_axes [M][3] unit vectors;
 * axes may be NULL = no slip). Builds the grids, the singular self blocks (FP64,
 * host) and allocates device memory. Set-up, not an operation of the paper: the
 * suspension's configuration (Sec. 3) and its discretisation (Sec. 5.1). */
pqn_status pqn_create(const pqn_config_desc* desc, const double* centers, const double* janus_axes, pqn_ctx** out);
pqn_status pqn_destroy(pqn_ctx* ctx);

/* Replace / read the configuration (sphere centres and Janus axes, [M][3]). */
pqn_status pqn_set_state(pqn_ctx* ctx, const double* centers, const double* janus_axes);
pqn_status pqn_get_state(const pqn_ctx* ctx, double* centers, double* janus_axes);
/* Far pair-sum precision (pqn_precision) for subsequent calls. */
pqn_status pqn_set_precision(pqn_ctx* ctx, int32_t precision);

/* U = M F (Sec. 2, eq. (mobility); Fig. 1): FT, UO [M][6] host arrays (row i = F_i, T_i
 * resp. U_i, Omega_i). Non-finite FT: PQN_ERR_NUMERIC. */
pqn_status pqn_mobility_apply(pqn_ctx* ctx, const double* FT, double* UO, int32_t fidelity, pqn_mvp_stats* stats);
/* Same with FT_dev, UO_dev [M][6] in device memory of the context's device (caller-owned);
 * returns when UO_dev is written. */
pqn_status pqn_mobility_apply_dev(pqn_ctx* ctx, const double* FT_dev, double* UO_dev, int32_t fidelity,
                                  pqn_mvp_stats* stats);
/* K <= 6 force sets at once: FT, UO [K][M][6] host arrays. The K boundary-integral solves
 * run in lockstep and share every geometry pass of the pair sums (multi-right-hand-side). */
pqn_status pqn_mobility_apply_multi(pqn_ctx* ctx, int32_t k_rhs, const double* FT, double* UO, int32_t fidelity,
                                    pqn_mvp_stats* stats);
/* Same with FT_dev, UO_dev [K][M][6] in device memory (caller-owned); returns when UO_dev is
 * written. A non-finite force set makes the right-hand-side norm non-finite: PQN_ERR_NUMERIC. */
pqn_status pqn_mobility_apply_multi_dev(pqn_ctx* ctx, int32_t k_rhs, const double* FT_dev, double* UO_dev,
                                        int32_t fidelity, pqn_mvp_stats* stats);
/* Slip-driven rigid velocities U_nc (F = T = 0), UO [M][6]. */
pqn_status pqn_nc_velocity(pqn_ctx* ctx, double* UO, int32_t fidelity, pqn_mvp_stats* stats);

/* Candidate contacts (eq. (collisional-set)): pairs i < j with gap |c_i - c_j| - 2a <= delta,
 * lexicographic order. pairs [cap][2], gaps [cap]. If more than cap pairs exist, returns
 * PQN_ERR_INVALID with *n_out set to the number needed. */
pqn_status pqn_find_contacts(pqn_ctx* ctx, double delta, int32_t cap, int32_t* n_out, int32_t* pairs, double* gaps);

/* pqn_find_contacts for callers that cannot allocate device memory during the call
 * (serving loops, harnesses that forbid allocation): same arguments, results and errors,
 * but the kernel's count and list are staged in a fixed device array of the library
 * (one per device, about 0.5 MB, held until the process ends) instead of context buffers;
 * no device memory is allocated or freed. At most 32768 contacts: a configuration with
 * more gives PQN_ERR_INVALID with *n_out set to the count. Every call on one device
 * shares that device's array: calls that overlap on one device (several host threads,
 * or contexts on different streams) race and must be serialised by the caller. */
pqn_status pqn_find_contacts_noalloc(pqn_ctx* ctx, double delta, int32_t cap, int32_t* n_out, int32_t* pairs,
                                     double* gaps);

/* One LCP product Ax = D^T M D x (eq. (defAandb)); pairs [n][2] (i, j), x, Ax [n]. */
pqn_status pqn_lcp_apply(pqn_ctx* ctx, int32_t n, const int32_t* pairs, const double* x, double* Ax, int32_t fidelity);

/* Solve 0 <= A x + b perp x >= 0 (eq. (LCP)). x: on entry the initial guess x^(-1) of
 * Alg. 1/4 (negative entries are projected to 0; all zeros = no guess, no extra product;
 * a nonzero guess costs one product to evaluate A x^(-1), or A^ x^(-1) for Bi-PQN, whose
 * initial low-fidelity solve starts there), on exit the solution. opts may be NULL (defaults). PQN_BI needs the context's
 * low-fidelity grid, PQN_BI_REC both low-fidelity grids (else PQN_ERR_STATE); for
 * PQN_BI_REC, k_max_inner bounds the outer steps of the middle level and the products
 * of each lowest-level solve. */
pqn_status pqn_lcp_solve(pqn_ctx* ctx, int32_t n, const int32_t* pairs, const double* b, double* x, int32_t solver,
                         const pqn_lcp_opts* opts, pqn_lcp_stats* stats);

/* pqn_lcp_solve with pairs [n][2], b [n] and x [n] in device memory (x: guess in,
 * solution out, as above). Runs on the context's stream and returns after the solve
 * (the PQN iterations read a few flags back per product); invalid pairs or non-finite
 * b / x give PQN_ERR_INVALID with x unchanged. */
pqn_status pqn_lcp_solve_dev(pqn_ctx* ctx, int32_t n, const int32_t* pairs_dev, const double* b_dev, double* x_dev,
                             int32_t solver, const pqn_lcp_opts* opts, pqn_lcp_stats* stats);

/* One step (eq. (dvi)): contacts(delta) -> U_nc -> b = Phi/dt + D^T U_nc -> LCP ->
 * U = U_nc + M D x -> centres += dt U, Janus axes rotated by Omega dt. An LCP that
 * hits its cap after meeting p.Ap <= 0 (A not positive definite) gives
 * PQN_ERR_INDEFINITE and leaves the configuration unchanged; any other cap gives
 * PQN_WARN_NOT_CONVERGED and the step is taken with the last iterate. A moved
 * configuration the context cannot hold (a sphere with more than 16 near partners:
 * PQN_ERR_INVALID; a non-finite centre: PQN_ERR_NUMERIC) is rejected and the context
 * keeps the configuration it had before the step. pqn_set_state rejects such a
 * configuration in the same way. */
pqn_status pqn_step(pqn_ctx* ctx, double dt, double delta, int32_t solver, const pqn_lcp_opts* opts,
                    pqn_step_stats* stats);

/* Batched independent suspensions of uneven size (one descriptor and one [M_b][3]
 * centre array per suspension; janus_axes may be NULL). Not an operation of the paper:
 * many instances of its mobility product (Sec. 2, eq. (mobility)) solved together. The
 * suspensions must share precision, restart length, refinement, device and
 * targets_per_thread; the first descriptor's stream and use_graphs are used for all
 * (use_graphs = 1: the first GMRES cycle of all suspensions is replayed from captured
 * graphs, one per Arnoldi index, with the Givens rotations and end tests on the device).
 * The returned context accepts only the pqn_batch_* calls and pqn_destroy. */
pqn_status pqn_batch_create(int32_t n_inst, const pqn_config_desc* descs, const double* const* centers,
                            const double* const* janus_axes, pqn_ctx** out);
/* One mobility product per suspension (FT[b], UO[b]: [M_b][6] host arrays), all GMRES
 * iterations in lockstep, every far pair sum of an iteration in one launch ordered by
 * decreasing cost. stats (may be NULL): aggregate over the suspensions; per_inst (may be
 * NULL): [n_inst] statistics of each suspension (gmres_iters and matvecs of its own
 * solve, converged, rel_residual; timings only in stats). */
pqn_status pqn_batch_mobility_apply(pqn_ctx* ctx, const double* const* FT, double* const* UO, pqn_mvp_stats* stats,
                                    pqn_mvp_stats* per_inst);
/* Same with FT_dev[b], UO_dev[b] device arrays [M_b][6] of the context's device (the
 * pointer arrays themselves on the host); returns when every UO_dev[b] is written. A
 * non-finite force makes that suspension's right-hand-side norm non-finite:
 * PQN_ERR_NUMERIC. */
pqn_status pqn_batch_mobility_apply_dev(pqn_ctx* ctx, const double* const* FT_dev, double* const* UO_dev,
                                        pqn_mvp_stats* stats, pqn_mvp_stats* per_inst);

/* Operator-level entry points (stage-by-stage checks of the discrete BIE).
 * pqn_bie_apply: y = (1/2 I + D + P) q for q, y [3][N] host arrays.
 * pqn_get_self_block: S [3n][3n] rows (c*n+i), columns (d*n+k).
 * pqn_get_grid: node offsets [n][3] and weights [n] of one sphere. */
pqn_status pqn_bie_apply(pqn_ctx* ctx, int32_t fidelity, const double* q, double* y);
/* pqn_bie_apply_multi: the same for k <= 6 densities in one pass (q, y [k][3][N] host
 * arrays): the k applications share every geometry pass of the pair sums, through the
 * kernels and launch layout of the context's k-density mobility products. */
pqn_status pqn_bie_apply_multi(pqn_ctx* ctx, int32_t fidelity, int32_t k, const double* q, double* y);
pqn_status pqn_get_self_block(pqn_ctx* ctx, int32_t fidelity, double* S);
/* pqn_bie_solve: q solving (1/2 I + D + P) q = rhs by GMRES (plus refinement in mixed
 * precision), rhs, q [3][N] host arrays. */
pqn_status pqn_bie_solve(pqn_ctx* ctx, int32_t fidelity, const double* rhs, double* q, pqn_mvp_stats* stats);
pqn_status pqn_get_grid(pqn_ctx* ctx, int32_t fidelity, int32_t* n_nodes, double* offsets, double* weights);

/* Host-only (no device needed): the grid and singular self block of one sphere as
 * pqn_create builds them. offsets [n][3], weights [n], S [3n][3n] (any may be NULL),
 * n = n_theta * n_phi. */
pqn_status pqn_host_self_block(int32_t n_theta, int32_t n_phi, double radius, double* offsets, double* weights,
                               double* S);

/* Host-only (no device needed): the single-sphere block D = 1/2 I + S + P_rigid (self
 * interaction and rigid projection of one sphere, the diagonal block of the discrete
 * operator) and its inverse, as the precond = 1 set-up builds them. D, Dinv [3n][3n]
 * row-major in the SoA order of one sphere (row c n + node); either may be NULL.
 * PQN_ERR_NUMERIC if D is singular. */
pqn_status pqn_host_sphere_block(int32_t n_theta, int32_t n_phi, double radius, double* D, double* Dinv);

const char* pqn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BIPQN_H */
