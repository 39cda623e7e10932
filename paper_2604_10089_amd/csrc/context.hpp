// Library context: device tables and buffers of both fidelity levels, the BIE
// operator on groups of densities, lockstep GMRES and the mobility product.
#pragma once
#include <chrono>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <utility>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/bipqn.h"
#include "kernels.hpp"

namespace bipqn {

struct Error : std::runtime_error {
  pqn_status code;
  Error(pqn_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(x)                                                                                   \
  do {                                                                                              \
    hipError_t e_ = (x);                                                                            \
    if (e_ != hipSuccess)                                                                           \
      throw ::bipqn::Error(e_ == hipErrorOutOfMemory ? PQN_ERR_OOM : PQN_ERR_DEVICE,                \
                           std::string(#x) + ": " + hipGetErrorString(e_));                          \
  } while (0)

// Device memory provider of a context (pqn_config_desc.dev_alloc / dev_free);
// null functions = hipMalloc / hipFree. `stream` is the context's stream: a
// buffer replaced by a larger one is returned only after it has drained.
struct DevAllocator {
  void* (*alloc)(size_t, void*) = nullptr;
  void (*free)(void*, void*) = nullptr;
  void* user = nullptr;
  hipStream_t stream = nullptr;
};

// Provider used by DevArray::alloc on this thread: set for the duration of each
// call on a context (AllocScope), null outside calls.
inline thread_local const DevAllocator* g_dev_allocator = nullptr;

struct AllocScope {
  const DevAllocator* prev;
  explicit AllocScope(const DevAllocator* a) : prev(g_dev_allocator) { g_dev_allocator = a; }
  ~AllocScope() { g_dev_allocator = prev; }
  AllocScope(const AllocScope&) = delete;
  AllocScope& operator=(const AllocScope&) = delete;
};

template <class T>
struct DevArray {
  T* p = nullptr;
  size_t count = 0;
  DevAllocator al{};  // provider that returned p
  DevArray() = default;
  DevArray(const DevArray&) = delete;
  DevArray& operator=(const DevArray&) = delete;
  ~DevArray() { release(); }
  // (the owner has synchronised the stream: pqn_destroy does before deleting a context)
  void release() {
    if (p) {
      if (al.free)
        al.free(p, al.user);
      else
        (void)hipFree(p);
    }
    p = nullptr;
    count = 0;
  }
  void alloc(size_t n) {
    if (n <= count && p) return;
    if (p && al.free) HIPCHK(hipStreamSynchronize(al.stream));  // kernels may still read the old block
    release();
    if (n == 0) return;
    const DevAllocator* cur = g_dev_allocator;
    if (cur && cur->alloc) {
      al = *cur;
      p = static_cast<T*>(al.alloc(n * sizeof(T), al.user));
      if (!p) throw Error(PQN_ERR_OOM, "dev_alloc returned NULL");
    } else {
      al = DevAllocator{};
      HIPCHK(hipMalloc((void**)&p, n * sizeof(T)));
    }
    count = n;
  }
  void upload(const T* h, size_t n, hipStream_t s) {
    alloc(n);
    if (n) HIPCHK(hipMemcpyAsync(p, h, n * sizeof(T), hipMemcpyHostToDevice, s));
  }
};

// Named range on the calling thread's roctx stack (seen by rocprofv3 --marker-trace;
// a push and a pop when no tool is attached).
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

struct Timer {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
};

// Work buffers of one density (one right-hand side) on one level.
// Far FP32 launch layout from the configuration: 0 = split (64 targets per
// block, four waves share the sources), 1 or 2 = targets per thread.
inline int far_layout(const pqn_config_desc& c) {
  if (c.far_split) return 0;
  return c.targets_per_thread == 1 ? 1 : 2;
}

struct Work {
  DevArray<double> far_part, near_part, coef, qup, selfo, mom;
  DevArray<double> qup2;  // densities on the close-pair grid, same interleaving as qup
  DevArray<double> qc;    // degree-truncated densities on the coarse far-source grid [M][nc][3K]
};

// Krylov storage of one linear system on one level.
struct SysBuf {
  DevArray<double> V, x, r, rhs, tmp, d, partial, ycoef, rcoef;
  DevArray<double> z;  // preconditioned Arnoldi vector (config precond)
};

// Right preconditioner of the level's GMRES (config precond; precond.hip): the
// single-sphere block D, its inverse, the near blocks A_ij, the Schur complements
// S_i = D - sum_j A_ij D^{-1} A_ji and their inverses, rebuilt at the first solve
// after a configuration change.
// Coarse level of the two-level preconditioner (precond_coarse): per sphere and component
// the real harmonics of degree <= 2 (kCoarseB = 27 unknowns per sphere, Mc = 27 M).
constexpr int kCoarseL = 9, kCoarseB = 27;
struct CoarsePc {
  bool tab = false;                // the level's tables below are built
  bool on = false;                 // the current configuration applies the coarse correction
  int ncs = 0;                     // coarse far-source nodes per sphere (both grids)
  int ncs1 = 0;                    // ... of the close pairs' grid (the first ncs1)
  int ns_iters = 0;                // Newton-Schulz steps of inv(E) in the last set-up
  bool have_x = false;             // X holds the last configuration's inverse (the next start)
  long x_mc = 0;                   // ... of that size
  bool warm = false;               // the last set-up started from it
  double ns_res = 0.0;             // its final residual ||I - E X||_F / sqrt(Mc)
  DevArray<double> R;              // [27][3n] row-major: the projection (rows c 9 + k)
  DevArray<double> Z;              // [3n][27] row-major: the synthesis at the nodes
  DevArray<double> DZ;             // [27][3n] by columns: D Z (the diagonal blocks of A~ Z)
  DevArray<double> Tlow;           // [9][n]: rows k < 9 of the analysis T
  DevArray<double> offc, wc, Yc;   // coarse far-source grids [ncs][3], [ncs], synthesis [ncs][9]
  DevArray<unsigned char> t1, t2;  // [M][M]: 0 for the far pairs on the close / the distant grid
  DevArray<double> X0, ES;         // inv(R D Z) and R D Z, [27][27] by columns
  DevArray<double> NL;             // near low columns per ordered slot [27][3n] by columns
  DevArray<_Float16> B16;          // D Z and the NL blocks in FP16 (by columns, ld rows)
  DevArray<float> bscale;
  DevArray<int> bptr, bcol;
  int nblk = 0, ld = 0;
  DevArray<double> E, X, X2, W;    // [Mc][Mc] by columns
  DevArray<double> res;
  DevArray<float> Ei;              // inv(E) in FP32 by columns
  DevArray<double> cr, cpart, ccI, ccC, qc, bpart;  // application work arrays
  DevArray<double> src;            // packed coarse far sources [M][ncs] (records of either precision)
  DevArray<GemmDesc> desc;         // R v and the Z c accumulation for K = 1 .. kMaxRhs (2 per K)
  int tr[kMaxRhs] = {}, tz[kMaxRhs] = {};
};

struct Precond {
  bool has_d = false;            // D^{-1}, TD and the application's GEMM descriptors are built
  unsigned long epoch = 0;       // configuration of the tables below (0 = none yet)
  unsigned long seen = 0;        // configuration last solved without them (precond = 1)
  bool use = false;              // the current solve (solve_lockstep) applies them
  DevArray<double> Dinv;         // [3n][3n] row-major
  DevArray<double> DinvT;        // D^{-1} by columns ([3n][3n] row-major of its transpose)
  DevArray<double> TT;           // the analysis T by columns [n][L]
  DevArray<double> TD;           // (I3 x T) D^{-1} [3L][3n] row-major
  DevArray<double> Ac, Gc;       // near blocks on coefficients / S_i^{-1} Ac: per slot [3L][3n] by columns, at aco[i]
  DevArray<double> Rr;           // TD Ac of the reverse slots: sphere i [npart_i 3L][3L] by columns, at rro[i]
  std::vector<long> aco, rro;
  DevArray<double> Q, Z, E;      // [M] x 3n x 3L by columns: Q_i, D^{-1} Q_i, E_i
  DevArray<double> Kc, Y, Y2, W; // [M] x 3L x 3L by columns: I - TD Q_i, its inverse (Newton-Schulz)
  DevArray<double> res;          // Newton-Schulz residuals, partial sums [M][slices]
  DevArray<_Float16> B16;        // the E_i and -Gc blocks in FP16, by columns, row of sphere i
  DevArray<float> bscale;        // each block's largest magnitude (its FP16 copy is divided by it)
  DevArray<int> bptr, bcol;      // first block of sphere i's row [M + 1]; column sphere of each block
  DevArray<double> vC;           // input densities by (density, sphere) columns [K][M][3n]
  DevArray<double> wI, yI;       // TD v [M][3L][K] and D^{-1} v [M][3n][K]
  DevArray<double> part;         // per-block partial products [nblk][K][3n]
  DevArray<GemmDesc> adesc;      // y and w GEMMs for K = 1 .. kMaxRhs (2 per K)
  std::vector<GemmDesc> adesc_h; // host copy (the batch path concatenates the K = 1 pairs)
  int aty[kMaxRhs] = {}, atw[kMaxRhs] = {};  // 64x64 tiles of those GEMMs
  int nblk = 0;                  // blocks: the spheres with near partners + the ordered near pairs
  int ld = 0;                    // padded column length of the FP16 blocks (multiple of 64)
  int fallback = 0;              // spheres left on D^{-1} (Newton-Schulz did not converge)
  int ns_iters = 0;              // Newton-Schulz steps of the last set-up
  double setup_ms = 0.0;         // wall time of the last set-up
  CoarsePc co;                   // the coarse level (precond_coarse)
};

// Reuse of earlier solutions across the mobility products of one LCP solve (the
// Krylov reuse Sec. 7 names as future work): densities Q of earlier solves and
// their operator images W = A Q, kept with W orthonormal. A new right-hand side r
// starts GMRES from x0 = Q (W^T r), whose residual r - W (W^T r) is known without
// an operator application. Active only inside pqn_lcp_solve / pqn_step calls that
// ask for it.
struct Recycle {
  DevArray<double> Q, W;  // [kmax][3N] each
  DevArray<double> c;     // coefficients W^T r [kmax]
  DevArray<double> nrm;   // squared norms of a new image before / after projection
  int k = 0, kmax = 0;
  bool active = false;
  unsigned long epoch = 0;  // configuration the stored pairs belong to
};

// Host staging of typed descriptor arrays, uploaded in one copy.
struct DescPack {
  std::vector<char> host;
  template <class T>
  size_t add(const std::vector<T>& v) {
    const size_t off = (host.size() + 63) & ~size_t(63);
    host.resize(off + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(host.data() + off, v.data(), v.size() * sizeof(T));
    return off;
  }
};

// Offsets (in a DescPack) and sizes of the segment tables of one batched operator
// application: descriptor counts (n*) and launch extents (blocks or elements).
struct BatchOpTables {
  size_t oa = 0, ob = 0, op = 0, on = 0, om = 0, oc = 0, of = 0;
  int na = 0, nga = 0, nb = 0, ngb = 0, npk_n = 0, npk = 0, nnd_n = 0, nnd = 0, nmd_n = 0, nmd = 0, ncd_n = 0,
      ncd = 0, nfd = 0, nfar = 0;
};

// Offsets and sizes of the segmented GEMM descriptor tables of one iteration.
struct IterTables {
  size_t oa = 0, ob = 0;
  int na = 0, nga = 0, nb = 0, ngb = 0;
};

// Captured GMRES iterations of one linear system (one graph per Arnoldi index k).
struct GraphCache {
  int prec = -1;
  unsigned long epoch = 0;
  const double* hp = nullptr;   // Hessenberg staging the graphs write to
  const double* qup = nullptr;  // upsampled-density buffers the graphs read
  const double* qup2 = nullptr;
  std::vector<hipGraphExec_t> execs;
  DevArray<char> dtab;  // per-k descriptor tables read by the captured kernels
  size_t stride = 0;
  void clear() {
    for (hipGraphExec_t& e : execs)
      if (e) (void)hipGraphExecDestroy(e);
    execs.clear();
  }
  ~GraphCache() { clear(); }
};

// Captured GMRES iterations of a batch of systems (one graph per Arnoldi index, all
// systems in lockstep; device-side Givens rotations and end tests, so a system that
// ends turns its segments of the later launches into no-ops).
struct BatchGraph {
  int m = 0, ns = 0, prec = -1;
  std::vector<const void*> key;  // (context, level, slot) of every system, in order
  DevArray<GmSys> sys;
  DevArray<double> hess, hbuf;
  DevArray<char> tabs;  // descriptor tables of every Arnoldi index (stride apart)
  size_t stride = 0;
  std::vector<hipGraphExec_t> execs;
  void clear() {
    for (hipGraphExec_t& e : execs)
      if (e) (void)hipGraphExecDestroy(e);
    execs.clear();
  }
  ~BatchGraph() { clear(); }
};

struct Level {
  SphereTables tab;
  int M = 0, n = 0, N = 0, L = 0, nup = 0, p = 0;
  DevArray<double> off, w, G, T, Yup, shab;
  DevArray<double4> offup;
  int nup2 = 0;  // close-pair grid (0 = none)
  DevArray<double> Yup2;
  DevArray<double4> offup2;
  int nc = 0, Lc = 0;  // coarse far-source grid (0 = far pairs by the node rule) and its truncation
  DevArray<double> offc, wc, Yc;
  DevArray<double> src;  // packed far sources, up to kMaxRhs densities (FP64 record is the larger)
  int nchunks = 1, spc = 1, tpt = 2;
  int restart = 50, max_iter = 500;
  double tol = 1e-8;
  int nb_dots = 128;
  std::vector<std::unique_ptr<Work>> work;
  std::vector<std::unique_ptr<SysBuf>> sys;
  std::vector<std::unique_ptr<GraphCache>> graphs;
  DevArray<double> q_nc;  // density of the last slip-driven solve (warm start of the next one)
  bool has_q_nc = false;
  Recycle rc;
  Precond pc;
  Work& wk(int k);
  SysBuf& sb(int k);
};

struct LcpState;
void lcp_release(LcpState* st);
struct pqn_ctx_impl;

// A group of K densities on one level of one context: K operator applications
// that share the geometry pass of the pair sums.
// All densities of one (context, level) form one group: the level's packed
// source buffer and the group's interleaved upsampled density are shared by
// the group, so a second group on the same level would overwrite them.
struct MvGroup {
  pqn_ctx_impl* c;
  Level* lv;
  int K;
  int slot[kMaxRhs];  // work slot of density r
  const double* in[kMaxRhs];
  double* out[kMaxRhs];
};

// The single-sphere block D = 1/2 I + S + P_rigid ([3n][3n] row-major, local order c n + x)
// and the in-place inverse of a row-major n x n matrix (Gauss-Jordan, partial pivoting).
void single_sphere_block(const SphereTables& t, std::vector<double>& D);
void invert_gauss_jordan(std::vector<double>& A, int n);

// Add density (in -> out, work slot) to the group of its (context, level).
void add_to_groups(std::vector<MvGroup>& groups, pqn_ctx_impl* c, Level* lv, int slot, const double* in,
                   double* out);

// Work buffers of a group (grown on first use with more densities): the interleaved
// upsampled densities [M][nup][3K] and the harmonic coefficients [M][3K][L].
double* group_qup(MvGroup& gr, bool close = false);
double* group_coef(MvGroup& gr);
// One GEMM problem of a segmented launch (see kernels.hpp, GemmDesc); big = 1 counts
// 64x64 tiles (launch_gemm64_multi_big), else 32x32 (launch_gemm64_multi).
void push_gemm(std::vector<GemmDesc>& v, int& blocks, int R, int Cn, int K, const double* A, int lda,
               const double* B, int ldb, double* C, int rb, long rbs, int ldc, int rs = 1, int cb = 0, long cbs = 0,
               int at = 0, int big = 0);
// The coefficient GEMMs of a group (list ga) and its self-interaction (with_self) and
// upsampling GEMMs (list gb).
void push_group_gemms(Level& lv, int K, const int* slot, const double* const* in, double* coef, double* qup,
                      double* qup2, const int* live_flag, std::vector<GemmDesc>& ga, int& nga,
                      std::vector<GemmDesc>& gb, int& ngb, bool with_self = true);

// One linear system (1/2 + D + P) x = rhs in the lockstep GMRES engine.
struct SysRef {
  pqn_ctx_impl* c;
  Level* lv;
  int slot;
  const double* rhs;
  double* x;
  double tol;
  int its = 0;
  double relres = 0.0;
  bool conv = false;
  const double* x0 = nullptr;  // initial guess (device, [3][N]); nullptr = start from 0
  const double* r0 = nullptr;  // its residual rhs - A x0 when known (no operator application then)
  double* res_out = nullptr;   // receives the final residual vector rhs - A x (from the Arnoldi relation)
};

struct pqn_ctx_impl {
  pqn_config_desc cfg{};
  int M = 0;
  double a = 1.0, mu = 1.0;
  std::vector<double> centers, axes;
  bool has_axes = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  DevAllocator dev_alloc;  // device memory provider (every DevArray of the context)
  Level hi, lo, lo2;  // fidelities PQN_HIFI, PQN_LOFI, PQN_LOFI2
  bool has_lo = false, has_lo2 = false;
  // configuration-dependent tables shared by both levels
  DevArray<double> ctr, dax;
  DevArray<unsigned char> cls;
  DevArray<int> partners, npart, near_list;
  int max_slots = 0, n_near = 0;
  DevArray<int> near_list2;  // close near pairs (gap < near_close_gap), same format as near_list
  int n_near2 = 0;
  std::vector<int> h_partners, h_npart;
  DevArray<double> FT, UO;
  // lockstep GMRES scratch: per-system Hessenberg columns, read back in one copy
  DevArray<double> hdev;
  std::vector<double> hhost;
  DevArray<char> ddesc;  // segment descriptors of the multi-suspension kernels
  char* push_desc_pack(const std::vector<char>& pack);
  char* push_desc_pack(const std::vector<char>& pack, hipStream_t st, DevArray<char>& table);
  // second stream for work that overlaps the far pair sum (config side_stream)
  hipStream_t side = nullptr;
  hipEvent_t ev_in = nullptr, ev_side = nullptr;
  DevArray<char> ddesc_side;  // descriptor table of the side stream's segmented launches
  hipStream_t side_stream();
  void side_work(MvGroup& gr, hipStream_t st);
  // profiling of far launches
  // profile = 1: HIP events around every launch of each stage of the operator, on the
  // main stream (the side stream is not used while profiling)
  // kStageFarK + K - 1: the far launches of one group with K densities
  enum { kStageFar = 0, kStageNear, kStageGemm, kStageLocal, kStageArnoldi, kStagePrecond, kStageFarK,
         kNumStages = kStageFarK + kMaxRhs };
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool[kNumStages];
  size_t ev_used[kNumStages] = {};
  double stage_ms[kNumStages] = {};  // totals of the last end_far_timing()
  void stage_begin(int st);
  void stage_end(int st);
  int n_matvec = 0, n_far = 0;
  int n_far_k[kMaxRhs] = {};  // far launches of one group by its density count
  unsigned long config_epoch = 1;  // bumped by every configuration change (invalidates graphs)
  int n_graph_launch = 0;
  LcpState* lcp = nullptr;
  // batched suspensions: one child context per suspension, sharing the stream
  bool is_batch = false;
  std::vector<std::unique_ptr<pqn_ctx_impl>> children;
  ~pqn_ctx_impl();

  Level& level(int fidelity) {
    if (is_batch) throw Error(PQN_ERR_STATE, "this entry point takes a single-suspension context");
    if (fidelity == PQN_LOFI) {
      if (!has_lo) throw Error(PQN_ERR_STATE, "no low-fidelity grid in this context");
      return lo;
    }
    if (fidelity == PQN_LOFI2) {
      if (!has_lo2) throw Error(PQN_ERR_STATE, "no second low-fidelity grid in this context");
      return lo2;
    }
    if (fidelity != PQN_HIFI) throw Error(PQN_ERR_INVALID, "fidelity must be PQN_HIFI, PQN_LOFI or PQN_LOFI2");
    return hi;
  }
  void setup_level(Level& lv, int nt, int np, double tol, int far_theta = 0);
  void set_configuration(const double* c, const double* ax);
  // operator on groups of densities (all on this context's stream)
  void matvec_groups(std::vector<MvGroup>& groups, int precision);
  void matvec_batched(std::vector<MvGroup>& groups, int prec);
  BatchOpTables batch_op_tables(std::vector<MvGroup>& groups, int prec, const std::vector<const int*>& live,
                                DescPack& dp);
  void batch_op_launch(const char* base, const BatchOpTables& t, int prec);
  // one GMRES iteration of a single system (operator + CGS2), kernels only, for capture
  IterTables iteration_tables(pqn_ctx_impl& c, Level& lv, int slot, const double* q, std::vector<char>& bytes);
  void iteration_launches(pqn_ctx_impl& c, Level& lv, int slot, int prec, const double* q, double* w,
                          const double* V, int nvec, double* hp, int m, const char* dtab, const IterTables& t);
  void launch_iteration_graph(pqn_ctx_impl& c, Level& lv, int slot, int prec, int k, double* hp, int m);
  void apply_operator(Level& lv, int precision, const double* q, double* y);
  // lockstep GMRES over systems; every system's x is overwritten (initial guess 0)
  void gmres_lockstep(std::vector<SysRef>& sys, int precision);
  void gmres_lockstep_eager(std::vector<SysRef>& sys, int precision);
  // batch contexts with use_graphs: the first cycle of cold-started systems from captured graphs
  std::unique_ptr<BatchGraph> bgraph;
  void gmres_batch_graph(std::vector<SysRef>& sys, int precision);
  void capture_batch_iteration(BatchGraph& bg, std::vector<SysRef>& sys, int j, int prec);
  // solve in the context's precision with optional FP64-residual refinement
  // its_per (optional): Krylov iterations of each system, correction solves included
  void solve_lockstep(std::vector<SysRef>& sys, pqn_mvp_stats* st, std::vector<int>* its_per = nullptr);
  // mobility products of K force sets on one level (K <= kMaxRhs)
  void mobility_multi(Level& lv, int K, const double* const* FT_dev, const double* axes_dev,
                      double* const* UO_dev, pqn_mvp_stats* st);
  // Recycle: warm start of a single force-driven solve from the stored pairs, and the
  // addition of its solution (rhs in sb(0).rhs, solution in sb(0).x, final residual in res)
  void recycle_start(Level& lv, SysRef& sr);
  void recycle_add(Level& lv, const double* res);
  // right preconditioner (precond.hip): set-up of a level for the current configuration
  // (no-op when up to date), and out_r = P in_r for the densities of a group (out_r may
  // be in_r: every read of the input precedes the write of the output)
  void precond_setup(Level& lv);
  void coarse_tables(Level& lv);
  void coarse_setup(Level& lv);
  void coarse_pre(MvGroup& gr);
  void precond_apply(MvGroup& gr);
  void precond_apply_groups(std::vector<MvGroup>& groups);
  // near tiles only: near_part of the group's slots from its densities (with their
  // coefficient and upsampling GEMMs; from_coef: from the coefficients already in the
  // group's buffer), on the main stream
  void near_stage(MvGroup& gr, bool from_coef = false);
  double pc_setup_ms = 0.0;  // preconditioner set-up time, fallbacks and applications since the last reset
  int pc_fallback = 0;
  int pc_coarse_steps = 0, pc_coarse_warm = 0;
  int pc_applies = 0;
  int pc_prec = 0;  // 1: the current GMRES solve's operator is mixed (the coarse far sum in FP32)
  void mobility(Level& lv, const double* FT_dev, const double* axes_dev, double* UO_dev, pqn_mvp_stats* st) {
    mobility_multi(lv, 1, &FT_dev, axes_dev, &UO_dev, st);
  }
  double dot_host(const double* x, const double* y, long len, Level& lv);
  void begin_far_timing();
  void end_far_launch();
  double end_far_timing();
};

}  // namespace bipqn

struct pqn_ctx : bipqn::pqn_ctx_impl {};
