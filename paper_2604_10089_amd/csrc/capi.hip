// extern "C" entry points: argument checks, host/device copies, error mapping.
#include <algorithm>
#include <cstring>

#include "context.hpp"
#include "lcp.hpp"

using namespace bipqn;

static thread_local std::string g_last_error;

static pqn_status fail(pqn_status s, const std::string& m) {
  g_last_error = m;
  return s;
}

template <class F>
static pqn_status guarded(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    return fail(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(PQN_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(PQN_ERR_INVALID, e.what());
  }
}

static void fill_defaults(pqn_config_desc& c) {
  if (c.radius <= 0) c.radius = 1.0;
  if (c.mu <= 0) c.mu = 1.0;
  if (c.gmres_tol <= 0) c.gmres_tol = 1e-8;
  if (c.gmres_tol_lo <= 0) c.gmres_tol_lo = 1e-8;
  if (c.gmres_tol_lo2 <= 0) c.gmres_tol_lo2 = 1e-8;
  if (c.gmres_restart <= 0) c.gmres_restart = 50;
  if (c.gmres_max_iter <= 0) c.gmres_max_iter = 500;
  if (c.near_gap <= 0) c.near_gap = 0.5 * c.radius;
  if (c.near_up <= 0) c.near_up = 2;
  if (c.near_close_gap < 0) c.near_close_gap = 0;
  if (c.near_close_up <= 0) c.near_close_up = 3;
  if (c.slip_speed == 0) c.slip_speed = 1.0;
  if (c.targets_per_thread <= 0) c.targets_per_thread = 2;
}

static bool is_batch(const pqn_ctx* ctx) { return ctx && ctx->is_batch; }

// Stage times of the last call (profile = 1), after end_far_timing.
static void stage_stats(const pqn_ctx_impl& c, pqn_mvp_stats& st) {
  st.t_near_ms = c.stage_ms[pqn_ctx_impl::kStageNear];
  st.t_gemm_ms = c.stage_ms[pqn_ctx_impl::kStageGemm];
  st.t_local_ms = c.stage_ms[pqn_ctx_impl::kStageLocal];
  st.t_arnoldi_ms = c.stage_ms[pqn_ctx_impl::kStageArnoldi];
  st.t_precond_ms = c.pc_setup_ms;
  st.precond_fallback = c.pc_fallback;
  st.precond_coarse_steps = c.pc_coarse_steps;
  st.precond_coarse_warm = c.pc_coarse_warm;
  st.precond_applies = c.pc_applies;
  st.t_precond_apply_ms = c.stage_ms[pqn_ctx_impl::kStagePrecond];
  for (int k = 0; k < kMaxRhs; ++k) {
    st.t_far_by_k_ms[k] = c.stage_ms[pqn_ctx_impl::kStageFarK + k];
    st.n_far_by_k[k] = c.n_far_k[k];
  }
}

// nullptr if the context has the fidelities the (valid) solver needs, else the reason.
static const char* solver_unavailable(const pqn_ctx_impl& c, int solver) {
  if (solver == PQN_BI && !c.has_lo) return "Bi-PQN needs a low-fidelity grid";
  if (solver == PQN_BI_REC && !c.has_lo2) return "recursive Bi-PQN needs two low-fidelity grids";
  return nullptr;
}

extern "C" {

const char* pqn_last_error(void) { return g_last_error.c_str(); }

static std::string check_desc(const pqn_config_desc& c) {
  if (c.n_particles <= 0) return "n_particles must be > 0";
  if (c.n_theta < 2 || c.n_phi < 2 * c.n_theta - 1)
    return "high-fidelity grid needs n_theta >= 2 and n_phi >= 2 n_theta - 1";
  if (c.n_theta_lo != 0 && (c.n_theta_lo < 2 || c.n_phi_lo < 2 * c.n_theta_lo - 1))
    return "low-fidelity grid needs n_theta >= 2 and n_phi >= 2 n_theta - 1";
  if (c.n_theta_lo2 != 0 && (c.n_theta_lo2 < 2 || c.n_phi_lo2 < 2 * c.n_theta_lo2 - 1))
    return "second low-fidelity grid needs n_theta >= 2 and n_phi >= 2 n_theta - 1";
  if (c.n_theta_lo2 != 0 && c.n_theta_lo == 0) return "a second low-fidelity grid needs the first";
  if (c.precision != PQN_FP64 && c.precision != PQN_MIXED) return "bad precision";
  if ((c.dev_alloc == nullptr) != (c.dev_free == nullptr)) return "dev_alloc and dev_free go together";
  if (c.near_up > 8 || c.near_close_up > 8) return "near upsampling factors above 8 are not supported";
  if (c.far_coarse_lo != 0 && (c.n_theta_lo == 0 || c.far_coarse_lo < 2 || c.far_coarse_lo > c.n_theta_lo))
    return "far_coarse_lo needs a low-fidelity grid and 2 <= far_coarse_lo <= n_theta_lo";
  if (c.far_coarse_lo2 != 0 && (c.n_theta_lo2 == 0 || c.far_coarse_lo2 < 2 || c.far_coarse_lo2 > c.n_theta_lo2))
    return "far_coarse_lo2 needs a second low-fidelity grid and 2 <= far_coarse_lo2 <= n_theta_lo2";
  if (c.precond < 0 || c.precond > 2) return "precond must be 0, 1 or 2";
  if (c.precond_coarse < 0 || c.precond_coarse > 1) return "precond_coarse must be 0 or 1";
  if (c.precond_coarse && (c.n_theta < 3 || (long)c.n_theta * c.n_phi > 512 ||
                           (c.n_theta_lo != 0 && c.n_theta_lo < 3) || (c.n_theta_lo2 != 0 && c.n_theta_lo2 < 3)))
    return "precond_coarse needs n_theta >= 3 on every grid and at most 512 nodes per sphere";
  if (c.precond_coarse && c.n_particles > 1024)
    return "precond_coarse supports at most 1024 spheres (its coarse matrix has (27 M)^2 entries)";
  return "";
}

// Build one suspension's context on the given stream (nullptr: create one).
static std::unique_ptr<pqn_ctx_impl> make_context(const pqn_config_desc& c, const double* centers,
                                                  const double* janus_axes, hipStream_t stream) {
  std::unique_ptr<pqn_ctx_impl> ctx(new pqn_ctx_impl());
  ctx->cfg = c;
  ctx->M = c.n_particles;
  ctx->a = c.radius;
  ctx->mu = c.mu;
  ctx->device = c.device;
  if (stream) {
    ctx->stream = stream;
  } else {
    HIPCHK(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
    ctx->own_stream = true;
  }
  ctx->dev_alloc = DevAllocator{c.dev_alloc, c.dev_free, c.alloc_user, ctx->stream};
  AllocScope scope(&ctx->dev_alloc);
  ctx->setup_level(ctx->hi, c.n_theta, c.n_phi, c.gmres_tol);
  if (c.n_theta_lo > 0) {
    ctx->setup_level(ctx->lo, c.n_theta_lo, c.n_phi_lo, c.gmres_tol_lo, c.far_coarse_lo);
    ctx->has_lo = true;
  }
  if (c.n_theta_lo2 > 0) {
    ctx->setup_level(ctx->lo2, c.n_theta_lo2, c.n_phi_lo2, c.gmres_tol_lo2, c.far_coarse_lo2);
    ctx->has_lo2 = true;
  }
  ctx->FT.alloc(6 * (size_t)kMaxRhs * ctx->M);
  ctx->UO.alloc(6 * (size_t)kMaxRhs * ctx->M);
  ctx->set_configuration(centers, janus_axes);
  return ctx;
}

pqn_status pqn_create(const pqn_config_desc* desc, const double* centers, const double* janus_axes, pqn_ctx** out) {
  return guarded([&]() -> pqn_status {
    if (!desc || !centers || !out) return fail(PQN_ERR_INVALID, "pqn_create: NULL argument");
    *out = nullptr;
    pqn_config_desc c = *desc;
    fill_defaults(c);
    const std::string bad = check_desc(c);
    if (!bad.empty()) return fail(PQN_ERR_INVALID, bad);
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (c.device < 0 || c.device >= ndev) return fail(PQN_ERR_DEVICE, "no such HIP device");
    HIPCHK(hipSetDevice(c.device));
    contact_scratch_setup(c.device);  // device address of pqn_find_contacts_noalloc's staging
    std::unique_ptr<pqn_ctx_impl> ctx = make_context(c, centers, janus_axes, (hipStream_t)c.stream);
    *out = static_cast<pqn_ctx*>(ctx.release());
    return PQN_OK;
  });
}

pqn_status pqn_batch_create(int32_t n_inst, const pqn_config_desc* descs, const double* const* centers,
                            const double* const* janus_axes, pqn_ctx** out) {
  return guarded([&]() -> pqn_status {
    if (n_inst <= 0 || !descs || !centers || !out) return fail(PQN_ERR_INVALID, "pqn_batch_create: bad argument");
    *out = nullptr;
    pqn_config_desc c0 = descs[0];
    fill_defaults(c0);
    for (int b = 0; b < n_inst; ++b) {
      pqn_config_desc c = descs[b];
      fill_defaults(c);
      const std::string bad = check_desc(c);
      if (!bad.empty()) return fail(PQN_ERR_INVALID, "instance " + std::to_string(b) + ": " + bad);
      if (!centers[b]) return fail(PQN_ERR_INVALID, "pqn_batch_create: NULL centres");
      if (c.precond_coarse)
        return fail(PQN_ERR_INVALID, "instance " + std::to_string(b) + ": precond_coarse is not for batch contexts");
      if (c.precision != c0.precision || c.gmres_restart != c0.gmres_restart || c.device != c0.device ||
          c.targets_per_thread != c0.targets_per_thread || c.far_split != c0.far_split ||
          c.refine_sweeps != c0.refine_sweeps || c.dev_alloc != c0.dev_alloc || c.dev_free != c0.dev_free ||
          c.alloc_user != c0.alloc_user)
        return fail(PQN_ERR_INVALID,
                    "batched instances must share precision, restart, refinement, device, tiling and allocator");
    }
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (c0.device < 0 || c0.device >= ndev) return fail(PQN_ERR_DEVICE, "no such HIP device");
    HIPCHK(hipSetDevice(c0.device));
    std::unique_ptr<pqn_ctx_impl> parent(new pqn_ctx_impl());
    parent->cfg = c0;
    parent->device = c0.device;
    parent->is_batch = true;
    if (c0.stream) {
      parent->stream = (hipStream_t)c0.stream;
    } else {
      HIPCHK(hipStreamCreateWithFlags(&parent->stream, hipStreamNonBlocking));
      parent->own_stream = true;
    }
    parent->dev_alloc = DevAllocator{c0.dev_alloc, c0.dev_free, c0.alloc_user, parent->stream};
    AllocScope scope(&parent->dev_alloc);
    for (int b = 0; b < n_inst; ++b) {
      pqn_config_desc c = descs[b];
      fill_defaults(c);
      parent->children.push_back(make_context(c, centers[b], janus_axes ? janus_axes[b] : nullptr, parent->stream));
    }
    *out = static_cast<pqn_ctx*>(parent.release());
    return PQN_OK;
  });
}

// One mobility product per suspension of a batch context; FT / UO are host arrays
// (dev = false) or device arrays (dev = true) of [M_b][6] per suspension.
static pqn_status batch_apply_common(pqn_ctx* ctx, const double* const* FT, double* const* UO, bool dev,
                                     pqn_mvp_stats* stats, pqn_mvp_stats* per_inst) {
  Timer tm;
  const int nb = (int)ctx->children.size();
  for (int b = 0; b < nb; ++b) {
    if (!FT[b] || !UO[b]) return fail(PQN_ERR_INVALID, "pqn_batch_mobility_apply: NULL force/velocity array");
    if (!dev)
      for (int k = 0; k < 6 * ctx->children[b]->M; ++k)
        if (!std::isfinite(FT[b][k])) return fail(PQN_ERR_NUMERIC, "non-finite force/torque");
  }
  ctx->n_matvec = 0;
  ctx->n_graph_launch = 0;
  ctx->pc_setup_ms = 0.0;
  ctx->pc_fallback = 0;
  ctx->pc_coarse_steps = 0;
  ctx->pc_coarse_warm = 0;
  ctx->pc_applies = 0;
  ctx->n_far = 0;
  std::fill(ctx->n_far_k, ctx->n_far_k + kMaxRhs, 0);
  for (auto& ch : ctx->children) {
    ch->pc_setup_ms = 0.0;
    ch->pc_fallback = 0;
    ch->pc_coarse_steps = 0;
    ch->pc_coarse_warm = 0;
  }
  std::vector<SysRef> sys;
  for (int b = 0; b < nb; ++b) {
    pqn_ctx_impl& c = *ctx->children[b];
    const double* ft = FT[b];
    if (!dev) {
      HIPCHK(hipMemcpyAsync(c.FT.p, FT[b], 6 * (size_t)c.M * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
      ft = c.FT.p;
    }
    SysBuf& sb = c.hi.sb(0);
    launch_rhs(ctx->stream, c.ctr.p, ft, nullptr, c.hi.off.p, c.hi.n, c.M, c.hi.N, c.a, c.mu, c.cfg.slip_speed,
               sb.rhs.p);
    sys.push_back(SysRef{&c, &c.hi, 0, sb.rhs.p, sb.x.p, c.hi.tol});
  }
  pqn_mvp_stats st{};
  std::vector<int> its_per;
  ctx->solve_lockstep(sys, &st, &its_per);
  for (int b = 0; b < nb; ++b) {
    pqn_ctx_impl& c = *ctx->children[b];
    Work& w = c.hi.wk(0);
    double* uo = dev ? UO[b] : c.UO.p;
    launch_moments(ctx->stream, c.hi.sb(0).x.p, c.hi.off.p, c.hi.w.p, c.hi.n, c.M, c.hi.N, w.mom.p);
    launch_rigid_velocity(ctx->stream, w.mom.p, c.M, c.a, uo);
    if (!dev)
      HIPCHK(hipMemcpyAsync(UO[b], c.UO.p, 6 * (size_t)c.M * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  st.t_far_ms = ctx->end_far_timing();
  stage_stats(*ctx, st);
  for (auto& ch : ctx->children) {  // the suspensions' preconditioner set-ups
    st.t_precond_ms += ch->pc_setup_ms;
    st.precond_fallback += ch->pc_fallback;
    st.precond_coarse_steps += ch->pc_coarse_steps;
    st.precond_coarse_warm += ch->pc_coarse_warm;
  }
  st.matvecs = ctx->n_matvec;
  st.n_far = ctx->n_far;
  st.graph_launches = ctx->n_graph_launch;
  st.t_total_ms = tm.ms();
  if (stats) *stats = st;
  if (per_inst)
    for (int b = 0; b < nb; ++b) {
      pqn_mvp_stats pi{};
      pi.gmres_iters = its_per[b];
      pi.matvecs = its_per[b];
      pi.converged = sys[b].conv ? 1 : 0;
      pi.rel_residual = sys[b].relres;
      pi.refine_sweeps = st.refine_sweeps;
      per_inst[b] = pi;
    }
  return st.converged ? PQN_OK : PQN_WARN_NOT_CONVERGED;
}

pqn_status pqn_batch_mobility_apply(pqn_ctx* ctx, const double* const* FT, double* const* UO, pqn_mvp_stats* stats,
                                    pqn_mvp_stats* per_inst) {
  return guarded([&]() -> pqn_status {
    AllocScope alloc_scope(ctx ? &ctx->dev_alloc : nullptr);
    TraceRange trace_range("pqn_batch_mobility_apply");
    if (!ctx || !FT || !UO) return fail(PQN_ERR_INVALID, "pqn_batch_mobility_apply: NULL argument");
    if (!ctx->is_batch) return fail(PQN_ERR_STATE, "pqn_batch_mobility_apply needs a batch context");
    HIPCHK(hipSetDevice(ctx->device));
    return batch_apply_common(ctx, FT, UO, false, stats, per_inst);
  });
}

pqn_status pqn_batch_mobility_apply_dev(pqn_ctx* ctx, const double* const* FT_dev, double* const* UO_dev,
                                        pqn_mvp_stats* stats, pqn_mvp_stats* per_inst) {
  return guarded([&]() -> pqn_status {
    AllocScope alloc_scope(ctx ? &ctx->dev_alloc : nullptr);
    TraceRange trace_range("pqn_batch_mobility_apply_dev");
    if (!ctx || !FT_dev || !UO_dev) return fail(PQN_ERR_INVALID, "pqn_batch_mobility_apply_dev: NULL argument");
    if (!ctx->is_batch) return fail(PQN_ERR_STATE, "pqn_batch_mobility_apply_dev needs a batch context");
    HIPCHK(hipSetDevice(ctx->device));
    return batch_apply_common(ctx, FT_dev, UO_dev, true, stats, per_inst);
  });
}

// K force sets already on the device: FT_dev, UO_dev [K][M][6].
static pqn_status mobility_multi_common(pqn_ctx* ctx, int32_t k_rhs, const double* FT_dev, double* UO_dev,
                                        int32_t fidelity, pqn_mvp_stats* stats) {
  Timer tm;
  Level& lv = ctx->level(fidelity);
  const size_t m6 = 6 * (size_t)ctx->M;
  const double* fp[kMaxRhs];
  double* up[kMaxRhs];
  for (int r = 0; r < k_rhs; ++r) {
    fp[r] = FT_dev + r * m6;
    up[r] = UO_dev + r * m6;
  }
  ctx->n_matvec = 0;
  ctx->n_graph_launch = 0;
  ctx->pc_setup_ms = 0.0;
  ctx->pc_fallback = 0;
  ctx->pc_coarse_steps = 0;
  ctx->pc_coarse_warm = 0;
  ctx->pc_applies = 0;
  ctx->n_far = 0;
  std::fill(ctx->n_far_k, ctx->n_far_k + kMaxRhs, 0);
  pqn_mvp_stats st{};
  ctx->mobility_multi(lv, k_rhs, fp, nullptr, up, &st);
  HIPCHK(hipStreamSynchronize(ctx->stream));
  st.t_far_ms = ctx->end_far_timing();
    stage_stats(*ctx, st);
  st.matvecs = ctx->n_matvec;
  st.n_far = ctx->n_far;
  st.graph_launches = ctx->n_graph_launch;
  st.t_total_ms = tm.ms();
  if (stats) *stats = st;
  return st.converged ? PQN_OK : PQN_WARN_NOT_CONVERGED;
}

pqn_status pqn_mobility_apply_multi(pqn_ctx* ctx, int32_t k_rhs, const double* FT, double* UO, int32_t fidelity,
                                    pqn_mvp_stats* stats) {
  return guarded([&]() -> pqn_status {
    AllocScope alloc_scope(ctx ? &ctx->dev_alloc : nullptr);
    TraceRange trace_range("pqn_mobility_apply_multi");
    if (is_batch(ctx)) return fail(PQN_ERR_STATE, "pqn_mobility_apply_multi needs a single-suspension context");
    if (!ctx || !FT || !UO || k_rhs < 1 || k_rhs > kMaxRhs)
      return fail(PQN_ERR_INVALID, "pqn_mobility_apply_multi: bad argument (1 <= k_rhs <= 6)");
    for (int k = 0; k < 6 * ctx->M * k_rhs; ++k)
      if (!std::isfinite(FT[k])) return fail(PQN_ERR_NUMERIC, "non-finite force/torque");
    HIPCHK(hipSetDevice(ctx->device));
    const size_t m6 = 6 * (size_t)ctx->M;
    HIPCHK(hipMemcpyAsync(ctx->FT.p, FT, k_rhs * m6 * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    const pqn_status s = mobility_multi_common(ctx, k_rhs, ctx->FT.p, ctx->UO.p, fidelity, stats);
    HIPCHK(hipMemcpyAsync(UO, ctx->UO.p, k_rhs * m6 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return s;
  });
}

pqn_status pqn_mobility_apply_multi_dev(pqn_ctx* ctx, int32_t k_rhs, const double* FT_dev, double* UO_dev,
                                        int32_t fidelity, pqn_mvp_stats* stats) {
  return guarded([&]() -> pqn_status {
    AllocScope alloc_scope(ctx ? &ctx->dev_alloc : nullptr);
    TraceRange trace_range("pqn_mobility_apply_multi_dev");
    if (is_batch(ctx)) return fail(PQN_ERR_STATE, "pqn_mobility_apply_multi_dev needs a single-suspension context");
    if (!ctx || !FT_dev || !UO_dev || k_rhs < 1 || k_rhs > kMaxRhs)
      return fail(PQN_ERR_INVALID, "pqn_mobility_apply_multi_dev: bad argument (1 <= k_rhs <= 6)");
    HIPCHK(hipSetDevice(ctx->device));
    return mobility_multi_common(ctx, k_rhs, FT_dev, UO_dev, fidelity, stats);
  });
}

pqn_status pqn_destroy(pqn_ctx* ctx) {
  if (!ctx) return PQN_OK;
  return guarded([&]() -> pqn_status {
    AllocScope alloc_scope(ctx ? &ctx->dev_alloc : nullptr);
    TraceRange trace_range("pqn_destroy");
    HIPCHK(hipSetDevice(ctx->device));
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    delete static_cast<pqn_ctx_impl*>(ctx);
    return PQN_OK;
  });
}

pqn_status pqn_set_state(pqn_ctx* ctx, const double* centers, const double* janus_axes) {
  return guarded([&]() -> pqn_status {
    AllocScope alloc_scope(ctx ? &ctx->dev_alloc : nullptr);
    TraceRange trace_range("pqn_set_state");
    if (is_batch(ctx)) return fail(PQN_ERR_STATE, "pqn_set_state needs a single-suspension context");
    if (!ctx || !centers) return fail(PQN_ERR_INVALID, "pqn_set_state: NULL argument");
    HIPCHK(hipSetDevice(ctx->device));
    ctx->set_configuration(centers, janus_axes ? janus_axes : (ctx->has_axes ? ctx->axes.data() : nullptr));
    return PQN_OK;
  });
}

pqn_status pqn_get_state(const pqn_ctx* ctx, double* centers, double* janus_axes) {
  if (is_batch(ctx)) return fail(PQN_ERR_STATE, "pqn_get_state needs a single-suspension context");
  if (!ctx) return fail(PQN_ERR_INVALID, "pqn_get_state: NULL context");
  if (centers) std::memcpy(centers, ctx->centers.data(), ctx->centers.size() * sizeof(double));
  if (janus_axes) std::memcpy(janus_axes, ctx->axes.data(), ctx->axes.size() * sizeof(double));
  return PQN_OK;
}

pqn_status pqn_set_precision(pqn_ctx* ctx, int32_t precision) {
  if (is_batch(ctx)) return fail(PQN_ERR_STATE, "pqn_set_precision needs a single-suspension context");
  if (!ctx) return fail(PQN_ERR_INVALID, "NULL context");
  if (precision != PQN_FP64 && precision != PQN_MIXED) return fail(PQN_ERR_INVALID, "bad precision");
  ctx->cfg.precision = precision;
  return PQN_OK;
}

static pqn_status mobility_common(pqn_ctx* ctx, const double* FT_dev, const double* axes_dev, double* UO_dev,
                                  int32_t fidelity, pqn_mvp_stats* stats) {
  Timer tm;
  Level& lv = ctx->level(fidelity);
  pqn_mvp_stats st{};
  ctx->n_matvec = 0;
  ctx->n_graph_launch = 0;
  ctx->pc_setup_ms = 0.0;
  ctx->pc_fallback = 0;
  ctx->pc_coarse_steps = 0;
  ctx->pc_coarse_warm = 0;
  ctx->pc_applies = 0;
  ctx->n_far = 0;
  std::fill(ctx->n_far_k, ctx->n_far_k + kMaxRhs, 0);
  ctx->mobility(lv, FT_dev, axes_dev, UO_dev, &st);
  HIPCHK(hipStreamSynchronize(ctx->stream));
  st.t_far_ms = ctx->end_far_timing();
    stage_stats(*ctx, st);
  st.matvecs = ctx->n_matvec;
  st.n_far = ctx->n_far;
  st.graph_launches = ctx->n_graph_launch;
  st.t_total_ms = tm.ms();
  if (stats) *stats = st;
  return st.converged ? PQN_OK : PQN_WARN_NOT_CONVERGED;
}

pqn_status pqn_mobility_apply_dev(pqn_ctx* ctx, const double* FT_dev, double* UO_dev, int32_t fidelity,
                                  pqn_mvp_stats* stats) {
  return guarded([&]() -> pqn_status {
    AllocScope alloc_scope(ctx ? &ctx->dev_alloc : nullptr);
    TraceRange trace_range("pqn_mobility_apply_dev");
    if (is_batch(ctx)) return fail(PQN_ERR_STATE, "pqn_mobility_apply_dev needs a single-suspension context");
    if (!ctx || !FT_dev || !UO_dev) return fail(PQN_ERR_INVALID, "pqn_mobility_apply_dev: NULL argument");
    HIPCHK(hipSetDevice(ctx->device));
    return mobility_common(ctx, FT_dev, nullptr, UO_dev, fidelity, stats);
  });
}

pqn_status pqn_mobility_apply(pqn_ctx* ctx, const double* FT, double* UO, int32_t fidelity, pqn_mvp_stats* stats) {
  return guarded([&]() -> pqn_status {
    AllocScope alloc_scope(ctx ? &ctx->dev_alloc : nullptr);
    TraceRange trace_range("pqn_mobility_apply");
    if (is_batch(ctx)) return fail(PQN_ERR_STATE, "pqn_mobility_apply needs a single-suspension context");
    if (!ctx || !FT || !UO) return fail(PQN_ERR_INVALID, "pqn_mobility_apply: NULL argument");
    for (int k = 0; k < 6 * ctx->M; ++k)
      if (!std::isfinite(FT[k])) return fail(PQN_ERR_NUMERIC, "non-finite force/torque");
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipMemcpyAsync(ctx->FT.p, FT, 6 * (size_t)ctx->M * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    pqn_status s = mobility_common(ctx, ctx->FT.p, nullptr, ctx->UO.p, fidelity, stats);
    HIPCHK(hipMemcpyAsync(UO, ctx->UO.p, 6 * (size_t)ctx->M * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return s;
  });
}

pqn_status pqn_nc_velocity(pqn_ctx* ctx, double* UO, int32_t fidelity, pqn_mvp_stats* stats) {
  return guarded([&]() -> pqn_status {
    AllocScope alloc_scope(ctx ? &ctx->dev_alloc : nullptr);
    TraceRange trace_range("pqn_nc_velocity");
    if (is_batch(ctx)) return fail(PQN_ERR_STATE, "pqn_nc_velocity needs a single-suspension context");
    if (!ctx || !UO) return fail(PQN_ERR_INVALID, "pqn_nc_velocity: NULL argument");
    HIPCHK(hipSetDevice(ctx->device));
    if (!ctx->has_axes) {
      std::fill(UO, UO + 6 * ctx->M, 0.0);
      if (stats) *stats = pqn_mvp_stats{};
      return PQN_OK;
    }
    pqn_status s = mobility_common(ctx, nullptr, ctx->dax.p, ctx->UO.p, fidelity, stats);
    HIPCHK(hipMemcpyAsync(UO, ctx->UO.p, 6 * (size_t)ctx->M * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return s;
  });
}

pqn_status pqn_bie_apply(pqn_ctx* ctx, int32_t fidelity, const double* q, double* y) {
  return guarded([&]() -> pqn_status {
    AllocScope alloc_scope(ctx ? &ctx->dev_alloc : nullptr);
    TraceRange trace_range("pqn_bie_apply");
    if (is_batch(ctx)) return fail(PQN_ERR_STATE, "pqn_bie_apply needs a single-suspension context");
    if (!ctx || !q || !y) return fail(PQN_ERR_INVALID, "pqn_bie_apply: NULL argument");
    HIPCHK(hipSetDevice(ctx->device));
    Level& lv = ctx->level(fidelity);
    const size_t len = 3 * (size_t)lv.N;
    SysBuf& b = lv.sb(0);
    HIPCHK(hipMemcpyAsync(b.rhs.p, q, len * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    ctx->apply_operator(lv, ctx->cfg.precision, b.rhs.p, b.tmp.p);
    HIPCHK(hipMemcpyAsync(y, b.tmp.p, len * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->end_far_timing();
    return PQN_OK;
  });
}

pqn_status pqn_bie_apply_multi(pqn_ctx* ctx, int32_t fidelity, int32_t k, const double* q, double* y) {
  return guarded([&]() -> pqn_status {
    AllocScope alloc_scope(ctx ? &ctx->dev_alloc : nullptr);
    TraceRange trace_range("pqn_bie_apply_multi");
    if (is_batch(ctx)) return fail(PQN_ERR_STATE, "pqn_bie_apply_multi needs a single-suspension context");
    if (!ctx || !q || !y) return fail(PQN_ERR_INVALID, "pqn_bie_apply_multi: NULL argument");
    if (k < 1 || k > kMaxRhs) return fail(PQN_ERR_INVALID, "pqn_bie_apply_multi: k must be 1..6");
    HIPCHK(hipSetDevice(ctx->device));
    Level& lv = ctx->level(fidelity);
    const size_t len = 3 * (size_t)lv.N;
    std::vector<MvGroup> groups;
    for (int r = 0; r < k; ++r) {
      SysBuf& b = lv.sb(r);
      HIPCHK(hipMemcpyAsync(b.rhs.p, q + r * len, len * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
      add_to_groups(groups, ctx, &lv, r, b.rhs.p, b.tmp.p);
    }
    ctx->matvec_groups(groups, ctx->cfg.precision);
    for (int r = 0; r < k; ++r)
      HIPCHK(hipMemcpyAsync(y + r * len, lv.sb(r).tmp.p, len * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->end_far_timing();
    return PQN_OK;
  });
}

pqn_status pqn_bie_solve(pqn_ctx* ctx, int32_t fidelity, const double* rhs, double* q, pqn_mvp_stats* stats) {
  return guarded([&]() -> pqn_status {
    AllocScope alloc_scope(ctx ? &ctx->dev_alloc : nullptr);
    TraceRange trace_range("pqn_bie_solve");
    if (is_batch(ctx)) return fail(PQN_ERR_STATE, "pqn_bie_solve needs a single-suspension context");
    if (!ctx || !rhs || !q) return fail(PQN_ERR_INVALID, "pqn_bie_solve: NULL argument");
    HIPCHK(hipSetDevice(ctx->device));
    Timer tm;
    Level& lv = ctx->level(fidelity);
    const size_t len = 3 * (size_t)lv.N;
    ctx->n_matvec = 0;
    ctx->n_graph_launch = 0;
    ctx->pc_setup_ms = 0.0;
    ctx->pc_fallback = 0;
    ctx->pc_coarse_steps = 0;
    ctx->pc_coarse_warm = 0;
    ctx->pc_applies = 0;
    ctx->n_far = 0;
    std::fill(ctx->n_far_k, ctx->n_far_k + kMaxRhs, 0);
    SysBuf& b = lv.sb(0);
    HIPCHK(hipMemcpyAsync(b.rhs.p, rhs, len * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    pqn_mvp_stats st{};
    std::vector<SysRef> sys{SysRef{ctx, &lv, 0, b.rhs.p, b.x.p, lv.tol}};
    ctx->solve_lockstep(sys, &st);
    HIPCHK(hipMemcpyAsync(q, b.x.p, len * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    st.t_far_ms = ctx->end_far_timing();
    stage_stats(*ctx, st);
    st.matvecs = ctx->n_matvec;
    st.n_far = ctx->n_far;
    st.graph_launches = ctx->n_graph_launch;
    st.t_total_ms = tm.ms();
    if (stats) *stats = st;
    return st.converged ? PQN_OK : PQN_WARN_NOT_CONVERGED;
  });
}

pqn_status pqn_get_self_block(pqn_ctx* ctx, int32_t fidelity, double* S) {
  return guarded([&]() -> pqn_status {
    AllocScope alloc_scope(ctx ? &ctx->dev_alloc : nullptr);
    TraceRange trace_range("pqn_get_self_block");
    if (is_batch(ctx)) return fail(PQN_ERR_STATE, "pqn_get_self_block needs a single-suspension context");
    if (!ctx || !S) return fail(PQN_ERR_INVALID, "pqn_get_self_block: NULL argument");
    Level& lv = ctx->level(fidelity);
    std::memcpy(S, lv.tab.S.data(), lv.tab.S.size() * sizeof(double));
    return PQN_OK;
  });
}

pqn_status pqn_get_grid(pqn_ctx* ctx, int32_t fidelity, int32_t* n_nodes, double* offsets, double* weights) {
  return guarded([&]() -> pqn_status {
    AllocScope alloc_scope(ctx ? &ctx->dev_alloc : nullptr);
    TraceRange trace_range("pqn_get_grid");
    if (is_batch(ctx)) return fail(PQN_ERR_STATE, "pqn_get_grid needs a single-suspension context");
    if (!ctx) return fail(PQN_ERR_INVALID, "pqn_get_grid: NULL context");
    Level& lv = ctx->level(fidelity);
    if (n_nodes) *n_nodes = lv.n;
    if (offsets) std::memcpy(offsets, lv.tab.off.data(), lv.tab.off.size() * sizeof(double));
    if (weights) std::memcpy(weights, lv.tab.w.data(), lv.tab.w.size() * sizeof(double));
    return PQN_OK;
  });
}

pqn_status pqn_host_self_block(int32_t n_theta, int32_t n_phi, double radius, double* offsets, double* weights,
                               double* S) {
  return guarded([&]() -> pqn_status {
    if (!(radius > 0.0)) return fail(PQN_ERR_INVALID, "radius must be > 0");
    SphereTables t;
    build_sphere_tables(n_theta, n_phi, radius, 1, t);
    if (offsets) std::memcpy(offsets, t.off.data(), t.off.size() * sizeof(double));
    if (weights) std::memcpy(weights, t.w.data(), t.w.size() * sizeof(double));
    if (S) std::memcpy(S, t.S.data(), t.S.size() * sizeof(double));
    return PQN_OK;
  });
}

pqn_status pqn_host_sphere_block(int32_t n_theta, int32_t n_phi, double radius, double* D, double* Dinv) {
  return guarded([&]() -> pqn_status {
    if (!(radius > 0.0)) return fail(PQN_ERR_INVALID, "radius must be > 0");
    if (n_theta < 2 || n_phi < 2 * n_theta - 1 || n_theta > kMaxDegree + 1)
      return fail(PQN_ERR_INVALID, "grid needs 2 <= n_theta <= 41 and n_phi >= 2 n_theta - 1");
    SphereTables t;
    build_sphere_tables(n_theta, n_phi, radius, 1, t);
    std::vector<double> d;
    single_sphere_block(t, d);
    if (D) std::memcpy(D, d.data(), d.size() * sizeof(double));
    if (Dinv) {
      invert_gauss_jordan(d, 3 * t.n);
      std::memcpy(Dinv, d.data(), d.size() * sizeof(double));
    }
    return PQN_OK;
  });
}

pqn_status pqn_find_contacts(pqn_ctx* ctx, double delta, int32_t cap, int32_t* n_out, int32_t* pairs, double* gaps) {
  return guarded([&]() -> pqn_status {
    AllocScope alloc_scope(ctx ? &ctx->dev_alloc : nullptr);
    TraceRange trace_range("pqn_find_contacts");
    if (is_batch(ctx)) return fail(PQN_ERR_STATE, "pqn_find_contacts needs a single-suspension context");
    if (!ctx || !n_out || (cap > 0 && (!pairs || !gaps)) || cap < 0)
      return fail(PQN_ERR_INVALID, "pqn_find_contacts: bad argument");
    HIPCHK(hipSetDevice(ctx->device));
    int n = lcp_find_contacts(*ctx, delta);
    *n_out = n;
    if (n > cap) return fail(PQN_ERR_INVALID, "pqn_find_contacts: cap too small");
    lcp_copy_contacts(*ctx, n, pairs, gaps);
    return PQN_OK;
  });
}

pqn_status pqn_find_contacts_noalloc(pqn_ctx* ctx, double delta, int32_t cap, int32_t* n_out, int32_t* pairs,
                                     double* gaps) {
  return guarded([&]() -> pqn_status {
    TraceRange trace_range("pqn_find_contacts_noalloc");
    if (is_batch(ctx)) return fail(PQN_ERR_STATE, "pqn_find_contacts_noalloc needs a single-suspension context");
    if (!ctx || !n_out || (cap > 0 && (!pairs || !gaps)) || cap < 0)
      return fail(PQN_ERR_INVALID, "pqn_find_contacts_noalloc: bad argument");
    HIPCHK(hipSetDevice(ctx->device));
    return lcp_find_contacts_noalloc(*ctx, delta, cap, n_out, pairs, gaps);
  });
}

pqn_status pqn_lcp_apply(pqn_ctx* ctx, int32_t n, const int32_t* pairs, const double* x, double* Ax,
                         int32_t fidelity) {
  return guarded([&]() -> pqn_status {
    AllocScope alloc_scope(ctx ? &ctx->dev_alloc : nullptr);
    TraceRange trace_range("pqn_lcp_apply");
    if (is_batch(ctx)) return fail(PQN_ERR_STATE, "pqn_lcp_apply needs a single-suspension context");
    if (!ctx || n < 0 || (n > 0 && (!pairs || !x || !Ax))) return fail(PQN_ERR_INVALID, "pqn_lcp_apply: bad argument");
    HIPCHK(hipSetDevice(ctx->device));
    lcp_check_pairs(*ctx, n, pairs);
    return lcp_apply_host(*ctx, n, pairs, x, Ax, fidelity);
  });
}

pqn_status pqn_lcp_solve(pqn_ctx* ctx, int32_t n, const int32_t* pairs, const double* b, double* x, int32_t solver,
                         const pqn_lcp_opts* opts, pqn_lcp_stats* stats) {
  return guarded([&]() -> pqn_status {
    AllocScope alloc_scope(ctx ? &ctx->dev_alloc : nullptr);
    TraceRange trace_range("pqn_lcp_solve");
    if (is_batch(ctx)) return fail(PQN_ERR_STATE, "pqn_lcp_solve needs a single-suspension context");
    if (!ctx || n < 0 || (n > 0 && (!pairs || !b || !x))) return fail(PQN_ERR_INVALID, "pqn_lcp_solve: bad argument");
    if (solver < PQN_BBPGD || solver > PQN_BI_REC) return fail(PQN_ERR_INVALID, "bad solver");
    if (const char* why = solver_unavailable(*ctx, solver)) return fail(PQN_ERR_STATE, why);
    HIPCHK(hipSetDevice(ctx->device));
    lcp_check_pairs(*ctx, n, pairs);
    return lcp_solve_host(*ctx, n, pairs, b, x, solver, opts, stats);
  });
}

pqn_status pqn_lcp_solve_dev(pqn_ctx* ctx, int32_t n, const int32_t* pairs_dev, const double* b_dev, double* x_dev,
                             int32_t solver, const pqn_lcp_opts* opts, pqn_lcp_stats* stats) {
  return guarded([&]() -> pqn_status {
    AllocScope alloc_scope(ctx ? &ctx->dev_alloc : nullptr);
    TraceRange trace_range("pqn_lcp_solve_dev");
    if (is_batch(ctx)) return fail(PQN_ERR_STATE, "pqn_lcp_solve_dev needs a single-suspension context");
    if (!ctx || n < 0 || (n > 0 && (!pairs_dev || !b_dev || !x_dev)))
      return fail(PQN_ERR_INVALID, "pqn_lcp_solve_dev: bad argument");
    if (solver < PQN_BBPGD || solver > PQN_BI_REC) return fail(PQN_ERR_INVALID, "bad solver");
    if (const char* why = solver_unavailable(*ctx, solver)) return fail(PQN_ERR_STATE, why);
    HIPCHK(hipSetDevice(ctx->device));
    return lcp_solve_dev(*ctx, n, pairs_dev, b_dev, x_dev, solver, opts, stats);
  });
}

pqn_status pqn_step(pqn_ctx* ctx, double dt, double delta, int32_t solver, const pqn_lcp_opts* opts,
                    pqn_step_stats* stats) {
  return guarded([&]() -> pqn_status {
    AllocScope alloc_scope(ctx ? &ctx->dev_alloc : nullptr);
    TraceRange trace_range("pqn_step");
    if (is_batch(ctx)) return fail(PQN_ERR_STATE, "pqn_step needs a single-suspension context");
    if (!ctx || !(dt > 0.0) || !std::isfinite(delta)) return fail(PQN_ERR_INVALID, "pqn_step: bad argument");
    if (solver < PQN_BBPGD || solver > PQN_BI_REC) return fail(PQN_ERR_INVALID, "bad solver");
    if (const char* why = solver_unavailable(*ctx, solver)) return fail(PQN_ERR_STATE, why);
    HIPCHK(hipSetDevice(ctx->device));
    return lcp_step(*ctx, dt, delta, solver, opts, stats);
  });
}

}  // extern "C"
