// Context set-up, the discrete BIE operator, GMRES and the mobility product.
#include "context.hpp"

#include <algorithm>
#include <cstring>

namespace bipqn {

pqn_ctx_impl::~pqn_ctx_impl() {
  lcp_release(lcp);
  lcp = nullptr;
  for (auto& e : ev_pool) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  if (own_stream && stream) (void)hipStreamDestroy(stream);
}

void pqn_ctx_impl::setup_level(Level& lv, int nt, int np, double tol) {
  build_sphere_tables(nt, np, a, cfg.near_up, lv.tab);
  SphereTables& t = lv.tab;
  lv.M = M;
  lv.n = t.n;
  lv.N = M * t.n;
  lv.L = t.L;
  lv.nup = t.n_up;
  lv.p = t.p;
  lv.off.upload(t.off.data(), t.off.size(), stream);
  lv.w.upload(t.w.data(), t.w.size(), stream);
  lv.G.upload(t.G.data(), t.G.size(), stream);
  lv.T.upload(t.T.data(), t.T.size(), stream);
  lv.Yup.upload(t.Y_up.data(), t.Y_up.size(), stream);
  std::vector<double4> ou(t.n_up);
  for (int f = 0; f < t.n_up; ++f)
    ou[f] = make_double4(t.off_up[3 * f], t.off_up[3 * f + 1], t.off_up[3 * f + 2], t.w_up[f]);
  lv.offup.upload(ou.data(), ou.size(), stream);
  const int N = lv.N;
  lv.tpt = cfg.targets_per_thread == 1 ? 1 : 2;
  const int nbt = (N + 256 * lv.tpt - 1) / (256 * lv.tpt);
  int nch = cfg.far_chunks > 0 ? cfg.far_chunks : std::max(1, (4096 + nbt - 1) / nbt);
  nch = std::min(nch, M);
  lv.spc = (M + nch - 1) / nch;
  lv.nchunks = (M + lv.spc - 1) / lv.spc;
  lv.src32.alloc(2 * (size_t)N);
  lv.src64.alloc(4 * (size_t)N);
  lv.far_part.alloc((size_t)lv.nchunks * 3 * N);
  lv.near_part.alloc((size_t)kMaxNear * 3 * N);
  lv.coef.alloc((size_t)3 * M * lv.L);
  lv.qup.alloc((size_t)3 * M * lv.nup);
  lv.selfo.alloc((size_t)9 * N);
  lv.mom.alloc((size_t)6 * M);
  lv.restart = cfg.gmres_restart;
  lv.max_iter = cfg.gmres_max_iter;
  lv.tol = tol;
  const size_t len = 3 * (size_t)N;
  lv.V.alloc((size_t)(lv.restart + 1) * len);
  lv.x.alloc(len);
  lv.r.alloc(len);
  lv.rhs.alloc(len);
  lv.tmp.alloc(len);
  lv.d.alloc(len);
  lv.nb_dots = (int)std::min<long>(256, std::max<long>(1, (long)(len / 2048)));
  lv.partial.alloc((size_t)lv.nb_dots * (lv.restart + 1));
  lv.h.alloc(4 * (size_t)(lv.restart + 2));
  lv.ycoef.alloc((size_t)lv.restart + 1);
}

void pqn_ctx_impl::set_configuration(const double* c, const double* ax) {
  centers.assign(c, c + 3 * (size_t)M);
  for (double v : centers)
    if (!std::isfinite(v)) throw Error(PQN_ERR_NUMERIC, "non-finite centre coordinate");
  has_axes = ax != nullptr;
  axes.assign(3 * (size_t)M, 0.0);
  if (ax) std::copy(ax, ax + 3 * (size_t)M, axes.begin());
  // pair classes: 2 = same sphere, 1 = near (gap < near_gap), 0 = far
  std::vector<unsigned char> hc((size_t)M * M, 0);
  h_partners.assign((size_t)M * kMaxNear, -1);
  h_npart.assign(M, 0);
  max_slots = 0;
  for (int i = 0; i < M; ++i) {
    for (int j = 0; j < M; ++j) {
      if (i == j) {
        hc[(size_t)i * M + j] = 2;
        continue;
      }
      double dx = centers[3 * i] - centers[3 * j], dy = centers[3 * i + 1] - centers[3 * j + 1],
             dz = centers[3 * i + 2] - centers[3 * j + 2];
      double gap = std::sqrt(dx * dx + dy * dy + dz * dz) - 2.0 * a;
      if (gap < cfg.near_gap) {
        hc[(size_t)i * M + j] = 1;
        int& k = h_npart[i];
        if (k >= kMaxNear) throw Error(PQN_ERR_INVALID, "more than 16 near neighbours of one sphere");
        h_partners[(size_t)i * kMaxNear + k] = j;
        ++k;
      }
    }
    max_slots = std::max(max_slots, h_npart[i]);
  }
  // ordered near pairs (target sphere, source sphere, partner slot)
  std::vector<int> nl;
  for (int i = 0; i < M; ++i)
    for (int s = 0; s < h_npart[i]; ++s) {
      nl.push_back(i);
      nl.push_back(h_partners[(size_t)i * kMaxNear + s]);
      nl.push_back(s);
    }
  n_near = (int)nl.size() / 3;
  near_list.upload(nl.data(), nl.size(), stream);
  ctr.upload(centers.data(), centers.size(), stream);
  dax.upload(axes.data(), axes.size(), stream);
  cls.upload(hc.data(), hc.size(), stream);
  partners.upload(h_partners.data(), h_partners.size(), stream);
  npart.upload(h_npart.data(), h_npart.size(), stream);
  HIPCHK(hipStreamSynchronize(stream));
}

void pqn_ctx_impl::begin_far_timing() {
  if (!cfg.profile) return;
  if (ev_used == ev_pool.size()) {
    hipEvent_t a0, b0;
    HIPCHK(hipEventCreate(&a0));
    HIPCHK(hipEventCreate(&b0));
    ev_pool.emplace_back(a0, b0);
  }
  HIPCHK(hipEventRecord(ev_pool[ev_used].first, stream));
}

double pqn_ctx_impl::end_far_timing() {
  // called after the stream has been synchronised: sums and recycles the events
  double t = 0.0;
  for (size_t k = 0; k < ev_used; ++k) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ev_pool[k].first, ev_pool[k].second));
    t += ms;
  }
  ev_used = 0;
  return t;
}

// y = (1/2 I + D + P) q on the level's grid; q, y device [3][N].
void pqn_ctx_impl::apply_operator(Level& lv, int precision, const double* q, double* y) {
  const int n = lv.n, N = lv.N, L = lv.L, nup = lv.nup;
  hipStream_t s = stream;
  const double scale = 3.0 / (4.0 * kPi * a);
  // harmonic coefficients of every sphere's density (per component): coef = T q
  launch_gemm64(s, L, M, n, lv.T.p, n, 0, q, N, n, 0, n, lv.coef.p, (long)M * L, L, 0, L, 3);
  // singular self interaction on the coefficients, one partial per source component d:
  // self_d = G[:, d block] coef_d
  launch_gemm64(s, 3 * n, M, L, lv.G.p, 3 * L, L, lv.coef.p, (long)M * L, L, 0, L, lv.selfo.p, 3L * N, n, N, n, 3);
  if (n_near > 0)   // density on the upsampled grid of every sphere: qup = Yup coef
    launch_gemm64(s, nup, M, L, lv.Yup.p, L, 0, lv.coef.p, (long)M * L, L, 0, L, lv.qup.p, (long)M * nup, nup, 0,
                  nup, 3);
  begin_far_timing();
  if (precision == PQN_MIXED) {
    launch_pack32(s, q, lv.off.p, lv.w.p, n, N, lv.src32.p);
    launch_far32(s, lv.tpt, lv.src32.p, lv.off.p, ctr.p, cls.p, n, M, N, lv.spc, lv.nchunks, scale, lv.far_part.p);
  } else {
    launch_pack64(s, q, lv.off.p, lv.w.p, n, N, lv.src64.p);
    launch_far64(s, lv.src64.p, lv.off.p, ctr.p, cls.p, n, M, N, lv.spc, lv.nchunks, scale, lv.far_part.p);
  }
  if (cfg.profile) {
    HIPCHK(hipEventRecord(ev_pool[ev_used].second, s));
    ++ev_used;
  }
  ++n_far;
  launch_near64p(s, n_near, ctr.p, lv.off.p, lv.offup.p, lv.qup.p, lv.coef.p, near_list.p, n, M, N, nup, lv.p, L,
                 scale, lv.near_part.p);
  launch_moments(s, q, lv.off.p, lv.w.p, n, M, N, lv.mom.p);
  launch_combine(s, q, lv.selfo.p, 3, lv.far_part.p, lv.nchunks, lv.near_part.p, npart.p, lv.mom.p, lv.off.p, n, N,
                 a, y);
  HIPCHK(hipGetLastError());
  ++n_matvec;
}

double pqn_ctx_impl::dot_host(const double* x, const double* y, long len, Level& lv) {
  launch_dots(stream, x, len, 1, y, len, lv.nb_dots, lv.partial.p, lv.h.p);
  double v = 0.0;
  HIPCHK(hipMemcpyAsync(&v, lv.h.p, sizeof(double), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  return v;
}

// Restarted GMRES(m): classical Gram-Schmidt with one reorthogonalisation
// (CGS2) in FP64 on the device, Givens rotations and the small least-squares
// problem on the host. x is overwritten (initial guess 0).
int pqn_ctx_impl::gmres(Level& lv, int precision, const double* rhs, double* x, double tol, double* relres,
                        bool* conv) {
  const long len = 3L * lv.N;
  const int m = lv.restart;
  hipStream_t s = stream;
  double* V = lv.V.p;
  const double bnorm = std::sqrt(dot_host(rhs, rhs, len, lv));
  if (!std::isfinite(bnorm)) throw Error(PQN_ERR_NUMERIC, "non-finite right-hand side");
  launch_scale_copy(s, x, rhs, 0.0, len);  // x = 0 (rhs finite)
  *conv = true;
  *relres = 0.0;
  if (bnorm == 0.0) return 0;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), hbuf(2 * (m + 1) + 1);
  int its = 0;
  double beta = bnorm;
  const double* r0 = rhs;
  for (;;) {
    launch_scale_copy(s, V, r0, 1.0 / beta, len);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0, done_k = 0;
    bool stop = false;
    for (k = 0; k < m; ++k) {
      double* vk = V + (size_t)k * len;
      double* w = V + (size_t)(k + 1) * len;
      apply_operator(lv, precision, vk, w);
      for (int pass = 0; pass < 2; ++pass) {
        double* hp = lv.h.p + pass * (m + 1);
        launch_dots(s, V, len, k + 1, w, len, lv.nb_dots, lv.partial.p, hp);
        launch_combo(s, w, 1.0, V, len, k + 1, hp, -1.0, len);
      }
      launch_dots(s, w, len, 1, w, len, lv.nb_dots, lv.partial.p, lv.h.p + 2 * (m + 1));
      HIPCHK(hipMemcpyAsync(hbuf.data(), lv.h.p, (2 * (m + 1) + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      ++its;
      for (int i = 0; i <= k; ++i) H[(size_t)i * m + k] = hbuf[i] + hbuf[m + 1 + i];
      const double hn = std::sqrt(std::max(0.0, hbuf[2 * (m + 1)]));
      if (!std::isfinite(hn)) throw Error(PQN_ERR_NUMERIC, "non-finite value in GMRES");
      H[(size_t)(k + 1) * m + k] = hn;
      if (hn > 0.0) launch_scale_copy(s, w, w, 1.0 / hn, len);
      for (int i = 0; i < k; ++i) {
        const double t0 = cs[i] * H[(size_t)i * m + k] + sn[i] * H[(size_t)(i + 1) * m + k];
        H[(size_t)(i + 1) * m + k] = -sn[i] * H[(size_t)i * m + k] + cs[i] * H[(size_t)(i + 1) * m + k];
        H[(size_t)i * m + k] = t0;
      }
      const double den = std::hypot(H[(size_t)k * m + k], H[(size_t)(k + 1) * m + k]);
      if (!(den > 0.0)) throw Error(PQN_ERR_NUMERIC, "GMRES breakdown: zero Hessenberg column");
      cs[k] = H[(size_t)k * m + k] / den;
      sn[k] = H[(size_t)(k + 1) * m + k] / den;
      H[(size_t)k * m + k] = den;
      H[(size_t)(k + 1) * m + k] = 0.0;
      g[k + 1] = -sn[k] * g[k];
      g[k] = cs[k] * g[k];
      done_k = k + 1;
      *relres = std::fabs(g[k + 1]) / bnorm;
      if (std::fabs(g[k + 1]) <= tol * bnorm || hn == 0.0) {
        stop = true;
        break;
      }
      if (its >= lv.max_iter) break;
    }
    // y = H^{-1} g (upper triangular), x += V y
    std::vector<double> y(done_k);
    for (int i = done_k - 1; i >= 0; --i) {
      double v = g[i];
      for (int j = i + 1; j < done_k; ++j) v -= H[(size_t)i * m + j] * y[j];
      y[i] = v / H[(size_t)i * m + i];
    }
    HIPCHK(hipMemcpyAsync(lv.ycoef.p, y.data(), done_k * sizeof(double), hipMemcpyHostToDevice, s));
    launch_combo(s, x, 1.0, V, len, done_k, lv.ycoef.p, 1.0, len);
    if (stop) {
      *conv = true;
      return its;
    }
    if (its >= lv.max_iter) {
      *conv = false;
      return its;
    }
    // restart from the true residual
    apply_operator(lv, precision, x, lv.r.p);
    launch_axpby(s, lv.r.p, rhs, 1.0, -1.0, len);  // r = rhs - A x
    beta = std::sqrt(dot_host(lv.r.p, lv.r.p, len, lv));
    *relres = beta / bnorm;
    if (beta <= tol * bnorm) {
      *conv = true;
      return its;
    }
    r0 = lv.r.p;
  }
}

// Solve (1/2 + D + P) x = rhs in the context's precision. Mixed precision:
// GMRES on the operator with FP32 far pair sums, then optional refinement
// sweeps whose residual uses the FP64 operator.
void pqn_ctx_impl::solve(Level& lv, const double* rhs, double* x, pqn_mvp_stats* st) {
  const long len = 3L * lv.N;
  double rel = 0.0;
  bool conv = false;
  const int prec = cfg.precision;
  int its = gmres(lv, prec, rhs, x, lv.tol, &rel, &conv);
  int sweeps = 0;
  if (prec == PQN_MIXED && cfg.refine_sweeps > 0) {
    const double bnorm = std::sqrt(dot_host(rhs, rhs, len, lv));
    for (int sw = 0; sw < cfg.refine_sweeps && bnorm > 0.0; ++sw) {
      apply_operator(lv, PQN_FP64, x, lv.tmp.p);
      launch_axpby(stream, lv.tmp.p, rhs, 1.0, -1.0, len);  // tmp = rhs - A64 x
      const double rn = std::sqrt(dot_host(lv.tmp.p, lv.tmp.p, len, lv));
      rel = rn / bnorm;
      conv = rel <= lv.tol;
      if (conv) break;
      ++sweeps;
      // correction d for A_mixed d = tmp, to the tolerance that makes |r| <= tol |rhs|
      double rel2 = 0.0;
      bool c2 = false;
      its += gmres(lv, prec, lv.tmp.p, lv.d.p, std::min(0.5, lv.tol * bnorm / rn), &rel2, &c2);
      launch_axpby(stream, x, lv.d.p, 1.0, 1.0, len);
    }
  }
  if (st) {
    st->gmres_iters += its;
    st->refine_sweeps += sweeps;
    st->rel_residual = rel;
    st->converged = conv ? 1 : 0;
  }
}

void pqn_ctx_impl::mobility(Level& lv, const double* FT_dev, const double* axes_dev, double* UO_dev,
                            pqn_mvp_stats* st) {
  launch_rhs(stream, ctr.p, FT_dev, axes_dev, lv.off.p, lv.n, M, lv.N, a, mu, cfg.slip_speed, lv.rhs.p);
  solve(lv, lv.rhs.p, lv.x.p, st);
  launch_moments(stream, lv.x.p, lv.off.p, lv.w.p, lv.n, M, lv.N, lv.mom.p);
  launch_rigid_velocity(stream, lv.mom.p, M, a, UO_dev);
  HIPCHK(hipGetLastError());
}

}  // namespace bipqn
