// Context set-up, the discrete BIE operator on groups of densities, lockstep
// GMRES and the mobility product.
#include "context.hpp"

#include <algorithm>
#include <array>
#include <cstring>

namespace bipqn {

constexpr int kMultiDotBlocks = 16;  // reduction blocks per vector in the segmented dot kernel


// One GEMM problem of a segmented launch: C(r, col) = sum_k A[r lda + k] B[col ldb + k],
// stored at C[(r / rb) rbs + (r % rb) rs + (col / cb) cbs + (col % cb) ldc] (cb = 0: no
// column blocks).
void push_gemm(std::vector<GemmDesc>& v, int& blocks, int R, int Cn, int K, const double* A, int lda,
               const double* B, int ldb, double* C, int rb, long rbs, int ldc, int rs, int cb, long cbs, int at,
               int big) {
  const int tile = big ? 64 : 32;
  GemmDesc d{A, B, C, rbs, R, Cn, K, lda, ldb, rb, ldc, (R + tile - 1) / tile, blocks, rs, cb > 0 ? cb : Cn, cbs,
             nullptr, at};
  blocks += d.tr * ((Cn + tile - 1) / tile);
  v.push_back(d);
}

char* pqn_ctx_impl::push_desc_pack(const std::vector<char>& pack) { return push_desc_pack(pack, stream, ddesc); }

char* pqn_ctx_impl::push_desc_pack(const std::vector<char>& pack, hipStream_t st, DevArray<char>& table) {
  if (pack.size() > table.count) {
    // growing the table: wait for kernels still reading the old one
    HIPCHK(hipStreamSynchronize(st));
    table.alloc(std::max<size_t>(pack.size() * 2, 1 << 16));
  }
  HIPCHK(hipMemcpyAsync(table.p, pack.data(), pack.size(), hipMemcpyHostToDevice, st));
  return table.p;
}

hipStream_t pqn_ctx_impl::side_stream() {
  if (!side) {
    HIPCHK(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&ev_in, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ev_side, hipEventDisableTiming));
  }
  return side;
}

Work& Level::wk(int k) {
  while ((int)work.size() <= k) work.emplace_back(new Work());
  Work& w = *work[k];
  if (!w.far_part.p) {
    w.far_part.alloc((size_t)nchunks * 3 * N);
    w.near_part.alloc((size_t)kMaxNear * 3 * N);
    w.coef.alloc((size_t)3 * M * L);
    w.qup.alloc((size_t)3 * M * nup);
    if (nup2 > 0) w.qup2.alloc((size_t)3 * M * nup2);
    w.selfo.alloc((size_t)9 * N);
    w.mom.alloc((size_t)6 * M);
  }
  return w;
}

SysBuf& Level::sb(int k) {
  while ((int)sys.size() <= k) sys.emplace_back(new SysBuf());
  SysBuf& b = *sys[k];
  if (!b.V.p) {
    const size_t len = 3 * (size_t)N;
    b.V.alloc((size_t)(restart + 1) * len);
    b.x.alloc(len);
    b.r.alloc(len);
    b.rhs.alloc(len);
    b.tmp.alloc(len);
    b.d.alloc(len);
    b.partial.alloc((size_t)std::max(nb_dots, kMultiDotBlocks) * (restart + 1));
    b.ycoef.alloc((size_t)restart + 1);
    b.rcoef.alloc((size_t)restart + 2);
  }
  return b;
}

pqn_ctx_impl::~pqn_ctx_impl() {
  lcp_release(lcp);
  lcp = nullptr;
  children.clear();
  for (auto& pool : ev_pool)
    for (auto& e : pool) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  if (side) {
    (void)hipStreamSynchronize(side);
    (void)hipStreamDestroy(side);
    (void)hipEventDestroy(ev_in);
    (void)hipEventDestroy(ev_side);
  }
  if (own_stream && stream) (void)hipStreamDestroy(stream);
}

void pqn_ctx_impl::setup_level(Level& lv, int nt, int np, double tol, int far_theta) {
  build_sphere_tables(nt, np, a, cfg.near_up, lv.tab, cfg.near_close_gap > 0.0 ? cfg.near_close_up : 0, far_theta);
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
  lv.shab.upload(t.shab.data(), t.shab.size(), stream);
  std::vector<double4> ou(t.n_up);
  for (int f = 0; f < t.n_up; ++f)
    ou[f] = make_double4(t.off_up[3 * f], t.off_up[3 * f + 1], t.off_up[3 * f + 2], t.w_up[f]);
  lv.offup.upload(ou.data(), ou.size(), stream);
  lv.nup2 = t.n_up2;
  if (lv.nup2 > 0) {
    std::vector<double4> ou2(t.n_up2);
    for (int f = 0; f < t.n_up2; ++f)
      ou2[f] = make_double4(t.off_up2[3 * f], t.off_up2[3 * f + 1], t.off_up2[3 * f + 2], t.w_up2[f]);
    lv.offup2.upload(ou2.data(), ou2.size(), stream);
    lv.Yup2.upload(t.Y_up2.data(), t.Y_up2.size(), stream);
  }
  lv.nc = t.nc;
  lv.Lc = t.Lc;
  if (lv.nc > 0) {
    lv.offc.upload(t.off_c.data(), t.off_c.size(), stream);
    lv.wc.upload(t.w_c.data(), t.w_c.size(), stream);
    lv.Yc.upload(t.Y_c.data(), t.Y_c.size(), stream);
  }
  const int N = lv.N;
  lv.tpt = far_layout(cfg);
  const int tgt_per_block = lv.tpt == 0 ? 64 : 256 * lv.tpt;
  const int nbt = (N + tgt_per_block - 1) / tgt_per_block;
  int nch = cfg.far_chunks > 0 ? cfg.far_chunks : std::max(1, (4096 + nbt - 1) / nbt);
  nch = std::min(nch, M);
  lv.spc = (M + nch - 1) / nch;
  lv.nchunks = (M + lv.spc - 1) / lv.spc;
  lv.src.alloc((size_t)N * src64_stride(kMaxRhs));
  lv.restart = cfg.gmres_restart;
  lv.max_iter = cfg.gmres_max_iter;
  lv.tol = tol;
  const size_t len = 3 * (size_t)N;
  lv.nb_dots = (int)std::min<long>(256, std::max<long>(1, (long)(len / 2048)));
}

void pqn_ctx_impl::set_configuration(const double* c, const double* ax) {
  // Everything is derived into locals and validated first; the context's state
  // changes only once no check can fail (a rejected configuration leaves it as it was).
  std::vector<double> cn(c, c + 3 * (size_t)M);
  for (double v : cn)
    if (!std::isfinite(v)) throw Error(PQN_ERR_NUMERIC, "non-finite centre coordinate");
  // ax may point into axes itself (re-setting the centres only): copy before overwriting
  std::vector<double> axn(3 * (size_t)M, 0.0);
  if (ax) std::copy(ax, ax + 3 * (size_t)M, axn.begin());
  // pair classes: 2 = same sphere, 1 = near (gap < near_gap), 0 = far
  std::vector<unsigned char> hc((size_t)M * M, 0);
  std::vector<int> hp((size_t)M * kMaxNear, -1), hn(M, 0);
  std::vector<char> h_close((size_t)M * kMaxNear, 0);
  int slots = 0;
  for (int i = 0; i < M; ++i) {
    for (int j = 0; j < M; ++j) {
      if (i == j) {
        hc[(size_t)i * M + j] = 2;
        continue;
      }
      double dx = cn[3 * i] - cn[3 * j], dy = cn[3 * i + 1] - cn[3 * j + 1], dz = cn[3 * i + 2] - cn[3 * j + 2];
      double gap = std::sqrt(dx * dx + dy * dy + dz * dz) - 2.0 * a;
      if (gap < cfg.near_gap) {
        hc[(size_t)i * M + j] = 1;
        int& k = hn[i];
        if (k >= kMaxNear) throw Error(PQN_ERR_INVALID, "more than 16 near neighbours of one sphere");
        hp[(size_t)i * kMaxNear + k] = j;
        h_close[(size_t)i * kMaxNear + k] = gap < cfg.near_close_gap;
        ++k;
      }
    }
    slots = std::max(slots, hn[i]);
  }
  // ordered near pairs (target sphere, source sphere, partner slot), grouped by
  // source sphere so that launches reading the same source data run together
  // (close pairs, gap < near_close_gap, in a list of their own for the finer grid)
  std::vector<int> nl, nl2;
  {
    std::vector<std::array<int, 3>> pr;
    for (int i = 0; i < M; ++i)
      for (int s = 0; s < hn[i]; ++s) pr.push_back({hp[(size_t)i * kMaxNear + s], i, s});
    std::sort(pr.begin(), pr.end());
    for (const auto& e : pr) {
      std::vector<int>& l = h_close[(size_t)e[1] * kMaxNear + e[2]] ? nl2 : nl;
      l.push_back(e[1]);
      l.push_back(e[0]);
      l.push_back(e[2]);
    }
  }
  centers.swap(cn);
  has_axes = ax != nullptr;
  axes.swap(axn);
  h_partners.swap(hp);
  h_npart.swap(hn);
  max_slots = slots;
  n_near = (int)nl.size() / 3;
  n_near2 = (int)nl2.size() / 3;
  ctr.upload(centers.data(), centers.size(), stream);
  dax.upload(axes.data(), axes.size(), stream);
  cls.upload(hc.data(), hc.size(), stream);
  partners.upload(h_partners.data(), h_partners.size(), stream);
  npart.upload(h_npart.data(), h_npart.size(), stream);
  near_list.upload(nl.data(), nl.size(), stream);
  near_list2.upload(nl2.data(), nl2.size(), stream);
  HIPCHK(hipStreamSynchronize(stream));
  ++config_epoch;
}

void pqn_ctx_impl::stage_begin(int st) {
  if (!cfg.profile) return;
  auto& pool = ev_pool[st];
  if (ev_used[st] == pool.size()) {
    hipEvent_t a0, b0;
    HIPCHK(hipEventCreate(&a0));
    HIPCHK(hipEventCreate(&b0));
    pool.emplace_back(a0, b0);
  }
  HIPCHK(hipEventRecord(pool[ev_used[st]].first, stream));
}

void pqn_ctx_impl::stage_end(int st) {
  if (!cfg.profile) return;
  HIPCHK(hipEventRecord(ev_pool[st][ev_used[st]].second, stream));
  ++ev_used[st];
}

void pqn_ctx_impl::begin_far_timing() { stage_begin(kStageFar); }

void pqn_ctx_impl::end_far_launch() { stage_end(kStageFar); }

double pqn_ctx_impl::end_far_timing() {
  // called after the stream has been synchronised: sums and recycles the events of every stage
  for (int st = 0; st < kNumStages; ++st) {
    double t = 0.0;
    for (size_t k = 0; k < ev_used[st]; ++k) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, ev_pool[st][k].first, ev_pool[st][k].second));
      t += ms;
    }
    ev_used[st] = 0;
    stage_ms[st] = t;
  }
  return stage_ms[kStageFar];
}

// y_r = (1/2 I + D + P) q_r for every density of every group.
void add_to_groups(std::vector<MvGroup>& groups, pqn_ctx_impl* c, Level* lv, int slot, const double* in,
                   double* out) {
  MvGroup* g = nullptr;
  for (MvGroup& gg : groups)
    if (gg.c == c && gg.lv == lv) g = &gg;
  if (!g) {
    groups.push_back(MvGroup{c, lv, 0, {}, {}, {}});
    g = &groups.back();
  }
  if (g->K >= kMaxRhs) throw Error(PQN_ERR_STATE, "more than 6 densities on one level in one pass");
  g->slot[g->K] = slot;
  g->in[g->K] = in;
  g->out[g->K] = out;
  ++g->K;
}

// The interleaved upsampled densities of a group: [M][nup][3K] in the work
// buffer of the group's first slot (grown on first use with more densities).
double* group_qup(MvGroup& gr, bool close) {
  Level& lv = *gr.lv;
  Work& w0 = lv.wk(gr.slot[0]);
  DevArray<double>& buf = close ? w0.qup2 : w0.qup;
  const size_t need = (size_t)3 * gr.K * lv.M * (close ? lv.nup2 : lv.nup);
  if (buf.count < need) {
    HIPCHK(hipDeviceSynchronize());  // the old buffer may still be read by queued work
    buf.alloc(need);
  }
  return buf.p;
}

// Harmonic coefficients of a group's K densities, [M][3K][L] (row 3r + c: density r,
// component c), in the work buffer of the group's first slot (grown on first use with
// more densities).
// Degree-truncated densities of a group on the coarse far-source grid, [M][nc][3K].
static double* group_qc(MvGroup& gr) {
  Level& lv = *gr.lv;
  DevArray<double>& buf = lv.wk(gr.slot[0]).qc;
  const size_t need = (size_t)3 * gr.K * lv.M * lv.nc;
  if (buf.count < need) {
    HIPCHK(hipDeviceSynchronize());  // the old buffer may still be read by queued work
    buf.alloc(need);
  }
  return buf.p;
}

double* group_coef(MvGroup& gr) {
  Level& lv = *gr.lv;
  DevArray<double>& buf = lv.wk(gr.slot[0]).coef;
  const size_t need = (size_t)3 * gr.K * lv.M * lv.L;
  if (buf.count < need) {
    HIPCHK(hipDeviceSynchronize());  // the old buffer may still be read by queued work
    buf.alloc(need);
  }
  return buf.p;
}

// The GEMMs of one group's densities (slot r of density r, input in[r]): coefficients
// coef = T q into the group's [M][3K][L] buffer (coefficient GEMM list ga); the singular
// self interaction on them, one partial per source component, and the densities on the
// upsampled grids (one GEMM per grid for all 3K components, stored node-interleaved
// [M][nup][3K] so that consecutive columns are consecutive addresses) (list gb).
void push_group_gemms(Level& lv, int K, const int* slot, const double* const* in, double* coef, double* qup,
                      double* qup2, const int* live_flag, std::vector<GemmDesc>& ga, int& nga,
                      std::vector<GemmDesc>& gb, int& ngb, bool with_self) {
  const int n = lv.n, N = lv.N, L = lv.L, M = lv.M, C = 3 * K;
  const size_t a0 = ga.size(), b0 = gb.size();
  for (int r = 0; r < K; ++r) {
    Work& w = lv.wk(slot[r]);
    for (int comp = 0; comp < 3; ++comp) {
      double* cb = coef + (size_t)(3 * r + comp) * L;
      push_gemm(ga, nga, L, M, n, lv.T.p, n, in[r] + (size_t)comp * N, n, cb, L, 0, C * L);
      if (with_self)
        push_gemm(gb, ngb, 3 * n, M, L, lv.G.p + comp * L, 3 * L, cb, C * L, w.selfo.p + (size_t)comp * 3 * N, n,
                  N, n);
    }
  }
  if (qup) push_gemm(gb, ngb, lv.nup, C * M, L, lv.Yup.p, L, coef, L, qup, lv.nup, 0, 1, C, C, (long)lv.nup * C);
  if (qup2)
    push_gemm(gb, ngb, lv.nup2, C * M, L, lv.Yup2.p, L, coef, L, qup2, lv.nup2, 0, 1, C, C, (long)lv.nup2 * C);
  for (size_t e = a0; e < ga.size(); ++e) ga[e].live = live_flag;
  for (size_t e = b0; e < gb.size(); ++e) gb[e].live = live_flag;
}

void pqn_ctx_impl::matvec_groups(std::vector<MvGroup>& groups, int precision) {
  hipStream_t s = stream;
  const int prec = precision == PQN_MIXED ? 1 : 0;
  for (size_t a = 0; a < groups.size(); ++a)
    for (size_t b = a + 1; b < groups.size(); ++b)
      if (groups[a].lv == groups[b].lv) throw Error(PQN_ERR_STATE, "internal: two density groups on one level");
  bool all_single = groups.size() > 1;
  for (MvGroup& gr : groups)
    if (gr.K != 1) all_single = false;
  if (all_single) {
    matvec_batched(groups, prec);
    return;
  }
  // One group, side_stream on: the coefficient and self-interaction GEMMs, the
  // near tiles and the rigid moments (none of which the far pair sum reads) run
  // on a second stream, concurrently with the packing and far pair sum; the
  // final combination waits for both.
  // With a coarse far-source grid the far sources come from the coefficients: the
  // coefficient and coarse-synthesis GEMMs then run on the main stream before the fork.
  const bool ov = cfg.side_stream && !cfg.profile && groups.size() == 1;
  hipStream_t sa = ov ? side_stream() : s;
  bool forked = false;
  auto fork = [&]() {
    if (ov && !forked) {
      HIPCHK(hipEventRecord(ev_in, s));
      HIPCHK(hipStreamWaitEvent(sa, ev_in, 0));
      forked = true;
    }
  };
  for (MvGroup& gr : groups) {
    Level& lv = *gr.lv;
    pqn_ctx_impl& c = *gr.c;
    const int n = lv.n, N = lv.N, C = 3 * gr.K;
    QPtrs qp{};
    std::vector<GemmDesc> ga, gb, gc;
    int nga = 0, ngb = 0, ngc = 0;
    double* qup = c.n_near > 0 ? group_qup(gr) : nullptr;
    double* qup2 = c.n_near2 > 0 ? group_qup(gr, true) : nullptr;
    double* coef = group_coef(gr);
    double* qc = lv.nc > 0 ? group_qc(gr) : nullptr;
    push_group_gemms(lv, gr.K, gr.slot, gr.in, coef, qup, qup2, nullptr, ga, nga, gb, ngb);
    if (qc)  // densities truncated to the coarse grid's degree, synthesised on it: [M][nc][3K]
      push_gemm(gc, ngc, lv.nc, C * lv.M, lv.Lc, lv.Yc.p, lv.Lc, coef, lv.L, qc, lv.nc, 0, 1, C, C, (long)lv.nc * C);
    for (int r = 0; r < gr.K; ++r) qp.p[r] = gr.in[r];
    DescPack dp;
    const size_t oa = dp.add(ga), ob = dp.add(gb), oc = dp.add(gc);
    stage_begin(kStageGemm);
    if (qc) {
      char* base = push_desc_pack(dp.host);  // main stream (read by the side stream after the fork)
      launch_gemm64_multi(s, (const GemmDesc*)(base + oa), (int)ga.size(), nga);
      launch_gemm64_multi(s, (const GemmDesc*)(base + oc), (int)gc.size(), ngc);
      fork();
      launch_gemm64_multi(sa, (const GemmDesc*)(base + ob), (int)gb.size(), ngb);
    } else {
      fork();
      char* base = ov ? push_desc_pack(dp.host, sa, ddesc_side) : push_desc_pack(dp.host);
      launch_gemm64_multi(sa, (const GemmDesc*)(base + oa), (int)ga.size(), nga);
      launch_gemm64_multi(sa, (const GemmDesc*)(base + ob), (int)gb.size(), ngb);
    }
    stage_end(kStageGemm);
    if (ov) side_work(gr, sa);
    stage_begin(kStageLocal);
    if (qc)
      launch_pack_coarse(s, prec, gr.K, qc, lv.offc.p, lv.wc.p, lv.nc, lv.M * lv.nc, lv.src.p);
    else
      launch_pack(s, prec, gr.K, qp, lv.off.p, lv.w.p, n, N, lv.src.p);
    stage_end(kStageLocal);
  }
  begin_far_timing();
  const int kf = groups.size() == 1 ? groups[0].K : 0;  // one group: its launches are also timed by K
  if (kf) stage_begin(kStageFarK + kf - 1);
  {
    for (MvGroup& gr : groups) {
      Level& lv = *gr.lv;
      OPtrs op{};
      for (int r = 0; r < gr.K; ++r) op.p[r] = lv.wk(gr.slot[r]).far_part.p;
      launch_far(s, prec, gr.K, lv.tpt, lv.src.p, lv.off.p, gr.c->ctr.p, gr.c->cls.p, lv.n, lv.nc > 0 ? lv.nc : lv.n,
                 lv.M, lv.N, lv.spc, lv.nchunks, 3.0 / (4.0 * kPi * gr.c->a), op);
    }
  }
  if (kf) {
    stage_end(kStageFarK + kf - 1);
    ++n_far_k[kf - 1];
  }
  end_far_launch();
  ++n_far;
  if (ov) {
    HIPCHK(hipEventRecord(ev_side, sa));
    HIPCHK(hipStreamWaitEvent(s, ev_side, 0));
  }
  for (MvGroup& gr : groups) {
    Level& lv = *gr.lv;
    pqn_ctx_impl& c = *gr.c;
    if (!ov) side_work(gr, s);
    stage_begin(kStageLocal);
    if (gr.K == 1) {
      Work& w = lv.wk(gr.slot[0]);
      launch_combine(s, gr.in[0], w.selfo.p, 3, w.far_part.p, lv.nchunks, w.near_part.p, c.npart.p, w.mom.p,
                     lv.off.p, lv.n, lv.N, c.a, gr.out[0]);
    } else {
      // the final combination of all K densities, one launch
      std::vector<CombDesc> cd;
      int ncd = 0;
      for (int r = 0; r < gr.K; ++r) {
        Work& w = lv.wk(gr.slot[r]);
        cd.push_back(CombDesc{gr.in[r], w.selfo.p, w.far_part.p, w.near_part.p, c.npart.p, w.mom.p, lv.off.p,
                              gr.out[r], c.a, lv.nchunks, lv.n, lv.N, ncd});
        ncd += 3 * lv.N;
      }
      DescPack dp;
      const size_t oc = dp.add(cd);
      char* base = push_desc_pack(dp.host);
      launch_combine_multi(s, (const CombDesc*)(base + oc), (int)cd.size(), ncd);
    }
    stage_end(kStageLocal);
    n_matvec += gr.K;
  }
  HIPCHK(hipGetLastError());
}

// Near tiles and rigid moments of one group on stream st (after its GEMMs on st).
void pqn_ctx_impl::side_work(MvGroup& gr, hipStream_t st) {
  Level& lv = *gr.lv;
  pqn_ctx_impl& c = *gr.c;
  OPtrs np{};
  for (int r = 0; r < gr.K; ++r) np.p[r] = lv.wk(gr.slot[r]).near_part.p;
  const double* cf = lv.wk(gr.slot[0]).coef.p;  // the group's [M][3K][L] coefficients
  const double* qup = lv.wk(gr.slot[0]).qup.p;
  // (stage events are recorded only while profiling, when st is the main stream)
  stage_begin(kStageNear);
  launch_near(st, gr.K, c.n_near, c.ctr.p, lv.off.p, lv.offup.p, lv.shab.p, qup, cf, c.near_list.p, lv.n, lv.M, lv.N,
              lv.nup, lv.p, lv.L, 3.0 / (4.0 * kPi * c.a), np);
  launch_near(st, gr.K, c.n_near2, c.ctr.p, lv.off.p, lv.offup2.p, lv.shab.p, lv.wk(gr.slot[0]).qup2.p, cf,
              c.near_list2.p, lv.n, lv.M, lv.N, lv.nup2, lv.p, lv.L, 3.0 / (4.0 * kPi * c.a), np);
  stage_end(kStageNear);
  stage_begin(kStageLocal);
  if (gr.K == 1) {
    Work& w = lv.wk(gr.slot[0]);
    launch_moments(st, gr.in[0], lv.off.p, lv.w.p, lv.n, lv.M, lv.N, w.mom.p);
  } else {
    std::vector<MomDesc> md;
    int nmd = 0;
    for (int r = 0; r < gr.K; ++r) {
      Work& w = lv.wk(gr.slot[r]);
      md.push_back(MomDesc{gr.in[r], lv.off.p, lv.w.p, w.mom.p, lv.n, lv.N, nmd});
      nmd += lv.M;
    }
    // own descriptor table per stream; on the main stream it follows the GEMMs' use of it
    DescPack dp;
    const size_t om = dp.add(md);
    char* base = st == stream ? push_desc_pack(dp.host) : push_desc_pack(dp.host, st, ddesc_side);
    launch_moments_multi(st, (const MomDesc*)(base + om), (int)md.size(), nmd);
  }
  stage_end(kStageLocal);
}

// Segment tables of one operator application to many suspensions (one density
// each), appended to dp: every phase is one segmented launch over all of them.
// live[g] (may be empty) is the flag of group g's system (graph-captured GMRES).
BatchOpTables pqn_ctx_impl::batch_op_tables(std::vector<MvGroup>& groups, int prec, const std::vector<const int*>& live,
                                            DescPack& dp) {
  std::vector<GemmDesc> ga, gb;
  std::vector<PackDesc> pk;
  std::vector<NearDesc> nd;
  std::vector<MomDesc> md;
  std::vector<CombDesc> cd;
  BatchOpTables t{};
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    MvGroup& gr = groups[gi];
    const int* lf = live.empty() ? nullptr : live[gi];
    Level& lv = *gr.lv;
    pqn_ctx_impl& c = *gr.c;
    Work& w = lv.wk(gr.slot[0]);
    const int n = lv.n, N = lv.N, L = lv.L, nup = lv.nup, M = lv.M;
    push_group_gemms(lv, 1, gr.slot, gr.in, w.coef.p, c.n_near > 0 ? w.qup.p : nullptr,
                     c.n_near2 > 0 ? w.qup2.p : nullptr, lf, ga, t.nga, gb, t.ngb);
    pk.push_back(PackDesc{gr.in[0], lv.off.p, lv.w.p, lv.src.p, n, N, t.npk, lf});
    t.npk += N;
    if (c.n_near > 0) {
      const int nch = (n + 63) / 64;
      nd.push_back(NearDesc{c.ctr.p, lv.off.p, lv.offup.p, lv.shab.p, w.qup.p, w.coef.p, c.near_list.p, w.near_part.p,
                            3.0 / (4.0 * kPi * c.a), n, M, N, nup, lv.p, L, nch, t.nnd, lf});
      t.nnd += c.n_near * nch;
    }
    if (c.n_near2 > 0) {
      const int nch = (n + 63) / 64;
      nd.push_back(NearDesc{c.ctr.p, lv.off.p, lv.offup2.p, lv.shab.p, w.qup2.p, w.coef.p, c.near_list2.p,
                            w.near_part.p, 3.0 / (4.0 * kPi * c.a), n, M, N, lv.nup2, lv.p, L, nch, t.nnd, lf});
      t.nnd += c.n_near2 * nch;
    }
    md.push_back(MomDesc{gr.in[0], lv.off.p, lv.w.p, w.mom.p, n, N, t.nmd, lf});
    t.nmd += M;
    cd.push_back(CombDesc{gr.in[0], w.selfo.p, w.far_part.p, w.near_part.p, c.npart.p, w.mom.p, lv.off.p, gr.out[0],
                          c.a, lv.nchunks, n, N, t.ncd, lf});
    t.ncd += 3 * N;
  }
  // far pair sums of all suspensions in one launch, work items by decreasing cost
  struct Item {
    FarDesc d;
    long cost;
  };
  std::vector<Item> items;
  const int tpt = far_layout(cfg);
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    MvGroup& gr = groups[gi];
    Level& lv = *gr.lv;
    FarDesc d{};
    d.src = lv.src.p;
    d.off = lv.off.p;
    d.ctr = gr.c->ctr.p;
    d.cls = gr.c->cls.p;
    d.part = lv.wk(gr.slot[0]).far_part.p;
    d.n = lv.n;
    d.M = lv.M;
    d.N = lv.N;
    d.spc = lv.spc;
    const int per_block = prec == 1 ? (tpt == 0 ? 64 : 256 * tpt) : 256;
    d.ntb = (lv.N + per_block - 1) / per_block;
    d.scale = 3.0 / (4.0 * kPi * gr.c->a);
    d.live = live.empty() ? nullptr : live[gi];
    items.push_back({d, (long)lv.n * lv.n * lv.spc});
  }
  std::stable_sort(items.begin(), items.end(), [](const Item& x, const Item& y) { return x.cost > y.cost; });
  std::vector<FarDesc> fd;
  for (Item& it : items) {
    it.d.item0 = t.nfar;
    t.nfar += it.d.ntb * ((it.d.M + it.d.spc - 1) / it.d.spc);
    fd.push_back(it.d);
  }
  t.na = (int)ga.size();
  t.nb = (int)gb.size();
  t.npk_n = (int)pk.size();
  t.nnd_n = (int)nd.size();
  t.nmd_n = (int)md.size();
  t.ncd_n = (int)cd.size();
  t.nfd = (int)fd.size();
  t.oa = dp.add(ga);
  t.ob = dp.add(gb);
  t.op = dp.add(pk);
  t.on = dp.add(nd);
  t.om = dp.add(md);
  t.oc = dp.add(cd);
  t.of = dp.add(fd);
  return t;
}

// Kernel launches of one batched operator application from uploaded tables (no copies
// or fills: capturable). side_stream: GEMMs, near tiles and moments on the second stream,
// forked and joined by events, beside the packing and far pair sums.
void pqn_ctx_impl::batch_op_launch(const char* base, const BatchOpTables& t, int prec) {
  hipStream_t s = stream;
  const bool ov = cfg.side_stream && !cfg.profile;
  hipStream_t sa = s;
  if (ov) {
    sa = side_stream();
    HIPCHK(hipEventRecord(ev_in, s));
    HIPCHK(hipStreamWaitEvent(sa, ev_in, 0));
  }
  stage_begin(kStageGemm);
  launch_gemm64_multi(sa, (const GemmDesc*)(base + t.oa), t.na, t.nga);  // coef = T q
  launch_gemm64_multi(sa, (const GemmDesc*)(base + t.ob), t.nb, t.ngb);  // self, qup
  stage_end(kStageGemm);
  if (ov) {
    if (t.nnd_n > 0) launch_near_multi(sa, (const NearDesc*)(base + t.on), t.nnd_n, t.nnd);
    launch_moments_multi(sa, (const MomDesc*)(base + t.om), t.nmd_n, t.nmd);
    HIPCHK(hipEventRecord(ev_side, sa));
  }
  stage_begin(kStageLocal);
  launch_pack_multi(s, (const PackDesc*)(base + t.op), t.npk_n, t.npk, prec);
  stage_end(kStageLocal);
  begin_far_timing();
  launch_far_multi(s, prec, far_layout(cfg), (const FarDesc*)(base + t.of), t.nfd, t.nfar);
  end_far_launch();
  ++n_far;
  if (ov) {
    HIPCHK(hipStreamWaitEvent(s, ev_side, 0));
  } else {
    stage_begin(kStageNear);
    if (t.nnd_n > 0) launch_near_multi(s, (const NearDesc*)(base + t.on), t.nnd_n, t.nnd);
    stage_end(kStageNear);
    stage_begin(kStageLocal);
    launch_moments_multi(s, (const MomDesc*)(base + t.om), t.nmd_n, t.nmd);
    stage_end(kStageLocal);
  }
  stage_begin(kStageLocal);
  launch_combine_multi(s, (const CombDesc*)(base + t.oc), t.ncd_n, t.ncd);
  stage_end(kStageLocal);
}

// Many suspensions (one density each): every phase of the operator is one
// segmented launch over all of them.
void pqn_ctx_impl::matvec_batched(std::vector<MvGroup>& groups, int prec) {
  DescPack dp;
  const BatchOpTables t = batch_op_tables(groups, prec, {}, dp);
  // (the table is read by both streams and rewritten only after the join)
  const char* base = push_desc_pack(dp.host);
  batch_op_launch(base, t, prec);
  n_matvec += (int)groups.size();
  HIPCHK(hipGetLastError());
}

void pqn_ctx_impl::apply_operator(Level& lv, int precision, const double* q, double* y) {
  std::vector<MvGroup> g;
  add_to_groups(g, this, &lv, 0, q, y);
  matvec_groups(g, precision);
}

double pqn_ctx_impl::dot_host(const double* x, const double* y, long len, Level& lv) {
  SysBuf& b = lv.sb(0);
  hdev.alloc(4);
  launch_dots(stream, x, len, 1, y, len, lv.nb_dots, b.partial.p, hdev.p);
  double v = 0.0;
  HIPCHK(hipMemcpyAsync(&v, hdev.p, sizeof(double), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  return v;
}

// Descriptor tables of the two segmented GEMM phases of one operator
// application to the single density q (context c, level lv, work slot).
IterTables pqn_ctx_impl::iteration_tables(pqn_ctx_impl& c, Level& lv, int slot, const double* q,
                                           std::vector<char>& bytes) {
  Work& w = lv.wk(slot);
  const int n = lv.n, N = lv.N, L = lv.L, nup = lv.nup, M = lv.M;
  std::vector<GemmDesc> ga, gb;
  IterTables t{};
  const double* in[1] = {q};
  push_group_gemms(lv, 1, &slot, in, w.coef.p, c.n_near > 0 ? w.qup.p : nullptr, c.n_near2 > 0 ? w.qup2.p : nullptr,
                   nullptr, ga, t.nga, gb, t.ngb);
  DescPack dp;
  t.oa = dp.add(ga);
  t.ob = dp.add(gb);
  t.na = (int)ga.size();
  t.nb = (int)gb.size();
  bytes = dp.host;
  return t;
}

// Kernels of one GMRES iteration on one system: w = A q, then two classical
// Gram-Schmidt passes against V[0..nvec) and the squared norm of w, with every
// Hessenberg entry written to hp. Kernel launches only (no copies or fills),
// so the sequence can be captured in a graph.
void pqn_ctx_impl::iteration_launches(pqn_ctx_impl& c, Level& lv, int slot, int prec, const double* q, double* w,
                                      const double* V, int nvec, double* hp, int m, const char* dtab,
                                      const IterTables& t) {
  hipStream_t s = stream;
  Work& wk = lv.wk(slot);
  SysBuf& b = lv.sb(slot);
  const long len = 3L * lv.N;
  const double scale = 3.0 / (4.0 * kPi * c.a);
  launch_gemm64_multi(s, (const GemmDesc*)(dtab + t.oa), t.na, t.nga);
  launch_gemm64_multi(s, (const GemmDesc*)(dtab + t.ob), t.nb, t.ngb);
  QPtrs qp{};
  qp.p[0] = q;
  launch_pack(s, prec, 1, qp, lv.off.p, lv.w.p, lv.n, lv.N, lv.src.p);
  OPtrs op{};
  op.p[0] = wk.far_part.p;
  launch_far(s, prec, 1, lv.tpt, lv.src.p, lv.off.p, c.ctr.p, c.cls.p, lv.n, lv.n, lv.M, lv.N, lv.spc, lv.nchunks, scale,
             op);
  OPtrs np{};
  np.p[0] = wk.near_part.p;
  launch_near(s, 1, c.n_near, c.ctr.p, lv.off.p, lv.offup.p, lv.shab.p, wk.qup.p, wk.coef.p, c.near_list.p, lv.n, lv.M,
              lv.N, lv.nup, lv.p, lv.L, scale, np);
  launch_near(s, 1, c.n_near2, c.ctr.p, lv.off.p, lv.offup2.p, lv.shab.p, wk.qup2.p, wk.coef.p, c.near_list2.p, lv.n,
              lv.M, lv.N, lv.nup2, lv.p, lv.L, scale, np);
  launch_moments(s, q, lv.off.p, lv.w.p, lv.n, lv.M, lv.N, wk.mom.p);
  launch_combine(s, q, wk.selfo.p, 3, wk.far_part.p, lv.nchunks, wk.near_part.p, c.npart.p, wk.mom.p, lv.off.p, lv.n,
                 lv.N, c.a, w);
  for (int pass = 0; pass < 2; ++pass) {
    launch_dots(s, V, len, nvec, w, len, lv.nb_dots, b.partial.p, hp + pass * (m + 1));
    launch_combo(s, w, 1.0, V, len, nvec, hp + pass * (m + 1), -1.0, len);
  }
  launch_dots(s, w, len, 1, w, len, lv.nb_dots, b.partial.p, hp + 2 * (m + 1));
}

// Replay the graph of GMRES iteration k of one system, capturing it on first
// use. Graphs hold device pointers of the level's buffers and the context's
// geometry, so they are rebuilt after any configuration change.
void pqn_ctx_impl::launch_iteration_graph(pqn_ctx_impl& c, Level& lv, int slot, int prec, int k, double* hp, int m) {
  while ((int)lv.graphs.size() <= slot) lv.graphs.emplace_back(new GraphCache());
  GraphCache& gc = *lv.graphs[slot];
  const double* qup_now = lv.wk(slot).qup.p;  // may move when a wider group grows it
  const double* qup2_now = lv.wk(slot).qup2.p;
  if (gc.epoch != c.config_epoch || gc.prec != prec || (int)gc.execs.size() != m || gc.hp != hp ||
      gc.qup != qup_now || gc.qup2 != qup2_now) {
    HIPCHK(hipStreamSynchronize(stream));
    gc.clear();
    gc.execs.assign(m, nullptr);
    gc.epoch = c.config_epoch;
    gc.prec = prec;
    gc.hp = hp;
    gc.qup = qup_now;
    gc.qup2 = qup2_now;
  }
  SysBuf& b = lv.sb(slot);
  const long len = 3L * lv.N;
  const double* q = b.V.p + (size_t)k * len;
  double* w = b.V.p + (size_t)(k + 1) * len;
  if (!gc.execs[k]) {
    std::vector<char> bytes;
    const IterTables t = iteration_tables(c, lv, slot, q, bytes);
    const size_t stride = (bytes.size() + 255) & ~size_t(255);
    if (!gc.dtab.p || gc.stride < stride) {
      // every cached graph points into the old table: drop them all
      HIPCHK(hipStreamSynchronize(stream));
      gc.clear();
      gc.execs.assign(m, nullptr);
      gc.stride = stride;
      gc.dtab.release();
      gc.dtab.alloc(gc.stride * m);
    }
    char* tab = gc.dtab.p + gc.stride * k;
    HIPCHK(hipMemcpyAsync(tab, bytes.data(), bytes.size(), hipMemcpyHostToDevice, stream));
    HIPCHK(hipStreamSynchronize(stream));
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    iteration_launches(c, lv, slot, prec, q, w, b.V.p, k + 1, hp, m, tab, t);
    const hipError_t ce = hipStreamEndCapture(stream, &graph);
    HIPCHK(ce);
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIPCHK(ie);
    gc.execs[k] = exec;
  }
  HIPCHK(hipGraphLaunch(gc.execs[k], stream));
  ++n_graph_launch;
  ++n_far;
  ++n_matvec;
}

namespace {
struct GmState {
  std::vector<double> H, cs, sn, g;
  double bnorm = 0.0;
  int k = 0;
  bool active = false, restart = false;
};
}  // namespace

void pqn_ctx_impl::gmres_lockstep(std::vector<SysRef>& sys, int precision) {
  bool graph = is_batch && cfg.use_graphs && !cfg.profile && sys.size() > 1 && precision == cfg.precision;
  for (SysRef& r : sys) graph = graph && !r.x0 && !r.res_out && !r.c->cfg.precond;
  if (graph)
    gmres_batch_graph(sys, precision);
  else
    gmres_lockstep_eager(sys, precision);
}

// Descriptor tables of Arnoldi index j for every system (operator on V[j] -> V[j+1],
// CGS2 against V[0..j], |w|^2, the Givens step and the normalisation of V[j+1]),
// uploaded once, then the launches captured into graph j.
void pqn_ctx_impl::capture_batch_iteration(BatchGraph& bg, std::vector<SysRef>& sys, int j, int prec) {
  const int ns = (int)sys.size(), m = bg.m;
  const int hs = 2 * (m + 1) + 2;
  std::vector<MvGroup> groups;
  std::vector<const int*> live;
  for (int i = 0; i < ns; ++i) {
    SysBuf& b = sys[i].lv->sb(sys[i].slot);
    const size_t len = 3 * (size_t)sys[i].lv->N;
    add_to_groups(groups, sys[i].c, sys[i].lv, sys[i].slot, b.V.p + (size_t)j * len, b.V.p + (size_t)(j + 1) * len);
    live.push_back(&bg.sys.p[i].active);
  }
  if ((int)groups.size() != ns) throw Error(PQN_ERR_STATE, "internal: batched systems must be on distinct levels");
  DescPack dp;
  const BatchOpTables t = batch_op_tables(groups, prec, live, dp);
  std::vector<DotDesc> dd[2], dn;
  std::vector<ComboDesc> cd[2];
  std::vector<ScaleDesc> sc;
  int nv[2] = {0, 0}, nn = 0, ne[2] = {0, 0}, nsc = 0;
  for (int i = 0; i < ns; ++i) {
    SysBuf& b = sys[i].lv->sb(sys[i].slot);
    const long len = 3L * sys[i].lv->N;
    double* w = b.V.p + (size_t)(j + 1) * len;
    double* hp = bg.hbuf.p + (size_t)i * hs;
    for (int pass = 0; pass < 2; ++pass) {
      dd[pass].push_back(DotDesc{b.V.p, w, b.partial.p, hp + pass * (m + 1), len, len, nv[pass], live[i]});
      nv[pass] += j + 1;
      cd[pass].push_back(ComboDesc{w, b.V.p, hp + pass * (m + 1), -1.0, 1.0, len, len, j + 1, ne[pass], live[i]});
      ne[pass] += (int)len;
    }
    dn.push_back(DotDesc{w, w, b.partial.p, hp + 2 * (m + 1), len, len, nn, live[i]});
    nn += 1;
    sc.push_back(ScaleDesc{w, &bg.sys.p[i].inv_hn, live[i], len, nsc});
    nsc += (int)len;
  }
  const size_t o0 = dp.add(dd[0]), o1 = dp.add(cd[0]), o2 = dp.add(dd[1]), o3 = dp.add(cd[1]), o4 = dp.add(dn),
               o5 = dp.add(sc);
  const size_t need = (dp.host.size() + 255) & ~size_t(255);
  if (!bg.tabs.p || need > bg.stride) {
    // every graph captured so far points into the old tables: drop them all
    HIPCHK(hipStreamSynchronize(stream));
    bg.clear();
    bg.execs.assign(m, nullptr);
    bg.stride = need;
    bg.tabs.release();
    bg.tabs.alloc(bg.stride * m);
  }
  char* base = bg.tabs.p + bg.stride * j;
  HIPCHK(hipMemcpyAsync(base, dp.host.data(), dp.host.size(), hipMemcpyHostToDevice, stream));
  HIPCHK(hipStreamSynchronize(stream));
  const int nfar0 = n_far;
  hipGraph_t graph = nullptr;
  HIPCHK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
  try {
    batch_op_launch(base, t, prec);
    launch_dots_multi(stream, (const DotDesc*)(base + o0), ns, nv[0], kMultiDotBlocks);
    launch_combo_multi(stream, (const ComboDesc*)(base + o1), ns, ne[0]);
    launch_dots_multi(stream, (const DotDesc*)(base + o2), ns, nv[1], kMultiDotBlocks);
    launch_combo_multi(stream, (const ComboDesc*)(base + o3), ns, ne[1]);
    launch_dots_multi(stream, (const DotDesc*)(base + o4), ns, nn, kMultiDotBlocks);
    launch_gmres_step(stream, bg.sys.p, bg.hess.p, bg.hbuf.p, hs, m, ns);
    launch_scale_multi(stream, (const ScaleDesc*)(base + o5), ns, nsc);
  } catch (...) {
    hipGraph_t g2 = nullptr;
    (void)hipStreamEndCapture(stream, &g2);
    if (g2) (void)hipGraphDestroy(g2);
    n_far = nfar0;
    throw;
  }
  n_far = nfar0;
  HIPCHK(hipStreamEndCapture(stream, &graph));
  hipGraphExec_t exec = nullptr;
  const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  HIPCHK(ie);
  bg.execs[j] = exec;
}

// First GMRES(m) cycle of many cold-started systems from captured graphs: all systems
// take Arnoldi step j together (graph j); the Givens rotations and the end test run on
// the device, so the host reads the state back only every 8 steps to stop early. The
// cycle's end (x += V y) is done from the read-back Hessenberg matrices; systems whose
// cycle filled continue in the eager lockstep loop from their iterate.
void pqn_ctx_impl::gmres_batch_graph(std::vector<SysRef>& sys, int precision) {
  const int ns = (int)sys.size();
  const int m = sys[0].lv->restart;
  for (SysRef& r : sys)
    if (r.lv->restart != m) throw Error(PQN_ERR_STATE, "internal: batched systems with different restart lengths");
  const int prec = precision == PQN_MIXED ? 1 : 0;
  const int hs = 2 * (m + 1) + 2;
  hipStream_t s = stream;
  std::vector<const void*> key;
  for (SysRef& r : sys) {
    key.push_back(r.c);
    key.push_back(r.lv);
    key.push_back(reinterpret_cast<const void*>(static_cast<intptr_t>(r.slot)));
    r.lv->wk(r.slot);  // every buffer exists before any capture
    r.lv->sb(r.slot);
  }
  if (cfg.side_stream) side_stream();  // created before any capture that forks onto it
  if (!bgraph) bgraph.reset(new BatchGraph());
  BatchGraph& bg = *bgraph;
  if (bg.key != key || bg.prec != prec || bg.m != m) {
    HIPCHK(hipStreamSynchronize(s));
    bg.clear();
    bg.key = key;
    bg.prec = prec;
    bg.m = m;
    bg.ns = ns;
    bg.execs.assign(m, nullptr);
    bg.sys.alloc(ns);
    bg.hess.alloc((size_t)ns * gm_stride(m));
    bg.hbuf.alloc((size_t)ns * hs);
  }
  // right-hand side norms
  for (int i = 0; i < ns; ++i) {
    SysBuf& b = sys[i].lv->sb(sys[i].slot);
    launch_dots(s, sys[i].rhs, 3L * sys[i].lv->N, 1, sys[i].rhs, 3L * sys[i].lv->N, sys[i].lv->nb_dots, b.partial.p,
                bg.hbuf.p + (size_t)i * hs + 2 * (m + 1));
  }
  std::vector<double> hb((size_t)ns * hs);
  HIPCHK(hipMemcpyAsync(hb.data(), bg.hbuf.p, hb.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<GmSys> hsys(ns);
  for (int i = 0; i < ns; ++i) {
    const long len = 3L * sys[i].lv->N;
    const double bn = std::sqrt(std::max(0.0, hb[(size_t)i * hs + 2 * (m + 1)]));
    if (!std::isfinite(bn)) throw Error(PQN_ERR_NUMERIC, "non-finite right-hand side");
    sys[i].its = 0;
    sys[i].relres = 0.0;
    sys[i].conv = bn == 0.0;
    launch_scale_copy(s, sys[i].x, sys[i].rhs, 0.0, len);  // x = 0
    GmSys g{};
    g.max_iter = sys[i].lv->max_iter;
    g.bnorm = bn;
    g.tol = sys[i].tol;
    if (bn > 0.0) {
      launch_scale_copy(s, sys[i].lv->sb(sys[i].slot).V.p, sys[i].rhs, 1.0 / bn, len);
      g.active = 1;
    }
    hsys[i] = g;
  }
  HIPCHK(hipMemcpyAsync(bg.sys.p, hsys.data(), ns * sizeof(GmSys), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  bool read_now = false;
  for (int j = 0; j < m; ++j) {
    TraceRange trace_iter("gmres_iteration_graph");
    if (!bg.execs[j]) capture_batch_iteration(bg, sys, j, prec);
    HIPCHK(hipGraphLaunch(bg.execs[j], s));
    ++n_graph_launch;
    ++n_far;
    read_now = j % 8 == 7 || j == m - 1;
    if (read_now) {
      HIPCHK(hipMemcpyAsync(hsys.data(), bg.sys.p, ns * sizeof(GmSys), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      bool any = false;
      for (const GmSys& g : hsys) any = any || g.active;
      if (!any) break;
    }
  }
  if (!read_now) {
    HIPCHK(hipMemcpyAsync(hsys.data(), bg.sys.p, ns * sizeof(GmSys), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  std::vector<double> hh((size_t)ns * gm_stride(m));
  HIPCHK(hipMemcpyAsync(hh.data(), bg.hess.p, hh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  // end of the cycle: y = R^{-1} g, x += V y
  std::vector<int> rest;
  std::vector<std::vector<double>> ys(ns);
  for (int i = 0; i < ns; ++i) {
    const GmSys& g = hsys[i];
    SysRef& sr = sys[i];
    if (g.bnorm == 0.0) continue;
    if (g.err) throw Error(PQN_ERR_NUMERIC, "non-finite value or breakdown in GMRES");
    if (g.active) throw Error(PQN_ERR_STATE, "internal: GMRES cycle still active after m steps");
    n_matvec += g.its;
    sr.its = g.its;
    sr.relres = g.relres;
    const double* H = hh.data() + (size_t)i * gm_stride(m);
    const double* gv = H + (size_t)(m + 1) * m + 2 * m;
    const int dk = g.k + 1;
    std::vector<double>& y = ys[i];
    y.assign(dk, 0.0);
    for (int r = dk - 1; r >= 0; --r) {
      double v = gv[r];
      for (int c2 = r + 1; c2 < dk; ++c2) v -= H[(size_t)r * m + c2] * y[c2];
      y[r] = v / H[(size_t)r * m + r];
    }
    SysBuf& b = sr.lv->sb(sr.slot);
    const long len = 3L * sr.lv->N;
    HIPCHK(hipMemcpyAsync(b.ycoef.p, y.data(), dk * sizeof(double), hipMemcpyHostToDevice, s));
    launch_combo(s, sr.x, 1.0, b.V.p, len, dk, b.ycoef.p, 1.0, len);
    if (g.conv) {
      sr.conv = true;
    } else if (g.its >= g.max_iter) {
      sr.conv = false;
    } else {
      rest.push_back(i);
    }
  }
  HIPCHK(hipStreamSynchronize(s));  // the y vectors leave scope only after their copies
  if (!rest.empty()) {
    // cycles that filled: continue from the iterate (the eager loop restarts from the true residual)
    std::vector<SysRef> sub;
    for (int i : rest) {
      SysRef r = sys[i];
      r.x0 = r.x;
      sub.push_back(r);
    }
    gmres_lockstep_eager(sub, precision);
    for (size_t k = 0; k < rest.size(); ++k) {
      SysRef& sr = sys[rest[k]];
      sr.its += sub[k].its;
      sr.relres = sub[k].relres;
      sr.conv = sub[k].conv;
    }
  }
}

// Restarted GMRES(m) on many systems in lockstep: every iteration applies the
// operator to all active systems at once (one joint launch of the pair sums)
// and reads back all Hessenberg columns in one copy. Per system: classical
// Gram-Schmidt with one reorthogonalisation (CGS2) in FP64 on the device,
// Givens rotations on the host; restarts from the true residual.
void pqn_ctx_impl::gmres_lockstep_eager(std::vector<SysRef>& sys, int precision) {
  const int ns = (int)sys.size();
  if (ns == 0) return;
  for (SysRef& r : sys) r.c->pc_prec = precision == PQN_MIXED ? 1 : 0;
  const int m = sys[0].lv->restart;
  const int hs = 2 * (m + 1) + 2;
  hdev.alloc((size_t)ns * hs);
  hhost.assign((size_t)ns * hs, 0.0);
  hipStream_t s = stream;
  std::vector<GmState> st(ns);
  auto len_of = [&](int i) { return 3L * sys[i].lv->N; };
  auto readback = [&]() {
    HIPCHK(hipMemcpyAsync(hhost.data(), hdev.p, (size_t)ns * hs * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  };
  auto nrm_slot = [&](int i) { return hdev.p + (size_t)i * hs + 2 * (m + 1); };
  // right preconditioning (config precond; whether this solve applies it was decided in
  // solve_lockstep): the Arnoldi vectors enter the operator as z = P V[k] and a cycle ends
  // with x += P (V y)
  std::vector<char> pcs(ns, 0);
  bool any_pc = false;
  for (int i = 0; i < ns; ++i) {
    Level& lv = *sys[i].lv;
    if (sys[i].c->cfg.precond && lv.pc.use && lv.pc.epoch == sys[i].c->config_epoch) {
      lv.sb(sys[i].slot).z.alloc((size_t)len_of(i));
      pcs[i] = 1;
      any_pc = true;
    }
  }
  // right-hand side norms
  for (int i = 0; i < ns; ++i) {
    SysBuf& b = sys[i].lv->sb(sys[i].slot);
    launch_dots(s, sys[i].rhs, len_of(i), 1, sys[i].rhs, len_of(i), sys[i].lv->nb_dots, b.partial.p, nrm_slot(i));
  }
  readback();
  auto start_cycle = [&](int i, const double* r0, double beta) {
    SysBuf& b = sys[i].lv->sb(sys[i].slot);
    launch_scale_copy(s, b.V.p, r0, 1.0 / beta, len_of(i));
    GmState& g = st[i];
    g.H.assign((size_t)(m + 1) * m, 0.0);
    g.cs.assign(m, 0.0);
    g.sn.assign(m, 0.0);
    g.g.assign(m + 1, 0.0);
    g.g[0] = beta;
    g.k = 0;
    g.active = true;
    g.restart = false;
  };
  // the final residual vector of a system that ends with its residual in v (res_out)
  auto residual_out = [&](int i, const double* v) {
    if (sys[i].res_out) launch_scale_copy(s, sys[i].res_out, v, 1.0, len_of(i));
  };
  std::vector<int> warm, given;  // initial guesses whose residual needs a product / is given
  for (int i = 0; i < ns; ++i) {
    const double bn = std::sqrt(std::max(0.0, hhost[(size_t)i * hs + 2 * (m + 1)]));
    if (!std::isfinite(bn)) throw Error(PQN_ERR_NUMERIC, "non-finite right-hand side");
    st[i].bnorm = bn;
    sys[i].its = 0;
    sys[i].relres = 0.0;
    sys[i].conv = true;
    if (bn > 0.0 && sys[i].x0) {
      launch_scale_copy(s, sys[i].x, sys[i].x0, 1.0, len_of(i));  // x = x0, residual below
      sys[i].conv = false;
      if (sys[i].r0) {
        SysBuf& b = sys[i].lv->sb(sys[i].slot);
        launch_scale_copy(s, b.r.p, sys[i].r0, 1.0, len_of(i));
        given.push_back(i);
      } else {
        warm.push_back(i);
      }
      continue;
    }
    launch_scale_copy(s, sys[i].x, sys[i].rhs, 0.0, len_of(i));  // x = 0 (rhs finite)
    if (bn > 0.0) {
      sys[i].conv = false;
      start_cycle(i, sys[i].rhs, bn);
    } else {
      residual_out(i, sys[i].rhs);  // zero
    }
  }
  auto build_groups = [&](const std::vector<int>& idx, bool use_x) {
    std::vector<MvGroup> groups;
    for (int i : idx) {
      SysBuf& b = sys[i].lv->sb(sys[i].slot);
      const double* in = use_x ? sys[i].x : pcs[i] ? b.z.p : b.V.p + (size_t)st[i].k * len_of(i);
      double* out = use_x ? b.r.p : b.V.p + (size_t)(st[i].k + 1) * len_of(i);
      add_to_groups(groups, sys[i].c, sys[i].lv, sys[i].slot, in, out);
    }
    return groups;
  };
  if (!warm.empty() || !given.empty()) {
    // initial residual r0 = rhs - A x0 of the warm-started systems (given, or by one product)
    if (!warm.empty()) {
      std::vector<MvGroup> wg = build_groups(warm, true);
      matvec_groups(wg, precision);
      for (int i : warm) {
        SysBuf& b = sys[i].lv->sb(sys[i].slot);
        launch_axpby(s, b.r.p, sys[i].rhs, 1.0, -1.0, len_of(i));
      }
    }
    warm.insert(warm.end(), given.begin(), given.end());
    for (int i : warm) {
      SysBuf& b = sys[i].lv->sb(sys[i].slot);
      launch_dots(s, b.r.p, len_of(i), 1, b.r.p, len_of(i), sys[i].lv->nb_dots, b.partial.p, nrm_slot(i));
    }
    readback();
    for (int i : warm) {
      SysBuf& b = sys[i].lv->sb(sys[i].slot);
      const double beta = std::sqrt(std::max(0.0, hhost[(size_t)i * hs + 2 * (m + 1)]));
      if (!std::isfinite(beta)) throw Error(PQN_ERR_NUMERIC, "non-finite initial residual");
      sys[i].relres = beta / st[i].bnorm;
      if (beta <= sys[i].tol * st[i].bnorm) {
        sys[i].conv = true;
        residual_out(i, b.r.p);
      } else {
        start_cycle(i, b.r.p, beta);
      }
    }
  }
  for (;;) {
    TraceRange trace_iter("gmres_iteration");
    std::vector<int> act;
    for (int i = 0; i < ns; ++i)
      if (st[i].active) act.push_back(i);
    if (act.empty()) break;
    const bool graph_iter = ns == 1 && cfg.use_graphs && !cfg.profile && sys[0].lv->nc == 0 && !any_pc;
    if (graph_iter) {
      const int i = act[0];
      launch_iteration_graph(*sys[i].c, *sys[i].lv, sys[i].slot, precision == PQN_MIXED ? 1 : 0, st[i].k,
                             hdev.p + (size_t)i * hs, m);
    } else {
      if (any_pc) {
        std::vector<MvGroup> pg;  // z = P V[k]
        for (int i : act)
          if (pcs[i]) {
            SysBuf& b = sys[i].lv->sb(sys[i].slot);
            add_to_groups(pg, sys[i].c, sys[i].lv, sys[i].slot, b.V.p + (size_t)st[i].k * len_of(i), b.z.p);
          }
        precond_apply_groups(pg);
      }
      std::vector<MvGroup> groups = build_groups(act, false);
      matvec_groups(groups, precision);
    }
    if (graph_iter) {
      // operator and CGS2 already in the replayed graph
    } else if (act.size() == 1) {
      stage_begin(kStageArnoldi);
      for (int i : act) {
        SysBuf& b = sys[i].lv->sb(sys[i].slot);
        const long len = len_of(i);
        const int k = st[i].k;
        double* w = b.V.p + (size_t)(k + 1) * len;
        double* hp = hdev.p + (size_t)i * hs;
        for (int pass = 0; pass < 2; ++pass) {
          launch_dots(s, b.V.p, len, k + 1, w, len, sys[i].lv->nb_dots, b.partial.p, hp + pass * (m + 1));
          launch_combo(s, w, 1.0, b.V.p, len, k + 1, hp + pass * (m + 1), -1.0, len);
        }
        launch_dots(s, w, len, 1, w, len, sys[i].lv->nb_dots, b.partial.p, hp + 2 * (m + 1));
      }
      stage_end(kStageArnoldi);
    } else {
      // CGS2 of every active system with segmented launches
      std::vector<DotDesc> dd[2], dn;
      std::vector<ComboDesc> cd[2];
      int nv[2] = {0, 0}, nn = 0, ne[2] = {0, 0};
      for (int i : act) {
        SysBuf& b = sys[i].lv->sb(sys[i].slot);
        const long len = len_of(i);
        const int k = st[i].k;
        double* w = b.V.p + (size_t)(k + 1) * len;
        double* hp = hdev.p + (size_t)i * hs;
        for (int pass = 0; pass < 2; ++pass) {
          dd[pass].push_back(DotDesc{b.V.p, w, b.partial.p, hp + pass * (m + 1), len, len, nv[pass]});
          nv[pass] += k + 1;
          cd[pass].push_back(ComboDesc{w, b.V.p, hp + pass * (m + 1), -1.0, 1.0, len, len, k + 1, ne[pass]});
          ne[pass] += (int)len;
        }
        dn.push_back(DotDesc{w, w, b.partial.p, hp + 2 * (m + 1), len, len, nn});
        nn += 1;
      }
      DescPack dp;
      const size_t o0 = dp.add(dd[0]), o1 = dp.add(cd[0]), o2 = dp.add(dd[1]), o3 = dp.add(cd[1]), o4 = dp.add(dn);
      char* base = push_desc_pack(dp.host);
      stage_begin(kStageArnoldi);
      launch_dots_multi(s, (const DotDesc*)(base + o0), (int)dd[0].size(), nv[0], kMultiDotBlocks);
      launch_combo_multi(s, (const ComboDesc*)(base + o1), (int)cd[0].size(), ne[0]);
      launch_dots_multi(s, (const DotDesc*)(base + o2), (int)dd[1].size(), nv[1], kMultiDotBlocks);
      launch_combo_multi(s, (const ComboDesc*)(base + o3), (int)cd[1].size(), ne[1]);
      launch_dots_multi(s, (const DotDesc*)(base + o4), (int)dn.size(), nn, kMultiDotBlocks);
      stage_end(kStageArnoldi);
    }
    readback();
    std::vector<int> need_restart, pc_end;
    std::vector<ComboDesc> scale_list;
    int scale_total = 0;
    for (int i : act) {
      GmState& g = st[i];
      SysRef& sr = sys[i];
      SysBuf& b = sr.lv->sb(sr.slot);
      const long len = len_of(i);
      const int k = g.k;
      const double* hb = &hhost[(size_t)i * hs];
      ++sr.its;
      for (int r = 0; r <= k; ++r) g.H[(size_t)r * m + k] = hb[r] + hb[m + 1 + r];
      const double hn = std::sqrt(std::max(0.0, hb[2 * (m + 1)]));
      if (!std::isfinite(hn)) throw Error(PQN_ERR_NUMERIC, "non-finite value in GMRES");
      g.H[(size_t)(k + 1) * m + k] = hn;
      for (int r = 0; r < k; ++r) {
        const double t0 = g.cs[r] * g.H[(size_t)r * m + k] + g.sn[r] * g.H[(size_t)(r + 1) * m + k];
        g.H[(size_t)(r + 1) * m + k] = -g.sn[r] * g.H[(size_t)r * m + k] + g.cs[r] * g.H[(size_t)(r + 1) * m + k];
        g.H[(size_t)r * m + k] = t0;
      }
      const double den = std::hypot(g.H[(size_t)k * m + k], g.H[(size_t)(k + 1) * m + k]);
      if (!(den > 0.0)) throw Error(PQN_ERR_NUMERIC, "GMRES breakdown: zero Hessenberg column");
      g.cs[k] = g.H[(size_t)k * m + k] / den;
      g.sn[k] = g.H[(size_t)(k + 1) * m + k] / den;
      g.H[(size_t)k * m + k] = den;
      g.H[(size_t)(k + 1) * m + k] = 0.0;
      g.g[k + 1] = -g.sn[k] * g.g[k];
      g.g[k] = g.cs[k] * g.g[k];
      sr.relres = std::fabs(g.g[k + 1]) / g.bnorm;
      const bool conv = std::fabs(g.g[k + 1]) <= sr.tol * g.bnorm || hn == 0.0;
      const bool full = (k + 1 == m) || sr.its >= sr.lv->max_iter;
      if (!conv && !full) {
        scale_list.push_back(ComboDesc{b.V.p + (size_t)(k + 1) * len, nullptr, nullptr, 0.0, 1.0 / hn, 0, len, 0,
                                       scale_total});
        scale_total += (int)len;
        g.k = k + 1;
        continue;
      }
      // end of cycle: y = H^{-1} g (upper triangular), x += V y
      const int dk = k + 1;
      std::vector<double> y(dk);
      for (int r = dk - 1; r >= 0; --r) {
        double v = g.g[r];
        for (int c2 = r + 1; c2 < dk; ++c2) v -= g.H[(size_t)r * m + c2] * y[c2];
        y[r] = v / g.H[(size_t)r * m + r];
      }
      HIPCHK(hipMemcpyAsync(b.ycoef.p, y.data(), dk * sizeof(double), hipMemcpyHostToDevice, s));
      if (pcs[i]) {
        // x += P (V y): z = V y here (tmp may hold this system's right-hand side); P in
        // place in z below, for all the systems whose cycle ends in this iteration at once
        launch_combo(s, b.z.p, 0.0, b.V.p, len, dk, b.ycoef.p, 1.0, len);
        pc_end.push_back(i);
      } else {
        launch_combo(s, sr.x, 1.0, b.V.p, len, dk, b.ycoef.p, 1.0, len);
      }
      g.active = false;
      const bool final_cycle = conv || sr.its >= sr.lv->max_iter;
      if (final_cycle && sr.res_out) {
        // final residual from the Arnoldi relation: r = V_{k+2} (beta e1 - Hbar y) =
        // V_{k+2} G_0^T ... G_k^T (0, ..., 0, g_{k+1}); V[k+1] still holds w unnormalised
        std::vector<double> e(dk + 1, 0.0);
        e[dk] = g.g[dk];
        for (int r = dk - 1; r >= 0; --r) {
          const double a0 = e[r], a1 = e[r + 1];
          e[r] = g.cs[r] * a0 - g.sn[r] * a1;
          e[r + 1] = g.sn[r] * a0 + g.cs[r] * a1;
        }
        e[dk] = hn > 0.0 ? e[dk] / hn : 0.0;
        HIPCHK(hipMemcpyAsync(b.rcoef.p, e.data(), (dk + 1) * sizeof(double), hipMemcpyHostToDevice, s));
        launch_combo(s, sr.res_out, 0.0, b.V.p, len, dk + 1, b.rcoef.p, 1.0, len);
      }
      if (conv) {
        sr.conv = true;
      } else if (sr.its >= sr.lv->max_iter) {
        sr.conv = false;
      } else {
        need_restart.push_back(i);
      }
    }
    if (!pc_end.empty()) {
      std::vector<MvGroup> eg;
      for (int i : pc_end) {
        SysBuf& b = sys[i].lv->sb(sys[i].slot);
        add_to_groups(eg, sys[i].c, sys[i].lv, sys[i].slot, b.z.p, b.z.p);
      }
      precond_apply_groups(eg);
      for (int i : pc_end) launch_axpby(s, sys[i].x, sys[i].lv->sb(sys[i].slot).z.p, 1.0, 1.0, len_of(i));
    }
    if (scale_list.size() == 1) {
      const ComboDesc& c0 = scale_list[0];
      launch_scale_copy(s, c0.w, c0.w, c0.beta, c0.len);
    } else if (!scale_list.empty()) {
      DescPack dp;
      const size_t o = dp.add(scale_list);
      char* base = push_desc_pack(dp.host);
      launch_combo_multi(s, (const ComboDesc*)(base + o), (int)scale_list.size(), scale_total);
    }
    if (!need_restart.empty()) {
      // true residual r = rhs - A x of the systems that exhausted a cycle
      std::vector<MvGroup> rg = build_groups(need_restart, true);
      matvec_groups(rg, precision);
      for (int i : need_restart) {
        SysBuf& b = sys[i].lv->sb(sys[i].slot);
        launch_axpby(s, b.r.p, sys[i].rhs, 1.0, -1.0, len_of(i));
        launch_dots(s, b.r.p, len_of(i), 1, b.r.p, len_of(i), sys[i].lv->nb_dots, b.partial.p, nrm_slot(i));
      }
      readback();
      for (int i : need_restart) {
        SysBuf& b = sys[i].lv->sb(sys[i].slot);
        const double beta = std::sqrt(std::max(0.0, hhost[(size_t)i * hs + 2 * (m + 1)]));
        sys[i].relres = beta / st[i].bnorm;
        if (beta <= sys[i].tol * st[i].bnorm) {
          sys[i].conv = true;
          residual_out(i, b.r.p);
        } else {
          start_cycle(i, b.r.p, beta);
        }
      }
    }
  }
}

// Solve every system in the context's precision. Mixed precision: GMRES on the
// operator with FP32 far pair sums, then optional refinement sweeps whose
// residual uses the FP64 operator.
void pqn_ctx_impl::solve_lockstep(std::vector<SysRef>& sys, pqn_mvp_stats* st, std::vector<int>* its_per) {
  const int prec = cfg.precision;
  // The preconditioner of a level (config precond) is built for the current configuration
  // at its first solve (precond = 2) or when the configuration is solved a second time
  // (precond = 1: a configuration solved once, such as a time step without contacts, never
  // pays for the set-up); decided once per level for this solve, refinement solves included.
  std::vector<Level*> decided;
  for (SysRef& r : sys) {
    pqn_ctx_impl& c = *r.c;
    Level& lv = *r.lv;
    if (!c.cfg.precond || std::find(decided.begin(), decided.end(), &lv) != decided.end()) continue;
    decided.push_back(&lv);
    lv.pc.use = false;
    if (lv.pc.epoch != c.config_epoch) {
      if (c.cfg.precond == 2 || lv.pc.seen == c.config_epoch) {
        c.precond_setup(lv);
      } else {
        lv.pc.seen = c.config_epoch;
        continue;
      }
    }
    lv.pc.use = true;
  }
  gmres_lockstep(sys, prec);
  int its = 0;
  for (SysRef& r : sys) its += r.its;
  if (its_per) {
    its_per->clear();
    for (SysRef& r : sys) its_per->push_back(r.its);
  }
  int sweeps = 0, fallback = 0;
  if (prec == PQN_MIXED && cfg.refine_sweeps > 0) {
    const int ns = (int)sys.size();
    std::vector<double> bn(ns);
    for (int i = 0; i < ns; ++i) {
      const long len = 3L * sys[i].lv->N;
      bn[i] = std::sqrt(dot_host(sys[i].rhs, sys[i].rhs, len, *sys[i].lv));
    }
    // checks 0..R (R = refine_sweeps) are each followed by a correction solve: mixed after
    // checks 0..R-1 (the sweeps), FP64 after check R (the fallback); check R+1 only measures
    for (int sw = 0; sw <= cfg.refine_sweeps + 1; ++sw) {
      std::vector<MvGroup> groups;
      for (int i = 0; i < ns; ++i) {
        SysBuf& b = sys[i].lv->sb(sys[i].slot);
        add_to_groups(groups, sys[i].c, sys[i].lv, sys[i].slot, sys[i].x, b.tmp.p);
      }
      matvec_groups(groups, PQN_FP64);
      std::vector<SysRef> corr;
      std::vector<int> owner;
      for (int i = 0; i < ns; ++i) {
        SysBuf& b = sys[i].lv->sb(sys[i].slot);
        const long len = 3L * sys[i].lv->N;
        launch_axpby(stream, b.tmp.p, sys[i].rhs, 1.0, -1.0, len);  // tmp = rhs - A64 x
        const double rn = std::sqrt(dot_host(b.tmp.p, b.tmp.p, len, *sys[i].lv));
        sys[i].relres = bn[i] > 0.0 ? rn / bn[i] : 0.0;
        sys[i].conv = sys[i].relres <= sys[i].tol;
        if (!sys[i].conv && bn[i] > 0.0) {
          corr.push_back(
              SysRef{sys[i].c, sys[i].lv, sys[i].slot, b.tmp.p, b.d.p, std::min(0.5, sys[i].tol * bn[i] / rn)});
          owner.push_back(i);
        }
      }
      if (corr.empty() || sw == cfg.refine_sweeps + 1) break;
      // after the last sweep's residual check, a system still above tolerance is finished in
      // FP64: the correction solve then runs with the FP64 operator
      const bool fb = sw == cfg.refine_sweeps;
      if (fb)
        fallback += (int)corr.size();
      else
        ++sweeps;
      gmres_lockstep(corr, fb ? PQN_FP64 : prec);  // corrections d for A d = rhs - A64 x
      for (size_t j = 0; j < corr.size(); ++j) {
        its += corr[j].its;
        if (its_per) (*its_per)[owner[j]] += corr[j].its;
        launch_axpby(stream, sys[owner[j]].x, corr[j].x, 1.0, 1.0, 3L * sys[owner[j]].lv->N);
      }
    }
  }
  if (st) {
    st->gmres_iters += its;
    st->refine_sweeps += sweeps;
    st->fp64_fallback += fallback;
    double rr = 0.0;
    bool conv = true;
    for (SysRef& r : sys) {
      rr = std::max(rr, r.relres);
      conv = conv && r.conv;
    }
    st->rel_residual = rr;
    st->converged = conv ? 1 : 0;
  }
}

// x0 = Q c and r0 = rhs - W c with c = W^T rhs (W orthonormal: the minimal residual over
// span(W), no operator application); the final residual goes to sb(0).tmp.
void pqn_ctx_impl::recycle_start(Level& lv, SysRef& sr) {
  Recycle& rc = lv.rc;
  const long len = 3L * lv.N;
  if (!rc.Q.p) {
    rc.kmax = std::min(32, lv.restart + 1);  // (dot partials hold restart + 1 vectors)
    rc.Q.alloc((size_t)rc.kmax * len);
    rc.W.alloc((size_t)rc.kmax * len);
    rc.c.alloc((size_t)rc.kmax);
    rc.nrm.alloc(2);
  }
  if (rc.epoch != config_epoch) {
    rc.k = 0;
    rc.epoch = config_epoch;
  }
  SysBuf& b = lv.sb(sr.slot);
  if (rc.k > 0) {
    launch_dots(stream, rc.W.p, len, rc.k, sr.rhs, len, lv.nb_dots, b.partial.p, rc.c.p);
    launch_combo(stream, b.d.p, 0.0, rc.Q.p, len, rc.k, rc.c.p, 1.0, len);
    launch_scale_copy(stream, b.tmp.p, sr.rhs, 1.0, len);
    launch_combo(stream, b.tmp.p, 1.0, rc.W.p, len, rc.k, rc.c.p, -1.0, len);
    sr.x0 = b.d.p;
    sr.r0 = b.tmp.p;
  }
  sr.res_out = b.tmp.p;
}

// Append the solution x (sb(0).x) and its image w = rhs - res to the store: both are
// projected against the stored pairs (two passes) and scaled so that the new w has unit
// norm (A q_new = w_new by linearity). An image within 1e-6 of the stored span adds
// nothing and is dropped; so is any once the store is full.
void pqn_ctx_impl::recycle_add(Level& lv, const double* res) {
  Recycle& rc = lv.rc;
  if (rc.k >= rc.kmax) return;
  const long len = 3L * lv.N;
  SysBuf& b = lv.sb(0);
  double* qn = rc.Q.p + (size_t)rc.k * len;
  double* wn = rc.W.p + (size_t)rc.k * len;
  launch_scale_copy(stream, qn, b.x.p, 1.0, len);
  launch_scale_copy(stream, wn, b.rhs.p, 1.0, len);
  launch_axpby(stream, wn, res, -1.0, 1.0, len);  // w = rhs - res
  launch_dots(stream, wn, len, 1, wn, len, lv.nb_dots, b.partial.p, rc.nrm.p);
  for (int pass = 0; pass < 2 && rc.k > 0; ++pass) {
    launch_dots(stream, rc.W.p, len, rc.k, wn, len, lv.nb_dots, b.partial.p, rc.c.p);
    launch_combo(stream, wn, 1.0, rc.W.p, len, rc.k, rc.c.p, -1.0, len);
    launch_combo(stream, qn, 1.0, rc.Q.p, len, rc.k, rc.c.p, -1.0, len);
  }
  launch_dots(stream, wn, len, 1, wn, len, lv.nb_dots, b.partial.p, rc.nrm.p + 1);
  double h[2] = {0.0, 0.0};
  HIPCHK(hipMemcpyAsync(h, rc.nrm.p, 2 * sizeof(double), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (!(std::isfinite(h[0]) && std::isfinite(h[1]))) throw Error(PQN_ERR_NUMERIC, "non-finite recycled image");
  if (h[1] > 1e-12 * h[0] && h[1] > 0.0) {
    const double sc = 1.0 / std::sqrt(h[1]);
    launch_scale_copy(stream, qn, qn, sc, len);
    launch_scale_copy(stream, wn, wn, sc, len);
    ++rc.k;
  }
}

void pqn_ctx_impl::mobility_multi(Level& lv, int K, const double* const* FT_dev, const double* axes_dev,
                                  double* const* UO_dev, pqn_mvp_stats* st) {
  if (K < 1 || K > kMaxRhs) throw Error(PQN_ERR_INVALID, "between 1 and 6 force sets per call");
  std::vector<SysRef> sys;
  for (int r = 0; r < K; ++r) {
    SysBuf& b = lv.sb(r);
    launch_rhs(stream, ctr.p, FT_dev ? FT_dev[r] : nullptr, axes_dev, lv.off.p, lv.n, M, lv.N, a, mu,
               cfg.slip_speed, b.rhs.p);
    sys.push_back(SysRef{this, &lv, r, b.rhs.p, b.x.p, lv.tol});
  }
  // slip-driven solve: the previous one's density is a close initial guess after a small step
  const bool slip_only = K == 1 && (!FT_dev || !FT_dev[0]) && axes_dev;
  if (slip_only && cfg.warm_start && lv.has_q_nc) sys[0].x0 = lv.q_nc.p;
  // force-driven solve inside an LCP solve that reuses earlier solutions
  const bool recycle = K == 1 && FT_dev && FT_dev[0] && lv.rc.active;
  if (recycle) recycle_start(lv, sys[0]);
  solve_lockstep(sys, st);
  if (recycle) recycle_add(lv, sys[0].res_out);
  if (slip_only && cfg.warm_start) {
    lv.q_nc.alloc(3 * (size_t)lv.N);
    HIPCHK(hipMemcpyAsync(lv.q_nc.p, lv.sb(0).x.p, 3 * (size_t)lv.N * sizeof(double), hipMemcpyDeviceToDevice,
                          stream));
    lv.has_q_nc = true;
  }
  for (int r = 0; r < K; ++r) {
    Work& w = lv.wk(r);
    launch_moments(stream, lv.sb(r).x.p, lv.off.p, lv.w.p, lv.n, M, lv.N, w.mom.p);
    launch_rigid_velocity(stream, w.mom.p, M, a, UO_dev[r]);
  }
  HIPCHK(hipGetLastError());
}

}  // namespace bipqn
