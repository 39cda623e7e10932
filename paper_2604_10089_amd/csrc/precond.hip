// Right preconditioner of the BIE's GMRES (config precond).
//
// Sec. 2 notes that practical mobility solves need preconditioned Krylov
// methods without fixing a preconditioner; this is the one used here. GMRES
// solves (1/2 I + D + P) P_r y = rhs and returns q = P_r y, so the solution and
// the stopping rule (true residual of q) are those of the unpreconditioned
// solve. For sphere i with near partners j (gap < near_gap):
//
//   (P_r v)_i = S_i^{-1} (v_i - sum_j A_ij D^{-1} v_j),  S_i = D - sum_j A_ij D^{-1} A_ji,
//
// where D is the single-sphere block (1/2 I + self interaction + rigid
// projection: one matrix for every sphere, the spheres being identical and
// their grids globally aligned) and A_ij the near block of the pair (the near
// rule's map from sphere j's density to sphere i's nodes). This is the row of
// sphere i of the inverse of its near patch [[D, A_ij], [A_ji, D], ...] with
// the coupling between its partners dropped: a restricted additive Schwarz
// preconditioner over near-pair patches with the patch solves reduced to Schur
// complements. For a lone near pair it is the pair's exact inverse; far
// interactions stay out (smooth, few GMRES iterations).
//
// Set-up, once per configuration and level (at the first solve after a change):
//   - D on the host from the self block and the rigid projection, D^{-1} by
//     Gauss-Jordan elimination with partial pivoting (once per level);
//   - the near blocks from the near stage of the operator (the same kernels as
//     every product) applied to unit harmonic-coefficient vectors, six at a
//     time (the near rule reads a density only through its coefficients), then
//     mapped to node space by the analysis T;
//   - S_i by FP64 matrix-core GEMMs, S_i^{-1} by the Newton-Schulz iteration
//     X <- X (2I - S_i X) from X = D^{-1} until every sphere's residual
//     ||I - S_i X||_F / sqrt(3n) is below kNsTol. A sphere whose iteration does
//     not get below kNsKeep keeps X = D^{-1} (block Jacobi for that sphere).
//
//   - G_ij = S_i^{-1} A_ij D^{-1} for every near pair, so that
//     (P_r v)_i = S_i^{-1} v_i - sum_j G_ij v_j: one block-sparse product whose
//     blocks (S_i^{-1} and the G_ij, 3n x 3n each) are stored in FP16, each
//     scaled by its largest magnitude (one FP32 factor per block). P_r is a
//     fixed linear map either way, so GMRES keeps its convergence theory and the
//     solution its accuracy; the rounding only perturbs the preconditioner (the
//     iteration counts on the test workloads are those of FP64 blocks).
// Each application streams the blocks once from HBM ((M + n_near) (3n)^2 2 bytes:
// 1.1 GB at 216 spheres and 12x24 nodes), whatever the number of densities K.
//
// Layouts (3n = per-sphere unknowns, local index c n + x: component c, node x):
//   D, D^{-1}: [3n][3n] row-major; near blocks of sphere i: [3n][npart_i 3n]
//   row-major (slot s in columns s 3n ..); S_i row-major; X_i by columns; the
//   FP16 blocks by columns padded to a multiple of 64 rows, sphere i's row of
//   blocks contiguous (S_i^{-1} first).
#include "context.hpp"

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

namespace bipqn {

constexpr double kNsTol = 1e-8;    // Newton-Schulz stop: residual of every sphere below this
constexpr double kNsKeep = 1e-3;   // spheres above this after the last step fall back to D^{-1}
constexpr int kNsMaxSteps = 14;

// ---------------------------------------------------------------- host set-up

// D = 1/2 I + S + P_rigid in local order (rows c n + x, columns d n + m). P_rigid
// is the rigid projection of the completed operator: the translation
// w_m delta_cd / (4 pi a^2) and the rotation -(3 / (8 pi a^4)) w_m [o_x]x [o_m]x,
// with ([a]x [b]x)_cd = b_c a_d - (a.b) delta_cd.
void single_sphere_block(const SphereTables& t, std::vector<double>& D) {
  const int n = t.n, n3 = 3 * n;
  const double a = t.radius;
  D = t.S;
  for (int r = 0; r < n3; ++r) D[(size_t)r * n3 + r] += 0.5;
  const double ctr = 1.0 / (4.0 * kPi * a * a), crot = 3.0 / (8.0 * kPi * a * a * a * a);
  for (int x = 0; x < n; ++x) {
    const double* ox = &t.off[3 * x];
    for (int m = 0; m < n; ++m) {
      const double* om = &t.off[3 * m];
      const double wm = t.w[m];
      const double dot = ox[0] * om[0] + ox[1] * om[1] + ox[2] * om[2];
      for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) {
          const double cross2 = om[c] * ox[d] - (c == d ? dot : 0.0);
          D[(size_t)(c * n + x) * n3 + d * n + m] += (c == d ? ctr * wm : 0.0) - crot * wm * cross2;
        }
    }
  }
}

// In-place inverse of the row-major n x n matrix A (Gauss-Jordan, partial pivoting).
void invert_gauss_jordan(std::vector<double>& A, int n) {
  std::vector<int> perm(n);
  for (int i = 0; i < n; ++i) perm[i] = i;
  std::vector<double> rowk(n);
  for (int k = 0; k < n; ++k) {
    int piv = k;
    double best = std::fabs(A[(size_t)k * n + k]);
    for (int r = k + 1; r < n; ++r)
      if (std::fabs(A[(size_t)r * n + k]) > best) {
        best = std::fabs(A[(size_t)r * n + k]);
        piv = r;
      }
    if (!(best > 0.0) || !std::isfinite(best)) throw Error(PQN_ERR_NUMERIC, "singular single-sphere block");
    if (piv != k) {
      std::swap_ranges(A.begin() + (size_t)k * n, A.begin() + (size_t)(k + 1) * n, A.begin() + (size_t)piv * n);
      std::swap(perm[k], perm[piv]);
    }
    double* ak = &A[(size_t)k * n];
    const double inv = 1.0 / ak[k];
    ak[k] = 1.0;
    for (int c = 0; c < n; ++c) ak[c] *= inv;
    std::copy(ak, ak + n, rowk.begin());
    for (int r = 0; r < n; ++r) {
      if (r == k) continue;
      double* ar = &A[(size_t)r * n];
      const double f = ar[k];
      if (f == 0.0) continue;
      ar[k] = 0.0;
      for (int c = 0; c < n; ++c) ar[c] -= f * rowk[c];
    }
  }
  // the row swaps act as a column permutation of the inverse: undo it
  std::vector<double> tmp(n);
  for (int r = 0; r < n; ++r) {
    double* ar = &A[(size_t)r * n];
    for (int c = 0; c < n; ++c) tmp[perm[c]] = ar[c];
    std::copy(tmp.begin(), tmp.end(), ar);
  }
}

// D, D^{-1} and D^{-1} by columns of one grid, built once per process (the same for
// every context and suspension on that grid; batch contexts have many).
struct SphereBlock {
  std::vector<double> D, Dinv, DinvT;
};

static const SphereBlock& sphere_block_cached(const SphereTables& t) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, double>, std::unique_ptr<SphereBlock>> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto key = std::make_tuple(t.n_theta, t.n_phi, t.radius);
  auto it = cache.find(key);
  if (it != cache.end()) return *it->second;
  auto sb = std::make_unique<SphereBlock>();
  const int n3 = 3 * t.n;
  single_sphere_block(t, sb->D);
  sb->Dinv = sb->D;
  invert_gauss_jordan(sb->Dinv, n3);
  sb->DinvT.resize((size_t)n3 * n3);
  for (int r = 0; r < n3; ++r)
    for (int c = 0; c < n3; ++c) sb->DinvT[(size_t)c * n3 + r] = sb->Dinv[(size_t)r * n3 + c];
  return *(cache[key] = std::move(sb));
}

// ------------------------------------------------------------------ kernels

// Harmonic coefficients of K unit columns of the coefficient space, the same on every
// sphere: coef[(i 3K + 3r + c) L + l] = 1 where c L + l = k0 + r ([M][3K][L] layout).
__global__ __launch_bounds__(256) void k_unit_coef(double* __restrict__ coef, int K, int k0, int L, int M) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  const long per = 3L * K * L;
  if (e >= (long)M * per) return;
  const long q = e % per;
  const int row = (int)(q / L), l = (int)(q - (long)row * L);
  const int r = row / 3, c = row - 3 * r;
  coef[e] = (c * L + l == k0 + r) ? 1.0 : 0.0;
}

// Columns k0 .. k0 + K - 1 of the coefficient-space near blocks from the near partials:
// NBc_i(row, s ncol + k0 + r) = near_part_r[s 3N + c N + i n + x], row = c n + x, ncol = 3L.
// Thread per (sphere, slot, row), writing its K consecutive columns.
__global__ __launch_bounds__(256) void k_nb_scatter(OPtrs np, int K, int k0, int ncol, const int* __restrict__ npart,
                                                    const long* __restrict__ nbo, int n, int M, int N,
                                                    double* __restrict__ NB) {
  const int n3 = 3 * n;
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)M * kMaxNear * n3) return;
  const int row = (int)(e % n3);
  const int s = (int)((e / n3) % kMaxNear);
  const int i = (int)(e / ((long)n3 * kMaxNear));
  const int ns = npart[i];
  if (s >= ns) return;
  const int c = row / n, x = row - c * n;
  double* dst = NB + nbo[i] + (size_t)row * ns * ncol + (size_t)s * ncol + k0;
  const size_t src = (size_t)s * 3 * N + (size_t)c * N + (size_t)i * n + x;
  for (int r = 0; r < K; ++r) dst[r] = np.p[r][src];
}

// The set-up's elementwise passes over [M][3n][3n] matrices: one block per (sphere,
// column), threads along the column (no 64-bit index division per element).

// S_i = D - C_i (row-major, in place over C), for every sphere.
__global__ __launch_bounds__(256) void k_schur_finish(const double* __restrict__ D, int n3,
                                                      double* __restrict__ S) {
  const size_t col = (size_t)blockIdx.x % n3, i = (size_t)blockIdx.x / n3;
  double* s = S + (i * n3 + col) * n3;
  const double* d = D + col * n3;
  for (int r = threadIdx.x; r < n3; r += 256) s[r] = d[r] - s[r];
}

// W <- 2I - W for every sphere (by columns; the diagonal is the same either way).
__global__ __launch_bounds__(256) void k_two_minus(double* __restrict__ W, int n3) {
  const int col = blockIdx.x % n3;
  double* w = W + (size_t)blockIdx.x * n3;
  for (int r = threadIdx.x; r < n3; r += 256) w[r] = (r == col ? 2.0 : 0.0) - w[r];
}

// Partial sums of ||I - W_i||_F^2: block (i, g) covers the columns c = g, g + kNsSlices, ...
// of sphere i; res[i kNsSlices + g] (the host adds the slices in order).
constexpr int kNsSlices = 32;
__global__ __launch_bounds__(256) void k_ns_residual(const double* __restrict__ W, int n3, double* __restrict__ res) {
  __shared__ double sh[256];
  const int i = blockIdx.x / kNsSlices, g = blockIdx.x % kNsSlices;
  const double* Wi = W + (size_t)i * n3 * n3;
  double acc = 0.0;
  for (int c = g; c < n3; c += kNsSlices)
    for (int r = threadIdx.x; r < n3; r += 256) {
      const double d = (r == c ? 1.0 : 0.0) - Wi[(size_t)c * n3 + r];
      acc = fma(d, d, acc);
    }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) res[blockIdx.x] = sh[0];
}

// vI[(j 3n + m) K + r] = v_r[c N + j n + x], m = c n + x: the K densities of a node
// next to each other, one scalar-load stream per block column.
__global__ __launch_bounds__(256) void k_pc_interleave(QPtrs v, int K, int n, int M, int N,
                                                       double* __restrict__ vI) {
  const int n3 = 3 * n;
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)M * n3 * K) return;
  const int r = (int)(e % K);
  const long jm = e / K;
  const int m = (int)(jm % n3), j = (int)(jm / n3);
  const int c = m / n, x = m - c * n;
  vI[e] = v.p[r][(size_t)c * N + (size_t)j * n + x];
}

// Largest magnitude of each FP64 block (one workgroup per block, fixed-order reduction).
__global__ __launch_bounds__(256) void k_block_absmax(const double* const* __restrict__ src, long nn,
                                                      float* __restrict__ scale) {
  __shared__ double sh[256];
  const double* s = src[blockIdx.x];
  double m = 0.0;
  for (long l = threadIdx.x; l < nn; l += 256) m = fmax(m, fabs(s[l]));
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) scale[blockIdx.x] = sh[0] > 0.0 ? (float)sh[0] : 1.0f;
}

// FP16 copies of FP64 blocks stored by columns: block b of the list is sgn[b] src[b] / scale[b]
// (entries in [-1, 1]; the product multiplies the scale back), each column padded with zeros
// to ld entries (a multiple of 64: every column starts on a 128-byte line).
__global__ __launch_bounds__(256) void k_blocks_f16(const double* const* __restrict__ src,
                                                    const double* __restrict__ sgn, const float* __restrict__ scale,
                                                    int n3, int ld, long nb, _Float16* __restrict__ dst) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  const long per = (long)n3 * ld;
  if (e >= nb * per) return;
  const long b = e / per;
  const long l = e - b * per;
  const int m = (int)(l / ld), r = (int)(l - (long)m * ld);
  dst[e] = r < n3 ? (_Float16)(float)(sgn[b] / scale[b] * src[b][(size_t)m * n3 + r]) : (_Float16)0.0f;
}

// part[(b K + r) 3n + row] = sum_m B_b(row, m) vI[(j 3n + m) K + r], j the column sphere of
// block b. Thread per (block, row): the block's columns are read by consecutive rows
// (coalesced), the densities of node m of sphere j are wave-uniform (scalar loads). A
// workgroup per (block, 256 rows), rather than per (sphere, rows), gives the launch
// enough waves to keep the loads in flight that stream the blocks from HBM.
// FP16 blocks scaled to [-1, 1] (scale[b] multiplied back at the end), FP64 products and sums.
template <int K>
__device__ __forceinline__ void bsr_block_body(const _Float16* __restrict__ B, const float* __restrict__ scale,
                                               const int* __restrict__ bcol, const double* __restrict__ vI,
                                               int n3, int ld, int rchunks, int wg, double* __restrict__ part) {
  const int b = wg / rchunks;
  const int row = (wg - b * rchunks) * 256 + threadIdx.x;
  const bool valid = row < n3;
  const int rr = valid ? row : n3 - 1;
  const _Float16* Bb = B + (size_t)b * n3 * ld + rr;
  const double* v = vI + (size_t)bcol[b] * n3 * K;
  double acc[K];
#pragma unroll
  for (int r = 0; r < K; ++r) acc[r] = 0.0;
#pragma unroll 8
  for (int m = 0; m < n3; ++m) {
    const double a = (double)(float)Bb[(size_t)m * ld];
#pragma unroll
    for (int r = 0; r < K; ++r) acc[r] = fma(a, v[m * K + r], acc[r]);
  }
  if (valid) {
    const double sc = scale[b];
#pragma unroll
    for (int r = 0; r < K; ++r) part[((size_t)b * K + r) * n3 + row] = sc * acc[r];
  }
}

template <int K>
__global__ __launch_bounds__(256) void k_bsr_block(const _Float16* __restrict__ B, const float* __restrict__ scale,
                                                   const int* __restrict__ bcol, const double* __restrict__ vI,
                                                   int n3, int ld, int rchunks, double* __restrict__ part) {
  bsr_block_body<K>(B, scale, bcol, vI, n3, ld, rchunks, blockIdx.x, part);
}

// Many suspensions in one launch (one density each): segment descriptors, workgroups
// [start, ...) of a segment for the block products, elements [estart, estart + M 3n)
// for the interleave and the sum.
struct PcDesc {
  const _Float16* B;
  const float* scale;
  const int* bcol;
  const int* bptr;
  const double* in;
  double* out;
  double* vI;
  double* part;
  int n, N, M, ld, rchunks, start;
  long estart;
};

__device__ __forceinline__ int pc_seg_blocks(const PcDesc* __restrict__ d, int nd, int wg) {
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].start <= wg)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int pc_seg_elems(const PcDesc* __restrict__ d, int nd, long e) {
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].estart <= e)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_pc_interleave_multi(const PcDesc* __restrict__ d, int nd, long total) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const PcDesc D = d[pc_seg_elems(d, nd, e)];
  const long l = e - D.estart;
  const int n3 = 3 * D.n;
  const int j = (int)(l / n3), m = (int)(l - (long)j * n3);
  const int c = m / D.n, x = m - c * D.n;
  D.vI[l] = D.in[(size_t)c * D.N + (size_t)j * D.n + x];
}

__global__ __launch_bounds__(256) void k_bsr_block_multi(const PcDesc* __restrict__ d, int nd) {
  const PcDesc D = d[pc_seg_blocks(d, nd, blockIdx.x)];
  bsr_block_body<1>(D.B, D.scale, D.bcol, D.vI, 3 * D.n, D.ld, D.rchunks, blockIdx.x - D.start, D.part);
}

__global__ __launch_bounds__(256) void k_bsr_sum_multi(const PcDesc* __restrict__ d, int nd, long total) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const PcDesc D = d[pc_seg_elems(d, nd, e)];
  const long l = e - D.estart;
  const int n3 = 3 * D.n;
  const int i = (int)(l / n3), row = (int)(l - (long)i * n3);
  double v = 0.0;
  for (int b = D.bptr[i]; b < D.bptr[i + 1]; ++b) v += D.part[(size_t)b * n3 + row];
  const int c = row / D.n, x = row - c * D.n;
  D.out[(size_t)c * D.N + (size_t)i * D.n + x] = v;
}

// out_r[c N + i n + x] = sum of the partials of sphere i's blocks (in block order), row = c n + x.
__global__ __launch_bounds__(256) void k_bsr_sum(const double* __restrict__ part, const int* __restrict__ bptr,
                                                 int K, int n, int M, int N, OPtrs out) {
  const int n3 = 3 * n;
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)M * K * n3) return;
  const int row = (int)(e % n3);
  const int r = (int)((e / n3) % K);
  const int i = (int)(e / ((long)n3 * K));
  double v = 0.0;
  for (int b = bptr[i]; b < bptr[i + 1]; ++b) v += part[((size_t)b * K + r) * n3 + row];
  const int c = row / n, x = row - c * n;
  out.p[r][(size_t)c * N + (size_t)i * n + x] = v;
}

static unsigned nblocks(long count) { return (unsigned)((count + 255) / 256); }

// ------------------------------------------------------------ near stage only

void pqn_ctx_impl::near_stage(MvGroup& gr, bool from_coef) {
  Level& lv = *gr.lv;
  hipStream_t s = stream;
  if (n_near + n_near2 == 0) return;
  double* qup = n_near > 0 ? group_qup(gr) : nullptr;
  double* qup2 = n_near2 > 0 ? group_qup(gr, true) : nullptr;
  double* coef = group_coef(gr);
  std::vector<GemmDesc> ga, gb;
  int nga = 0, ngb = 0;
  push_group_gemms(lv, gr.K, gr.slot, gr.in, coef, qup, qup2, nullptr, ga, nga, gb, ngb, false);
  DescPack dp;
  const size_t oa = dp.add(ga), ob = dp.add(gb);
  char* base = push_desc_pack(dp.host);
  if (!from_coef) launch_gemm64_multi(s, (const GemmDesc*)(base + oa), (int)ga.size(), nga);
  launch_gemm64_multi(s, (const GemmDesc*)(base + ob), (int)gb.size(), ngb);
  OPtrs np{};
  for (int r = 0; r < gr.K; ++r) np.p[r] = lv.wk(gr.slot[r]).near_part.p;
  const double scale = 3.0 / (4.0 * kPi * a);
  launch_near(s, gr.K, n_near, ctr.p, lv.off.p, lv.offup.p, lv.shab.p, qup, coef, near_list.p, lv.n, lv.M, lv.N,
              lv.nup, lv.p, lv.L, scale, np);
  launch_near(s, gr.K, n_near2, ctr.p, lv.off.p, lv.offup2.p, lv.shab.p, qup2, coef, near_list2.p, lv.n, lv.M,
              lv.N, lv.nup2, lv.p, lv.L, scale, np);
}

// ----------------------------------------------------------------- set-up

void pqn_ctx_impl::precond_setup(Level& lv) {
  Precond& pc = lv.pc;
  if (!cfg.precond || pc.epoch == config_epoch) return;
  TraceRange trace("precond_setup");
  HIPCHK(hipStreamSynchronize(stream));
  Timer tm;
  hipStream_t s = stream;
  const int n = lv.n, n3 = 3 * n, M = lv.M, N = lv.N;
  const size_t nn = (size_t)n3 * n3;
  if (!pc.has_d) {
    const SphereBlock& sb = sphere_block_cached(lv.tab);
    pc.D.upload(sb.D.data(), nn, s);
    pc.Dinv.upload(sb.Dinv.data(), nn, s);
    pc.DinvT.upload(sb.DinvT.data(), nn, s);
    HIPCHK(hipStreamSynchronize(s));
    pc.has_d = true;
  }
  pc.X.alloc((size_t)M * nn);
  pc.res.alloc((size_t)M * kNsSlices);
  long total = 0;
  pc.nbo.assign(M, 0);
  for (int i = 0; i < M; ++i) {
    pc.nbo[i] = total;
    total += (long)h_npart[i] * nn;
  }
  pc.fallback = 0;
  pc.ns_iters = 0;
  if (total == 0) {
    // no near pairs: block Jacobi
    for (int i = 0; i < M; ++i)
      HIPCHK(hipMemcpyAsync(pc.X.p + (size_t)i * nn, pc.DinvT.p, nn * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else {
    pc.NB.alloc((size_t)total);
    pc.TB.alloc((size_t)total);
    // Near blocks. The near rule reads a density only through its harmonic coefficients
    // (coef = T q: the upsampled values and the foot-point expansion), so A_ij = Ac_ij (I3 x T)
    // with Ac_ij [3n][3L]: Ac from unit coefficient columns through the near stage (3L / 6
    // passes instead of 3n / 6), then A = Ac (I3 x T) by GEMMs into NB.
    const int L = lv.L, n3L = 3 * L;
    std::vector<long> nbco(M);
    long totc = 0;
    for (int i = 0; i < M; ++i) {
      nbco[i] = totc;
      totc += (long)h_npart[i] * n3 * n3L;
    }
    pc.NBc.alloc((size_t)totc);
    DevArray<long> dnbco;
    dnbco.upload(nbco.data(), nbco.size(), s);
    for (int k0 = 0; k0 < n3L; k0 += kMaxRhs) {
      const int K = std::min(kMaxRhs, n3L - k0);
      MvGroup g{this, &lv, K, {}, {}, {}};
      OPtrs np{};
      for (int r = 0; r < K; ++r) {
        g.slot[r] = r;
        g.in[r] = lv.off.p;  // not read: the coefficients are given
        np.p[r] = lv.wk(r).near_part.p;
      }
      double* coef = group_coef(g);
      hipLaunchKernelGGL(k_unit_coef, dim3(nblocks((long)M * 3 * K * L)), dim3(256), 0, s, coef, K, k0, L, M);
      near_stage(g, true);
      hipLaunchKernelGGL(k_nb_scatter, dim3(nblocks((long)M * kMaxNear * n3)), dim3(256), 0, s, np, K, k0, n3L,
                         npart.p, dnbco.p, n, M, N, pc.NBc.p);
    }
    {
      // NB_i(:, s 3n + d n + m) = sum_l Ac_i(:, s 3L + d L + l) T(l, m), T read by columns (TT)
      if (!pc.TT.p) {
        std::vector<double> tt((size_t)n * L);
        for (int l = 0; l < L; ++l)
          for (int m = 0; m < n; ++m) tt[(size_t)m * L + l] = lv.tab.T[(size_t)l * n + m];
        pc.TT.upload(tt.data(), tt.size(), s);
      }
      std::vector<GemmDesc> gc;
      int ngc = 0;
      for (int i = 0; i < M; ++i) {
        const int ns = h_npart[i];
        for (int sl = 0; sl < ns; ++sl)
          for (int d = 0; d < 3; ++d)
            push_gemm(gc, ngc, n3, n, L, pc.NBc.p + nbco[i] + (size_t)sl * n3L + (size_t)d * L, ns * n3L, pc.TT.p, L,
                      pc.NB.p + pc.nbo[i] + (size_t)sl * n3 + (size_t)d * n, n3, 0, 1, ns * n3, n, 0, 0, 1);
      }
      DescPack dc;
      const size_t occ = dc.add(gc);
      char* cb = push_desc_pack(dc.host);
      launch_gemm64_multi_big(s, (const GemmDesc*)(cb + occ), (int)gc.size(), ngc);
    }
    // T_(i,s) = D^{-1} A_(j,s'), j the partner in slot s of i and s' the slot of i in j's list,
    // stored as TB_i(c, s 3n + m) = T_(i,s)(m, c): computed as C(c, m) = sum_k A_(j,s')(k, c) D^{-1}(m, k)
    pc.S.alloc((size_t)M * nn);
    std::vector<GemmDesc> gt, gs;
    int ngt = 0, ngs = 0;
    for (int i = 0; i < M; ++i) {
      const int ns = h_npart[i];
      if (ns == 0) {  // C_i = 0: a product with no terms writes zeros
        push_gemm(gs, ngs, n3, n3, 0, pc.Dinv.p, n3, pc.Dinv.p, n3, pc.S.p + (size_t)i * nn, n3, 0, 1, n3, n3, 0, 0, 1);
        continue;
      }
      const int ldi = ns * n3;
      for (int sl = 0; sl < ns; ++sl) {
        const int j = h_partners[(size_t)i * kMaxNear + sl];
        int sj = -1;
        for (int q = 0; q < h_npart[j]; ++q)
          if (h_partners[(size_t)j * kMaxNear + q] == i) sj = q;
        if (sj < 0) throw Error(PQN_ERR_STATE, "internal: near pair list is not symmetric");
        const int ldj = h_npart[j] * n3;
        push_gemm(gt, ngt, n3, n3, n3, pc.NB.p + pc.nbo[j] + (size_t)sj * n3, ldj, pc.Dinv.p, n3,
                  pc.TB.p + pc.nbo[i] + (size_t)sl * n3, n3, 0, 1, ldi, n3, 0, 1, 1);
      }
      // C_i = sum_s A_(i,s) T_(i,s): one product over the concatenated slots, row-major into S_i
      push_gemm(gs, ngs, n3, n3, ldi, pc.NB.p + pc.nbo[i], ldi, pc.TB.p + pc.nbo[i], ldi, pc.S.p + (size_t)i * nn,
                n3, 0, 1, n3, n3, 0, 0, 1);
    }
    DescPack dp;
    const size_t ot = dp.add(gt), os = dp.add(gs);
    char* base = push_desc_pack(dp.host);
    launch_gemm64_multi_big(s, (const GemmDesc*)(base + ot), (int)gt.size(), ngt);
    launch_gemm64_multi_big(s, (const GemmDesc*)(base + os), (int)gs.size(), ngs);
    hipLaunchKernelGGL(k_schur_finish, dim3(M * n3), dim3(256), 0, s, pc.D.p, n3, pc.S.p);
    // Newton-Schulz from X = D^{-1}
    pc.X2.alloc((size_t)M * nn);
    pc.W.alloc((size_t)M * nn);
    for (int i = 0; i < M; ++i)
      HIPCHK(hipMemcpyAsync(pc.X.p + (size_t)i * nn, pc.DinvT.p, nn * sizeof(double), hipMemcpyDeviceToDevice, s));
    std::vector<double> res(M), resp((size_t)M * kNsSlices);
    for (int step = 0;; ++step) {
      // W = S X (by columns): C(r, c) = sum_k S(r, k) X(k, c)
      launch_gemm64_big(s, n3, n3, n3, pc.S.p, n3, (long)nn, pc.X.p, (long)nn, n3, pc.W.p, (long)nn, n3, 0, n3, M, 0);
      hipLaunchKernelGGL(k_ns_residual, dim3(M * kNsSlices), dim3(256), 0, s, pc.W.p, n3, pc.res.p);
      HIPCHK(hipMemcpyAsync(resp.data(), pc.res.p, resp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (int i = 0; i < M; ++i) {
        double t = 0.0;
        for (int g = 0; g < kNsSlices; ++g) t += resp[(size_t)i * kNsSlices + g];
        res[i] = t / n3;
      }
      double worst = 0.0;
      for (double v : res) worst = std::isfinite(v) ? std::max(worst, std::sqrt(v)) : 1e300;
      if (worst <= kNsTol || step == kNsMaxSteps) break;
      // X <- X (2I - W): C(r, c) = sum_k X(r, k) F(k, c), X read by columns
      hipLaunchKernelGGL(k_two_minus, dim3(M * n3), dim3(256), 0, s, pc.W.p, n3);
      launch_gemm64_big(s, n3, n3, n3, pc.X.p, n3, (long)nn, pc.W.p, (long)nn, n3, pc.X2.p, (long)nn, n3, 0, n3, M, 1);
      std::swap(pc.X.p, pc.X2.p);
      ++pc.ns_iters;
    }
    for (int i = 0; i < M; ++i)
      if (!(std::sqrt(res[i]) <= kNsKeep)) {
        HIPCHK(hipMemcpyAsync(pc.X.p + (size_t)i * nn, pc.DinvT.p, nn * sizeof(double), hipMemcpyDeviceToDevice, s));
        ++pc.fallback;
      }
    // G_(i,s) = X_i A_(i,s) D^{-1}: H = A_(i,s) D^{-1} by columns into TB (slot s at s (3n)^2),
    // then G = X_i H by columns into NB (the near blocks are no longer needed)
    std::vector<GemmDesc> gh, gg;
    int ngh = 0, ngg = 0;
    for (int i = 0; i < M; ++i) {
      const int ns = h_npart[i];
      const int ldi = ns * n3;
      for (int sl = 0; sl < ns; ++sl) {
        push_gemm(gh, ngh, n3, n3, n3, pc.NB.p + pc.nbo[i] + (size_t)sl * n3, ldi, pc.DinvT.p, n3,
                  pc.TB.p + pc.nbo[i] + (size_t)sl * nn, n3, 0, n3, 1, n3, 0, 0, 1);
        push_gemm(gg, ngg, n3, n3, n3, pc.X.p + (size_t)i * nn, n3, pc.TB.p + pc.nbo[i] + (size_t)sl * nn, n3,
                  pc.NB.p + pc.nbo[i] + (size_t)sl * nn, n3, 0, n3, 1, n3, 0, 1, 1);
      }
    }
    DescPack dq;
    const size_t oh = dq.add(gh), og = dq.add(gg);
    char* qb = push_desc_pack(dq.host);
    launch_gemm64_multi_big(s, (const GemmDesc*)(qb + oh), (int)gh.size(), ngh);
    launch_gemm64_multi_big(s, (const GemmDesc*)(qb + og), (int)gg.size(), ngg);
    HIPCHK(hipStreamSynchronize(s));  // dnbco and the descriptor tables are released/reused after this
  }
  // block rows in FP16: sphere i holds S_i^{-1} (or D^{-1}) then G_(i,s) for its slots
  {
    std::vector<int> bp(M + 1, 0), bc;
    std::vector<const double*> src;
    std::vector<double> sg;
    for (int i = 0; i < M; ++i) {
      bp[i] = (int)bc.size();
      bc.push_back(i);
      src.push_back(pc.X.p + (size_t)i * nn);
      sg.push_back(1.0);
      for (int sl = 0; sl < h_npart[i]; ++sl) {
        bc.push_back(h_partners[(size_t)i * kMaxNear + sl]);
        src.push_back(pc.NB.p + pc.nbo[i] + (size_t)sl * nn);
        sg.push_back(-1.0);
      }
    }
    bp[M] = (int)bc.size();
    const long nb = (long)bc.size();
    pc.nblk = (int)nb;
    pc.ld = (n3 + 63) / 64 * 64;
    pc.B16.alloc((size_t)nb * n3 * pc.ld);
    pc.bscale.alloc((size_t)nb);
    pc.bptr.upload(bp.data(), bp.size(), s);
    pc.bcol.upload(bc.data(), bc.size(), s);
    DevArray<const double*> dsrc;
    DevArray<double> dsg;
    dsrc.upload(src.data(), src.size(), s);
    dsg.upload(sg.data(), sg.size(), s);
    hipLaunchKernelGGL(k_block_absmax, dim3(nb), dim3(256), 0, s, dsrc.p, (long)nn, pc.bscale.p);
    hipLaunchKernelGGL(k_blocks_f16, dim3(nblocks(nb * (long)n3 * pc.ld)), dim3(256), 0, s, dsrc.p, dsg.p,
                       pc.bscale.p, n3, pc.ld, nb, pc.B16.p);
    HIPCHK(hipStreamSynchronize(s));  // dsrc is released after this
  }
  HIPCHK(hipGetLastError());
  pc.epoch = config_epoch;
  pc.setup_ms = tm.ms();
  pc_setup_ms += pc.setup_ms;
  pc_fallback += pc.fallback;
}

// ------------------------------------------------------------ application

// Every group's densities through its own level's preconditioner: one segmented launch
// per phase when the groups are single densities of different contexts (the suspensions
// of a batch), else one application per group.
void pqn_ctx_impl::precond_apply_groups(std::vector<MvGroup>& groups) {
  bool multi = groups.size() > 1;
  for (MvGroup& gr : groups) multi = multi && gr.K == 1;
  if (!multi) {
    for (MvGroup& gr : groups) gr.c->precond_apply(gr);
    return;
  }
  hipStream_t s = stream;
  std::vector<PcDesc> pd;
  int wg = 0;
  long el = 0;
  for (MvGroup& gr : groups) {
    pqn_ctx_impl& c = *gr.c;
    Level& lv = *gr.lv;
    Precond& pc = lv.pc;
    if (pc.epoch != c.config_epoch) throw Error(PQN_ERR_STATE, "internal: preconditioner not set up");
    const int n3 = 3 * lv.n;
    pc.vI.alloc((size_t)lv.M * n3 * kMaxRhs);
    pc.part.alloc((size_t)pc.nblk * kMaxRhs * n3);
    const int rchunks = (n3 + 255) / 256;
    pd.push_back(PcDesc{pc.B16.p, pc.bscale.p, pc.bcol.p, pc.bptr.p, gr.in[0], gr.out[0], pc.vI.p, pc.part.p, lv.n,
                        lv.N, lv.M, pc.ld, rchunks, wg, el});
    wg += pc.nblk * rchunks;
    el += (long)lv.M * n3;
  }
  DescPack dp;
  const size_t od = dp.add(pd);
  const PcDesc* dd = (const PcDesc*)(push_desc_pack(dp.host) + od);
  const int nd = (int)pd.size();
  stage_begin(kStagePrecond);
  hipLaunchKernelGGL(k_pc_interleave_multi, dim3(nblocks(el)), dim3(256), 0, s, dd, nd, el);
  hipLaunchKernelGGL(k_bsr_block_multi, dim3(wg), dim3(256), 0, s, dd, nd);
  hipLaunchKernelGGL(k_bsr_sum_multi, dim3(nblocks(el)), dim3(256), 0, s, dd, nd, el);
  stage_end(kStagePrecond);
  ++pc_applies;
}

void pqn_ctx_impl::precond_apply(MvGroup& gr) {
  Level& lv = *gr.lv;
  Precond& pc = lv.pc;
  if (pc.epoch != config_epoch) throw Error(PQN_ERR_STATE, "internal: preconditioner not set up");
  hipStream_t s = stream;
  const int n = lv.n, n3 = 3 * n, M = lv.M, N = lv.N, K = gr.K;
  pc.vI.alloc((size_t)M * n3 * kMaxRhs);
  QPtrs vin{};
  OPtrs out{};
  for (int r = 0; r < K; ++r) {
    vin.p[r] = gr.in[r];
    out.p[r] = gr.out[r];
  }
  stage_begin(kStagePrecond);
  hipLaunchKernelGGL(k_pc_interleave, dim3(nblocks((long)M * n3 * K)), dim3(256), 0, s, vin, K, n, M, N, pc.vI.p);
  const int rchunks = (n3 + 255) / 256;
  const dim3 g(pc.nblk * rchunks);
  pc.part.alloc((size_t)pc.nblk * kMaxRhs * n3);
#define BSRK(KK) \
  hipLaunchKernelGGL(k_bsr_block<KK>, g, dim3(256), 0, s, pc.B16.p, pc.bscale.p, pc.bcol.p, pc.vI.p, n3, pc.ld, \
                     rchunks, pc.part.p)
  switch (K) {
    case 1: BSRK(1); break;
    case 2: BSRK(2); break;
    case 3: BSRK(3); break;
    case 4: BSRK(4); break;
    case 5: BSRK(5); break;
    default: BSRK(6); break;
  }
#undef BSRK
  hipLaunchKernelGGL(k_bsr_sum, dim3(nblocks((long)M * K * n3)), dim3(256), 0, s, pc.part.p, pc.bptr.p, K, n, M, N,
                     out);
  stage_end(kStagePrecond);
  ++pc_applies;
}

}  // namespace bipqn
