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
// Factorisation through harmonic coefficients. The near rule reads a density
// only through its coefficients coef = T q (the upsampled values and the
// foot-point expansion are both synthesised from them), so every near block is
// A_ij = Ac_ij (I3 x T) with Ac_ij [3n][3L]. With TD = (I3 x T) D^{-1} [3L][3n]
// (one matrix per grid) and R_ij = TD Ac_ij [3L][3L]:
//
//   sum_j A_ij D^{-1} A_ji = Q_i (I3 x T),  Q_i = sum_j Ac_ij R_ji,
//
// a correction of D of rank at most 3L, so (Sherman-Morrison-Woodbury)
//
//   S_i^{-1} = D^{-1} + E_i TD,  E_i = D^{-1} Q_i Y_i,  Y_i = (I - TD Q_i)^{-1} [3L][3L],
//
// and with w_j = TD v_j, the coefficient-space image of every sphere's input,
//
//   (P_r v)_i = D^{-1} v_i + E_i w_i - sum_j Gc_ij w_j,  Gc_ij = S_i^{-1} Ac_ij = D^{-1} Ac_ij + E_i R_ij.
//
// Set-up, once per configuration and level (at the first solve it applies to):
//   - D on the host from the self block and the rigid projection, D^{-1} by
//     Gauss-Jordan elimination with partial pivoting (once per grid and
//     process), TD by FP64 GEMMs (once per level);
//   - Ac_ij from the near stage of the operator (the same kernels as every
//     product) applied to unit harmonic-coefficient vectors, six at a time;
//   - R, Q_i, TD Q_i, E_i and Gc_ij by FP64 matrix-core GEMMs; Y_i by the
//     Newton-Schulz iteration Y <- Y (2I - K_i Y), K_i = I - TD Q_i, from Y = I
//     until every sphere's residual ||I - K_i Y||_F / sqrt(3L) is below kNsTol.
//     At Y = I the residual is TD Q_i, whose nonzero eigenvalues are those of
//     I - S_i D^{-1}: the iteration converges as one on S_i from D^{-1} would,
//     on matrices of (3L)^2 instead of (3n)^2 entries. A sphere still above
//     kNsKeep gets Y_i = 0, i.e. S_i^{-1} replaced by D^{-1} (block Jacobi for
//     that sphere).
// Application: w = TD v and y = D^{-1} v for all spheres and densities by one
// FP64 GEMM launch (the two matrices are shared by all spheres), then one
// block-sparse product over the E_i and Gc_ij (3n x 3L each) stored in FP16,
// each scaled by its largest magnitude (one FP32 factor per block). P_r is a
// fixed linear map either way, so GMRES keeps its convergence theory and the
// solution its accuracy; the rounding only perturbs the correction terms (the
// D^{-1} v part is exact FP64). Each application streams the blocks once from
// HBM ((M' + n_near) 3n 3L 2 bytes, M' the spheres with near partners: 0.5 GB
// at 216 spheres and 12x24 nodes), whatever the number of densities K.
//
// Layouts (3n = per-sphere unknowns, local index c n + x: component c, node x;
// 3L = coefficient unknowns, index d L + l):
//   Dinv [3n][3n] row-major, DinvT its transpose; TD [3L][3n] row-major;
//   Ac_ij, Gc_ij: by columns (column c' holds 3n rows), sphere i's slot s at
//   aco[i] + s 3n 3L; R: sphere i's [npart_i 3L][3L] by columns at rro[i], its
//   slot s holding R_(j s') = TD Ac_(j s') for the reverse (j, s') of (i, s);
//   Q, Z = D^{-1} Q, E: [M] x 3n x 3L by columns; K_i, Y, W: [M] x 3L x 3L by
//   columns; the FP16 blocks by columns padded to a multiple of 64 rows, sphere
//   i's row of blocks contiguous (E_i first); vC [K][M][3n] (column (r, j):
//   density r on sphere j), wI [M][3L][K], yI [M][3n][K].
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
// Ac_(i,s)(row, k0 + r) = near_part_r[s 3N + c N + i n + x], row = c n + x, stored by columns
// (aco[i] + (s ncol + k0 + r) 3n + row, ncol = 3L). Thread per (sphere, slot, row).
__global__ __launch_bounds__(256) void k_nb_scatter(OPtrs np, int K, int k0, int ncol, const int* __restrict__ npart,
                                                    const long* __restrict__ aco, int n, int M, int N,
                                                    double* __restrict__ Ac) {
  const int n3 = 3 * n;
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)M * kMaxNear * n3) return;
  const int row = (int)(e % n3);
  const int s = (int)((e / n3) % kMaxNear);
  const int i = (int)(e / ((long)n3 * kMaxNear));
  if (s >= npart[i]) return;
  const int c = row / n, x = row - c * n;
  double* dst = Ac + aco[i] + ((size_t)s * ncol + k0) * n3 + row;
  const size_t src = (size_t)s * 3 * N + (size_t)c * N + (size_t)i * n + x;
  for (int r = 0; r < K; ++r) dst[(size_t)r * n3] = np.p[r][src];
}

// The set-up's elementwise passes over [M][m][m] matrices by columns: one block per (sphere,
// column), threads along the column (no 64-bit index division per element).

// W <- dg I - W for every sphere.
__global__ __launch_bounds__(256) void k_diag_minus(double* __restrict__ W, int m, double dg) {
  const int col = blockIdx.x % m;
  double* w = W + (size_t)blockIdx.x * m;
  for (int r = threadIdx.x; r < m; r += 256) w[r] = (r == col ? dg : 0.0) - w[r];
}

// W <- I for every sphere.
__global__ __launch_bounds__(256) void k_eye(double* __restrict__ W, int m) {
  const int col = blockIdx.x % m;
  double* w = W + (size_t)blockIdx.x * m;
  for (int r = threadIdx.x; r < m; r += 256) w[r] = r == col ? 1.0 : 0.0;
}

// Partial sums of ||I - W_i||_F^2: block (i, g) covers the columns c = g, g + kNsSlices, ...
// of sphere i; res[i kNsSlices + g] (the host adds the slices in order).
constexpr int kNsSlices = 32;
__global__ __launch_bounds__(256) void k_ns_residual(const double* __restrict__ W, int m, double* __restrict__ res) {
  __shared__ double sh[256];
  const int i = blockIdx.x / kNsSlices, g = blockIdx.x % kNsSlices;
  const double* Wi = W + (size_t)i * m * m;
  double acc = 0.0;
  for (int c = g; c < m; c += kNsSlices)
    for (int r = threadIdx.x; r < m; r += 256) {
      const double d = (r == c ? 1.0 : 0.0) - Wi[(size_t)c * m + r];
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

// FP16 copies of FP64 blocks of rows x cols entries stored by columns: block b of the list is
// sgn[b] src[b] / scale[b] (entries in [-1, 1]; the product multiplies the scale back), each
// column padded with zeros to ld entries (a multiple of 64: every column starts on a 128-byte line).
__global__ __launch_bounds__(256) void k_blocks_f16(const double* const* __restrict__ src,
                                                    const double* __restrict__ sgn, const float* __restrict__ scale,
                                                    int rows, int cols, int ld, long nb, _Float16* __restrict__ dst) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  const long per = (long)cols * ld;
  if (e >= nb * per) return;
  const long b = e / per;
  const long l = e - b * per;
  const int m = (int)(l / ld), r = (int)(l - (long)m * ld);
  dst[e] = r < rows ? (_Float16)(float)(sgn[b] / scale[b] * src[b][(size_t)m * rows + r]) : (_Float16)0.0f;
}

// ------------------------------------------------------------ application kernels

// vC[(r M + j) 3n + m] = v_r[c N + j n + x], m = c n + x: every (density, sphere) a column.
__global__ __launch_bounds__(256) void k_pc_gather(QPtrs v, int K, int n, int M, int N, double* __restrict__ vC) {
  const int n3 = 3 * n;
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)K * M * n3) return;
  const int m = (int)(e % n3);
  const long rj = e / n3;
  const int j = (int)(rj % M), r = (int)(rj / M);
  const int c = m / n, x = m - c * n;
  vC[e] = v.p[r][(size_t)c * N + (size_t)j * n + x];
}

// part[(b K + r) 3n + row] = sum_m B_b(row, m) wI[(j 3L + m) K + r], j the column sphere of
// block b, m < 3L. Thread per (block, row): the block's columns are read by consecutive rows
// (coalesced), the coefficients of sphere j are wave-uniform (scalar loads). A workgroup per
// (block, 256 rows) gives the launch enough waves to keep the loads in flight that stream the
// blocks from HBM. FP16 blocks scaled to [-1, 1] (scale[b] multiplied back at the end), FP64
// products and sums.
template <int K>
__device__ __forceinline__ void bsr_block_body(const _Float16* __restrict__ B, const float* __restrict__ scale,
                                               const int* __restrict__ bcol, const double* __restrict__ wI,
                                               int n3, int nc, int ld, int rchunks, int wg, double* __restrict__ part) {
  const int b = wg / rchunks;
  const int row = (wg - b * rchunks) * 256 + threadIdx.x;
  const bool valid = row < n3;
  const int rr = valid ? row : n3 - 1;
  const _Float16* Bb = B + (size_t)b * nc * ld + rr;
  const double* v = wI + (size_t)bcol[b] * nc * K;
  double acc[K];
#pragma unroll
  for (int r = 0; r < K; ++r) acc[r] = 0.0;
#pragma unroll 8
  for (int m = 0; m < nc; ++m) {
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
                                                   const int* __restrict__ bcol, const double* __restrict__ wI,
                                                   int n3, int nc, int ld, int rchunks, double* __restrict__ part) {
  bsr_block_body<K>(B, scale, bcol, wI, n3, nc, ld, rchunks, blockIdx.x, part);
}

// out_r[c N + i n + x] = yI[(i 3n + row) K + r] + the partials of sphere i's blocks (in block
// order), row = c n + x.
__global__ __launch_bounds__(256) void k_pc_sum(const double* __restrict__ yI, const double* __restrict__ part,
                                                const int* __restrict__ bptr, int K, int n, int M, int N, OPtrs out) {
  const int n3 = 3 * n;
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)M * K * n3) return;
  const int row = (int)(e % n3);
  const int r = (int)((e / n3) % K);
  const int i = (int)(e / ((long)n3 * K));
  double v = yI[((size_t)i * n3 + row) * K + r];
  for (int b = bptr[i]; b < bptr[i + 1]; ++b) v += part[((size_t)b * K + r) * n3 + row];
  const int c = row / n, x = row - c * n;
  out.p[r][(size_t)c * N + (size_t)i * n + x] = v;
}

// Many suspensions in one launch (one density each): segment descriptors, workgroups
// [start, ...) of a segment for the block products, elements [estart, estart + M 3n)
// for the gather and the sum.
struct PcDesc {
  const _Float16* B;
  const float* scale;
  const int* bcol;
  const int* bptr;
  const double* in;
  double* out;
  double* vC;
  const double* wI;
  const double* yI;
  double* part;
  int n, N, M, nc, ld, rchunks, start;
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

__global__ __launch_bounds__(256) void k_pc_gather_multi(const PcDesc* __restrict__ d, int nd, long total) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const PcDesc D = d[pc_seg_elems(d, nd, e)];
  const long l = e - D.estart;
  const int n3 = 3 * D.n;
  const int j = (int)(l / n3), m = (int)(l - (long)j * n3);
  const int c = m / D.n, x = m - c * D.n;
  D.vC[l] = D.in[(size_t)c * D.N + (size_t)j * D.n + x];
}

__global__ __launch_bounds__(256) void k_bsr_block_multi(const PcDesc* __restrict__ d, int nd) {
  const PcDesc D = d[pc_seg_blocks(d, nd, blockIdx.x)];
  bsr_block_body<1>(D.B, D.scale, D.bcol, D.wI, 3 * D.n, D.nc, D.ld, D.rchunks, blockIdx.x - D.start, D.part);
}

__global__ __launch_bounds__(256) void k_pc_sum_multi(const PcDesc* __restrict__ d, int nd, long total) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const PcDesc D = d[pc_seg_elems(d, nd, e)];
  const long l = e - D.estart;
  const int n3 = 3 * D.n;
  const int i = (int)(l / n3), row = (int)(l - (long)i * n3);
  double v = D.yI[l];
  for (int b = D.bptr[i]; b < D.bptr[i + 1]; ++b) v += D.part[(size_t)b * n3 + row];
  const int c = row / D.n, x = row - c * D.n;
  D.out[(size_t)c * D.N + (size_t)i * D.n + x] = v;
}

// ------------------------------------------------- coarse level (precond_coarse)

// Coarse far-source grids, whatever the discretisation (their error is that of integrating
// the far kernel against degree <= 2 densities, set by the geometry): far pairs whose centres
// are closer than kCoarseClose radii on kCoarseThetaClose x 2 kCoarseThetaClose nodes, the
// others on kCoarseTheta x 2 kCoarseTheta. One grid for all far pairs, at 216 spheres and
// 12x24: 3x6 gives 11.0 GMRES iterations per MVP, 4x8 10.0, 5x10 9.5, 6x12 9.25 (the
// six-force-set pass 59.1, 56.0, 56.3 and 58.2 ms): the closest far pairs carry most of the
// coarse operator's error, and the distant ones, most of its cost.
constexpr int kCoarseTheta = 3;
constexpr int kCoarseThetaClose = 6;
constexpr double kCoarseClose = 3.5;
// Newton-Schulz stop for inv(E): it only shapes the preconditioner (at 216 spheres 1e-2 and
// 1e-4 give the same 10.0 iterations per MVP; 1e-2 takes 7 instead of 10 GEMMs of (27 M)^3)
constexpr double kCoarseTol = 1e-2;
constexpr double kCoarseWarm = 0.5;    // largest residual of the previous inverse used as the start
constexpr double kCoarseKeep = 1e-1;   // above this after the last step the coarse level stays off
constexpr int kCoarseMaxSteps = 12;
constexpr int kCmvCols = 256;          // columns of inv(E) per workgroup of the coarse product

// NL[(g 27 + c 9 + k) 3n + row] = column c L + k of the coefficient near block of slot g (at
// acs[g]): A_ij Z = Ac_ij (I3 x T) Z picks the coefficient columns of the degree <= 2
// harmonics (T Z = I on them).
__global__ __launch_bounds__(256) void k_low_cols(const double* __restrict__ Ac, const long* __restrict__ acs,
                                                  int nslots, int n3, int L, double* __restrict__ NL) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)nslots * kCoarseB * n3) return;
  const int row = (int)(e % n3);
  const long gb = e / n3;
  const int b = (int)(gb % kCoarseB), g = (int)(gb / kCoarseB);
  const int c = b / kCoarseL, k = b - c * kCoarseL;
  NL[e] = Ac[acs[g] + ((size_t)c * L + k) * n3 + row];
}

// The diagonal blocks of E (by columns): E(i 27 + b', i 27 + b) = ES(b', b) for every sphere.
__global__ __launch_bounds__(256) void k_eself_fill(const double* __restrict__ ES, int M, long Mc,
                                                    double* __restrict__ E) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)M * kCoarseB * kCoarseB) return;
  const int i = (int)(e / (kCoarseB * kCoarseB)), q = (int)(e % (kCoarseB * kCoarseB));
  const int b = q / kCoarseB, bp = q - b * kCoarseB;
  E[((size_t)i * kCoarseB + b) * Mc + (size_t)i * kCoarseB + bp] = ES[q];
}

// X = blockdiag(X0) by columns (the Newton-Schulz start).
__global__ __launch_bounds__(256) void k_blockdiag(const double* __restrict__ X0, long Mc, double* __restrict__ X) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= Mc * Mc) return;
  const long col = e / Mc, r = e - col * Mc;
  X[e] = (r / kCoarseB == col / kCoarseB) ? X0[(col % kCoarseB) * kCoarseB + r % kCoarseB] : 0.0;
}

// res[col] = sum over the rows of column col of (I - W)^2 (W by columns; the host adds the
// columns in order).
__global__ __launch_bounds__(256) void k_col_residual(const double* __restrict__ W, long m, double* __restrict__ res) {
  __shared__ double sh[256];
  const long col = blockIdx.x;
  const double* w = W + col * m;
  double acc = 0.0;
  for (long r = threadIdx.x; r < m; r += 256) {
    const double d = (r == col ? 1.0 : 0.0) - w[r];
    acc = fma(d, d, acc);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) res[col] = sh[0];
}

__global__ __launch_bounds__(256) void k_to_f32(const double* __restrict__ x, long len, float* __restrict__ y) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e < len) y[e] = (float)x[e];
}

// Far blocks of E: for every far pair (i, j), E(i 27 + c' 9 + k', j 27 + c 9 + k) =
// sum_x T(k', x) u_c'(x) with u the far double layer at sphere i's node x of the density
// e_c Y_k on sphere j, summed on the coarse source grid (offsets offc, weights wc, harmonics
// Yc): u_c'(x) = s sum_f (r.o_f) / |r|^5 r_c' r_c wc_f Y_k(f), r = x - y_f, s = 3 / (4 pi a).
// Workgroup per sphere pair, thread per target (64 ceil(n / 64) threads): the six products
// r_c r_c' (symmetric) x nine harmonics are accumulated per target; the projection on the
// nine analysis rows goes through LDS, a third of the 54 sums at a time (each output a dot
// product over the targets in a fixed order).
constexpr int kCfbMaxWaves = 8;  // one target per thread: n <= 512 nodes per sphere
constexpr int kCfbChunk = 18;    // u values per target staged in LDS at a time (54 = 3 x 18)
__global__ __launch_bounds__(64 * kCfbMaxWaves) void k_coarse_far_blocks(const double* __restrict__ ctr,
                                                                         const double* __restrict__ off,
                                                                         const unsigned char* __restrict__ cls,
                                                                         const unsigned char* __restrict__ t1,
                                                                         const double* __restrict__ offc,
                                                                         const double* __restrict__ wc,
                                                                         const double* __restrict__ Yc,
                                                                         const double* __restrict__ Tlow, int n,
                                                                         int ncs_all, int ncs1, int M, double a,
                                                                         double* __restrict__ E) {
  constexpr int NP = 6, NV = NP * kCoarseL;  // 54 per target
  // dynamic LDS: source positions (rel. c_i) and offsets [nmax][6], s wc Y_k [nmax][9], staged
  // u [blockDim][kCfbChunk + 1] (padded rows); nmax the larger grid's node count
  extern __shared__ double lds_cfb[];
  const int nmax = max(ncs1, ncs_all - ncs1);
  double(*sy)[6] = reinterpret_cast<double(*)[6]>(lds_cfb);
  double(*swy)[kCoarseL] = reinterpret_cast<double(*)[kCoarseL]>(lds_cfb + 6 * nmax);
  double(*su)[kCfbChunk + 1] = reinterpret_cast<double(*)[kCfbChunk + 1]>(lds_cfb + (6 + kCoarseL) * nmax);
  const int i = blockIdx.x / M, j = blockIdx.x - (blockIdx.x / M) * M;
  if (i == j || cls[(size_t)i * M + j] != 0) return;  // uniform over the block
  // the pair's grid: the first ncs1 nodes of the tables (close pairs) or the rest
  const int f0 = t1[(size_t)i * M + j] == 0 ? 0 : ncs1;
  const int ncs = f0 == 0 ? ncs1 : ncs_all - ncs1;
  offc += 3 * f0;
  wc += f0;
  Yc += (size_t)f0 * kCoarseL;
  const int t = threadIdx.x;
  const double dx = ctr[3 * j] - ctr[3 * i], dy = ctr[3 * j + 1] - ctr[3 * i + 1], dz = ctr[3 * j + 2] - ctr[3 * i + 2];
  const double s = 3.0 / (4.0 * kPi * a);
  for (int f = t; f < ncs; f += blockDim.x) {
    sy[f][0] = dx + offc[3 * f];
    sy[f][1] = dy + offc[3 * f + 1];
    sy[f][2] = dz + offc[3 * f + 2];
    sy[f][3] = offc[3 * f];
    sy[f][4] = offc[3 * f + 1];
    sy[f][5] = offc[3 * f + 2];
    for (int k = 0; k < kCoarseL; ++k) swy[f][k] = s * wc[f] * Yc[f * kCoarseL + k];
  }
  __syncthreads();
  const bool valid = t < n;
  const int xx = valid ? t : n - 1;
  const double Xx = off[3 * xx], Xy = off[3 * xx + 1], Xz = off[3 * xx + 2];
  double u[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) u[q] = 0.0;
  for (int f = 0; f < ncs; ++f) {
    const double rx = Xx - sy[f][0], ry = Xy - sy[f][1], rz = Xz - sy[f][2];
    const double r2 = rx * rx + ry * ry + rz * rz;
    const double ri = 1.0 / sqrt(r2);
    const double ri2 = ri * ri;
    const double g = (rx * sy[f][3] + ry * sy[f][4] + rz * sy[f][5]) * ri * ri2 * ri2;
    const double tp[NP] = {g * rx * rx, g * rx * ry, g * rx * rz, g * ry * ry, g * ry * rz, g * rz * rz};
#pragma unroll
    for (int k = 0; k < kCoarseL; ++k) {
      const double wy = swy[f][k];
#pragma unroll
      for (int p = 0; p < NP; ++p) u[p * kCoarseL + k] = fma(tp[p], wy, u[p * kCoarseL + k]);
    }
  }
  const size_t Mc = (size_t)M * kCoarseB;
#pragma unroll
  for (int ch = 0; ch < NV / kCfbChunk; ++ch) {
#pragma unroll
    for (int q = 0; q < kCfbChunk; ++q) su[t][q] = valid ? u[ch * kCfbChunk + q] : 0.0;
    __syncthreads();
    // outputs (k', q) of this chunk: 9 x 18 dot products over the targets
    for (int o = t; o < kCoarseL * kCfbChunk; o += blockDim.x) {
      const int kp = o / kCfbChunk, q = o - kp * kCfbChunk;
      const double* tr = Tlow + (size_t)kp * n;
      double v = 0.0;
      for (int x = 0; x < n; ++x) v = fma(tr[x], su[x][q], v);
      const int pk = ch * kCfbChunk + q, p = pk / kCoarseL, k = pk - p * kCoarseL;
      // p -> (c, c'): 0 xx, 1 xy, 2 xz, 3 yy, 4 yz, 5 zz
      const int ca = p < 3 ? 0 : (p < 5 ? 1 : 2);
      const int cb = p < 3 ? p : (p < 5 ? p - 2 : 2);
      E[((size_t)j * kCoarseB + cb * kCoarseL + k) * Mc + (size_t)i * kCoarseB + ca * kCoarseL + kp] = v;
      if (ca != cb) E[((size_t)j * kCoarseB + ca * kCoarseL + k) * Mc + (size_t)i * kCoarseB + cb * kCoarseL + kp] = v;
    }
    __syncthreads();  // su is rewritten by the next chunk
  }
}

// cpart[(h Mc + r) K + k] = sum over the columns m of chunk h of inv(E)(r, m) cr[m K + k]
// (inv(E) in FP32 by columns: consecutive rows read consecutive words; cr wave-uniform).
template <int K>
__global__ __launch_bounds__(256) void k_coarse_mv(const float* __restrict__ Ei, const double* __restrict__ cr,
                                                   int Mc, double* __restrict__ cpart) {
  const int r = blockIdx.x * 256 + threadIdx.x, h = blockIdx.y;
  const bool valid = r < Mc;
  const int rr = valid ? r : Mc - 1;
  const int m0 = h * kCmvCols, m1 = min(Mc, m0 + kCmvCols);
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
#pragma unroll 4
  for (int m = m0; m < m1; ++m) {
    const double e = (double)Ei[(size_t)m * Mc + rr];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = fma(e, cr[(size_t)m * K + k], acc[k]);
  }
  if (valid)
#pragma unroll
    for (int k = 0; k < K; ++k) cpart[((size_t)h * Mc + r) * K + k] = acc[k];
}

// ccI[r K + k] = sum over the chunks (in order); ccC[(k M + j) 27 + b] the same, r = j 27 + b.
__global__ __launch_bounds__(256) void k_coarse_mv_sum(const double* __restrict__ cpart, int nh, int Mc, int M, int K,
                                                       double* __restrict__ ccI, double* __restrict__ ccC) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)Mc * K) return;
  const int r = (int)(e / K), k = (int)(e - (long)r * K);
  double v = 0.0;
  for (int h = 0; h < nh; ++h) v += cpart[((size_t)h * Mc + r) * K + k];
  ccI[e] = v;
  const int j = r / kCoarseB, b = r - j * kCoarseB;
  ccC[((size_t)k * M + j) * kCoarseB + b] = v;
}

// qc[(j ncs + f) 3K + 3k + c] = sum_l Yc(f, l) ccI[(j 27 + c 9 + l) K + k]: the coarse density
// at the coarse far-source nodes, in the layout of the far source packing.
__global__ __launch_bounds__(256) void k_coarse_qc(const double* __restrict__ Yc, const double* __restrict__ ccI,
                                                   int ncs, int M, int K, double* __restrict__ qc) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  const int K3 = 3 * K;
  if (e >= (long)M * ncs * K3) return;
  const int q = (int)(e % K3);
  const long jf = e / K3;
  const int f = (int)(jf % ncs), j = (int)(jf / ncs);
  const int k = q / 3, c = q - 3 * k;
  double v = 0.0;
#pragma unroll
  for (int l = 0; l < kCoarseL; ++l)
    v = fma(Yc[f * kCoarseL + l], ccI[((size_t)j * kCoarseB + c * kCoarseL + l) * K + k], v);
  qc[e] = v;
}

// vC[(k M + i) 3n + m] -= (A~ z1) at node m of sphere i: the coarse block partials (self and
// near) and the far partials of the coarse far sum (nchunks each), m = c n + x.
__global__ __launch_bounds__(256) void k_coarse_resid(double* __restrict__ vC, const double* __restrict__ bpart,
                                                      const int* __restrict__ bptr, OPtrs far, int nchunks, int K,
                                                      int n, int M, int N) {
  const int n3 = 3 * n;
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)K * M * n3) return;
  const int m = (int)(e % n3);
  const long ki = e / n3;
  const int i = (int)(ki % M), k = (int)(ki / M);
  const int c = m / n, x = m - c * n;
  double v = 0.0;
  for (int b = bptr[i]; b < bptr[i + 1]; ++b) v += bpart[((size_t)b * K + k) * n3 + m];
  for (int h = 0; h < nchunks; ++h) v += far.p[k][(size_t)h * 3 * N + (size_t)c * N + (size_t)i * n + x];
  vC[e] -= v;
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

// The application's GEMMs for K = 1 .. kMaxRhs densities over the level's fixed buffers
// (vC columns (r, j) = (r M + j), yI[(j 3n + m) K + r], wI[(j 3L + l) K + r]), three
// descriptors each: y = D^{-1} v and w = TD v for one launch, and w alone (for a launch
// of its own while y runs on the side stream).
static void build_apply_descs(Precond& pc, int n3, int nc, int M, hipStream_t s) {
  pc.adesc_h.clear();
  for (int K = 1; K <= kMaxRhs; ++K) {
    int blocks = 0;
    push_gemm(pc.adesc_h, blocks, n3, K * M, n3, pc.Dinv.p, n3, pc.vC.p, n3, pc.yI.p, n3, 0, n3 * K, K, M, 1, 0, 1);
    pc.aty[K - 1] = blocks;
    push_gemm(pc.adesc_h, blocks, nc, K * M, n3, pc.TD.p, n3, pc.vC.p, n3, pc.wI.p, nc, 0, nc * K, K, M, 1, 0, 1);
    pc.atw[K - 1] = blocks - pc.aty[K - 1];
    blocks = 0;
    push_gemm(pc.adesc_h, blocks, nc, K * M, n3, pc.TD.p, n3, pc.vC.p, n3, pc.wI.p, nc, 0, nc * K, K, M, 1, 0, 1);
  }
  pc.adesc.upload(pc.adesc_h.data(), pc.adesc_h.size(), s);
}

void pqn_ctx_impl::precond_setup(Level& lv) {
  Precond& pc = lv.pc;
  if (!cfg.precond || pc.epoch == config_epoch) return;
  TraceRange trace("precond_setup");
  HIPCHK(hipStreamSynchronize(stream));
  Timer tm;
  hipStream_t s = stream;
  const int n = lv.n, n3 = 3 * n, M = lv.M, N = lv.N, L = lv.L, nc = 3 * L;
  const size_t nn = (size_t)n3 * n3, ncn = (size_t)nc * n3, ncc = (size_t)nc * nc;
  if (!pc.has_d) {
    const SphereBlock& sb = sphere_block_cached(lv.tab);
    pc.Dinv.upload(sb.Dinv.data(), nn, s);
    pc.DinvT.upload(sb.DinvT.data(), nn, s);
    std::vector<double> tt((size_t)n * L);  // T by columns
    for (int l = 0; l < L; ++l)
      for (int m = 0; m < n; ++m) tt[(size_t)m * L + l] = lv.tab.T[(size_t)l * n + m];
    pc.TT.upload(tt.data(), tt.size(), s);
    // TD(d L + l, :) = sum_x T(l, x) D^{-1}(d n + x, :), row-major
    pc.TD.alloc(ncn);
    std::vector<GemmDesc> gd;
    int ngd = 0;
    for (int d = 0; d < 3; ++d)
      push_gemm(gd, ngd, L, n3, n, pc.TT.p, L, pc.DinvT.p + (size_t)d * n, n3, pc.TD.p + (size_t)d * L * n3, L, 0, 1,
                n3, n3, 0, 1, 1);
    DescPack dd;
    const size_t od = dd.add(gd);
    char* db = push_desc_pack(dd.host);
    launch_gemm64_multi_big(s, (const GemmDesc*)(db + od), (int)gd.size(), ngd);
    pc.vC.alloc((size_t)kMaxRhs * M * n3);
    pc.yI.alloc((size_t)M * n3 * kMaxRhs);
    pc.wI.alloc((size_t)M * nc * kMaxRhs);
    build_apply_descs(pc, n3, nc, M, s);
    HIPCHK(hipStreamSynchronize(s));  // the descriptor staging is reused after this
    pc.has_d = true;
  }
  pc.fallback = 0;
  pc.ns_iters = 0;
  pc.aco.assign(M, 0);
  pc.rro.assign(M, 0);
  long tota = 0, totr = 0;
  int nslots = 0;
  for (int i = 0; i < M; ++i) {
    pc.aco[i] = tota;
    pc.rro[i] = totr;
    tota += (long)h_npart[i] * ncn;
    totr += (long)h_npart[i] * ncc;
    nslots += h_npart[i];
  }
  // rev[i kMaxNear + s]: the slot of sphere i in the list of its partner in slot s
  std::vector<int> rev((size_t)M * kMaxNear, -1);
  for (int i = 0; i < M; ++i)
    for (int sl = 0; sl < h_npart[i]; ++sl) {
      const int j = h_partners[(size_t)i * kMaxNear + sl];
      for (int q = 0; q < h_npart[j]; ++q)
        if (h_partners[(size_t)j * kMaxNear + q] == i) rev[(size_t)i * kMaxNear + sl] = q;
      if (rev[(size_t)i * kMaxNear + sl] < 0) throw Error(PQN_ERR_STATE, "internal: near pair list is not symmetric");
    }
  if (nslots > 0) {
    pc.Ac.alloc((size_t)tota);
    pc.Gc.alloc((size_t)tota);
    pc.Rr.alloc((size_t)totr);
    DevArray<long> daco;
    daco.upload(pc.aco.data(), pc.aco.size(), s);
    // Ac from unit coefficient columns through the near stage (3L / 6 passes)
    for (int k0 = 0; k0 < nc; k0 += kMaxRhs) {
      const int K = std::min(kMaxRhs, nc - k0);
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
      hipLaunchKernelGGL(k_nb_scatter, dim3(nblocks((long)M * kMaxNear * n3)), dim3(256), 0, s, np, K, k0, nc,
                         npart.p, daco.p, n, M, N, pc.Ac.p);
    }
    // R: slot s of sphere i holds TD Ac_(j, s'), (j, s') the reverse of (i, s); then
    // Q_i = sum_s Ac_(i,s) R-slot s over the concatenated slots (a sphere without
    // partners gets Q_i = 0: a product with no terms writes zeros)
    pc.Q.alloc((size_t)M * ncn);
    std::vector<GemmDesc> gr, gq;
    int ngr = 0, ngq = 0;
    for (int i = 0; i < M; ++i) {
      const int ns = h_npart[i];
      for (int sl = 0; sl < ns; ++sl) {
        const int j = h_partners[(size_t)i * kMaxNear + sl], sj = rev[(size_t)i * kMaxNear + sl];
        push_gemm(gr, ngr, nc, nc, n3, pc.TD.p, n3, pc.Ac.p + pc.aco[j] + (size_t)sj * ncn, n3,
                  pc.Rr.p + pc.rro[i] + (size_t)sl * nc, nc, 0, ns * nc, 1, nc, 0, 0, 1);
      }
      push_gemm(gq, ngq, n3, nc, ns * nc, ns ? pc.Ac.p + pc.aco[i] : pc.TD.p, n3, ns ? pc.Rr.p + pc.rro[i] : pc.TD.p,
                std::max(ns * nc, 1), pc.Q.p + (size_t)i * ncn, n3, 0, n3, 1, nc, 0, 1, 1);
    }
    DescPack dp;
    const size_t orr = dp.add(gr), oq = dp.add(gq);
    char* base = push_desc_pack(dp.host);
    launch_gemm64_multi_big(s, (const GemmDesc*)(base + orr), (int)gr.size(), ngr);
    launch_gemm64_multi_big(s, (const GemmDesc*)(base + oq), (int)gq.size(), ngq);
    // K_i = I - TD Q_i (by columns)
    pc.Kc.alloc((size_t)M * ncc);
    launch_gemm64_big(s, nc, nc, n3, pc.TD.p, n3, 0, pc.Q.p, (long)ncn, n3, pc.Kc.p, (long)ncc, nc, 0, nc, M, 0);
    hipLaunchKernelGGL(k_diag_minus, dim3(M * nc), dim3(256), 0, s, pc.Kc.p, nc, 1.0);
    // Newton-Schulz from Y = I
    pc.Y.alloc((size_t)M * ncc);
    pc.Y2.alloc((size_t)M * ncc);
    pc.W.alloc((size_t)M * ncc);
    pc.res.alloc((size_t)M * kNsSlices);
    hipLaunchKernelGGL(k_eye, dim3(M * nc), dim3(256), 0, s, pc.Y.p, nc);
    std::vector<double> res(M), resp((size_t)M * kNsSlices);
    for (int step = 0;; ++step) {
      // W = K Y: C(r, c) = sum_k K(r, k) Y(k, c), K read by columns
      launch_gemm64_big(s, nc, nc, nc, pc.Kc.p, nc, (long)ncc, pc.Y.p, (long)ncc, nc, pc.W.p, (long)ncc, nc, 0, nc, M,
                        1);
      hipLaunchKernelGGL(k_ns_residual, dim3(M * kNsSlices), dim3(256), 0, s, pc.W.p, nc, pc.res.p);
      HIPCHK(hipMemcpyAsync(resp.data(), pc.res.p, resp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (int i = 0; i < M; ++i) {
        double t = 0.0;
        for (int g = 0; g < kNsSlices; ++g) t += resp[(size_t)i * kNsSlices + g];
        res[i] = t / nc;
      }
      double worst = 0.0;
      for (double v : res) worst = std::isfinite(v) ? std::max(worst, std::sqrt(v)) : 1e300;
      if (worst <= kNsTol || step == kNsMaxSteps) break;
      // Y <- Y (2I - W): C(r, c) = sum_k Y(r, k) F(k, c), Y read by columns
      hipLaunchKernelGGL(k_diag_minus, dim3(M * nc), dim3(256), 0, s, pc.W.p, nc, 2.0);
      launch_gemm64_big(s, nc, nc, nc, pc.Y.p, nc, (long)ncc, pc.W.p, (long)ncc, nc, pc.Y2.p, (long)ncc, nc, 0, nc, M,
                        1);
      std::swap(pc.Y.p, pc.Y2.p);
      ++pc.ns_iters;
    }
    for (int i = 0; i < M; ++i)
      if (!(std::sqrt(res[i]) <= kNsKeep)) {
        HIPCHK(hipMemsetAsync(pc.Y.p + (size_t)i * ncc, 0, ncc * sizeof(double), s));
        ++pc.fallback;
      }
    // Z = D^{-1} Q_i, E_i = Z_i Y_i (by columns)
    pc.Z.alloc((size_t)M * ncn);
    pc.E.alloc((size_t)M * ncn);
    launch_gemm64_big(s, n3, nc, n3, pc.Dinv.p, n3, 0, pc.Q.p, (long)ncn, n3, pc.Z.p, (long)ncn, n3, 0, n3, M, 0);
    launch_gemm64_big(s, n3, nc, nc, pc.Z.p, n3, (long)ncn, pc.Y.p, (long)ncc, nc, pc.E.p, (long)ncn, n3, 0, n3, M, 1);
    // Gc_(i,s) = D^{-1} Ac_(i,s), then += E_i R_(i,s); R_(i,s) = TD Ac_(i,s) is slot s' of
    // partner j's R
    std::vector<GemmDesc> ga, gb;
    int nga = 0, ngb = 0;
    for (int i = 0; i < M; ++i)
      for (int sl = 0; sl < h_npart[i]; ++sl) {
        const int j = h_partners[(size_t)i * kMaxNear + sl], sj = rev[(size_t)i * kMaxNear + sl];
        double* gcb = pc.Gc.p + pc.aco[i] + (size_t)sl * ncn;
        push_gemm(ga, nga, n3, nc, n3, pc.Dinv.p, n3, pc.Ac.p + pc.aco[i] + (size_t)sl * ncn, n3, gcb, n3, 0, n3, 1,
                  nc, 0, 0, 1);
        push_gemm(gb, ngb, n3, nc, nc, pc.E.p + (size_t)i * ncn, n3, pc.Rr.p + pc.rro[j] + (size_t)sj * nc,
                  h_npart[j] * nc, gcb, n3, 0, n3, 1, nc, 0, 1 | 2, 1);
      }
    DescPack dq;
    const size_t oa = dq.add(ga), ob = dq.add(gb);
    char* qb = push_desc_pack(dq.host);
    launch_gemm64_multi_big(s, (const GemmDesc*)(qb + oa), (int)ga.size(), nga);
    launch_gemm64_multi_big(s, (const GemmDesc*)(qb + ob), (int)gb.size(), ngb);
    HIPCHK(hipStreamSynchronize(s));  // daco and the descriptor tables are released/reused after this
  }
  // block rows in FP16: sphere i (if it has near partners) holds E_i, then -Gc_(i,s) for its slots
  {
    std::vector<int> bp(M + 1, 0), bc;
    std::vector<const double*> src;
    std::vector<double> sg;
    for (int i = 0; i < M; ++i) {
      bp[i] = (int)bc.size();
      if (h_npart[i] == 0) continue;
      bc.push_back(i);
      src.push_back(pc.E.p + (size_t)i * ncn);
      sg.push_back(1.0);
      for (int sl = 0; sl < h_npart[i]; ++sl) {
        bc.push_back(h_partners[(size_t)i * kMaxNear + sl]);
        src.push_back(pc.Gc.p + pc.aco[i] + (size_t)sl * ncn);
        sg.push_back(-1.0);
      }
    }
    bp[M] = (int)bc.size();
    const long nb = (long)bc.size();
    pc.nblk = (int)nb;
    pc.ld = (n3 + 63) / 64 * 64;
    pc.bptr.upload(bp.data(), bp.size(), s);
    if (nb > 0) {
      pc.B16.alloc((size_t)nb * nc * pc.ld);
      pc.bscale.alloc((size_t)nb);
      pc.bcol.upload(bc.data(), bc.size(), s);
      pc.part.alloc((size_t)nb * kMaxRhs * n3);
      DevArray<const double*> dsrc;
      DevArray<double> dsg;
      dsrc.upload(src.data(), src.size(), s);
      dsg.upload(sg.data(), sg.size(), s);
      hipLaunchKernelGGL(k_block_absmax, dim3(nb), dim3(256), 0, s, dsrc.p, (long)ncn, pc.bscale.p);
      hipLaunchKernelGGL(k_blocks_f16, dim3(nblocks(nb * (long)nc * pc.ld)), dim3(256), 0, s, dsrc.p, dsg.p,
                         pc.bscale.p, n3, nc, pc.ld, nb, pc.B16.p);
    }
    HIPCHK(hipStreamSynchronize(s));  // dsrc and the host tables are released after this
  }
  if (cfg.precond_coarse)
    coarse_setup(lv);
  else
    pc.co.on = false;
  HIPCHK(hipGetLastError());
  pc.epoch = config_epoch;
  pc.setup_ms = tm.ms();
  pc_setup_ms += pc.setup_ms;
  pc_fallback += pc.fallback;
}

// ------------------------------------------------- coarse level (precond_coarse): set-up

// Tables of the level (once): R, Z, D Z, R D Z and its inverse, the analysis rows of the
// degree <= 2 harmonics, the coarse far-source grid, and the application's GEMM descriptors
// (R v; y += Z c) for K = 1 .. kMaxRhs.
void pqn_ctx_impl::coarse_tables(Level& lv) {
  CoarsePc& co = lv.pc.co;
  if (co.tab) return;
  hipStream_t s = stream;
  const SphereTables& t = lv.tab;
  const int n = lv.n, n3 = 3 * n, M = lv.M, Mc = kCoarseB * M;
  const double a = t.radius;
  if (t.L < kCoarseL) throw Error(PQN_ERR_INVALID, "precond_coarse needs n_theta >= 3");
  // Y_k(x) = T(k, x) / (w(x) / a^2) (the analysis is the synthesis times the unit-sphere weights)
  std::vector<double> R((size_t)kCoarseB * n3, 0.0), Z((size_t)n3 * kCoarseB, 0.0), Tl((size_t)kCoarseL * n);
  for (int k = 0; k < kCoarseL; ++k)
    for (int x = 0; x < n; ++x) {
      const double tk = t.T[(size_t)k * n + x];
      Tl[(size_t)k * n + x] = tk;
      for (int c = 0; c < 3; ++c) {
        R[(size_t)(c * kCoarseL + k) * n3 + c * n + x] = tk;
        Z[(size_t)(c * n + x) * kCoarseB + c * kCoarseL + k] = tk / (t.w[x] / (a * a));
      }
    }
  const SphereBlock& sb = sphere_block_cached(t);
  std::vector<double> DZ((size_t)kCoarseB * n3, 0.0), ES((size_t)kCoarseB * kCoarseB, 0.0);
  for (int b = 0; b < kCoarseB; ++b)
    for (int r = 0; r < n3; ++r) {
      double v = 0.0;
      for (int m = 0; m < n3; ++m) v += sb.D[(size_t)r * n3 + m] * Z[(size_t)m * kCoarseB + b];
      DZ[(size_t)b * n3 + r] = v;
    }
  for (int b = 0; b < kCoarseB; ++b)
    for (int bp = 0; bp < kCoarseB; ++bp) {
      double v = 0.0;
      for (int r = 0; r < n3; ++r) v += R[(size_t)bp * n3 + r] * DZ[(size_t)b * n3 + r];
      ES[(size_t)b * kCoarseB + bp] = v;
    }
  std::vector<double> X0r((size_t)kCoarseB * kCoarseB), X0((size_t)kCoarseB * kCoarseB);
  for (int b = 0; b < kCoarseB; ++b)
    for (int bp = 0; bp < kCoarseB; ++bp) X0r[(size_t)bp * kCoarseB + b] = ES[(size_t)b * kCoarseB + bp];
  invert_gauss_jordan(X0r, kCoarseB);  // row-major inverse of R D Z
  for (int b = 0; b < kCoarseB; ++b)
    for (int bp = 0; bp < kCoarseB; ++bp) X0[(size_t)b * kCoarseB + bp] = X0r[(size_t)bp * kCoarseB + b];
  // the two coarse grids' tables, close grid first: offsets [ncs][3], weights [ncs], Y [ncs][9]
  std::vector<double> oc, wcv, Yc;
  coarse_sh_grid(kCoarseThetaClose, 2 * kCoarseThetaClose, a, 2, oc, wcv, Yc);
  {
    std::vector<double> oc2, wc2, Yc2;
    coarse_sh_grid(kCoarseTheta, 2 * kCoarseTheta, a, 2, oc2, wc2, Yc2);
    oc.insert(oc.end(), oc2.begin(), oc2.end());
    wcv.insert(wcv.end(), wc2.begin(), wc2.end());
    Yc.insert(Yc.end(), Yc2.begin(), Yc2.end());
  }
  co.ncs1 = 2 * kCoarseThetaClose * kCoarseThetaClose;
  co.ncs = co.ncs1 + 2 * kCoarseTheta * kCoarseTheta;
  co.R.upload(R.data(), R.size(), s);
  co.Z.upload(Z.data(), Z.size(), s);
  co.DZ.upload(DZ.data(), DZ.size(), s);
  co.Tlow.upload(Tl.data(), Tl.size(), s);
  co.ES.upload(ES.data(), ES.size(), s);
  co.X0.upload(X0.data(), X0.size(), s);
  co.offc.upload(oc.data(), oc.size(), s);
  co.wc.upload(wcv.data(), wcv.size(), s);
  co.Yc.upload(Yc.data(), Yc.size(), s);
  co.cr.alloc((size_t)Mc * kMaxRhs);
  co.ccI.alloc((size_t)Mc * kMaxRhs);
  co.ccC.alloc((size_t)Mc * kMaxRhs);
  co.cpart.alloc((size_t)((Mc + kCmvCols - 1) / kCmvCols) * Mc * kMaxRhs);
  co.qc.alloc((size_t)M * co.ncs * 3 * kMaxRhs);
  co.src.alloc((size_t)M * co.ncs * src64_stride(kMaxRhs));
  std::vector<GemmDesc> d;
  for (int K = 1; K <= kMaxRhs; ++K) {
    int blocks = 0;
    push_gemm(d, blocks, kCoarseB, K * M, n3, co.R.p, n3, lv.pc.vC.p, n3, co.cr.p, kCoarseB, 0, kCoarseB * K, K, M, 1,
              0, 1);
    co.tr[K - 1] = blocks;
    blocks = 0;
    push_gemm(d, blocks, n3, K * M, kCoarseB, co.Z.p, kCoarseB, co.ccC.p, kCoarseB, lv.pc.yI.p, n3, 0, n3 * K, K, M,
              1, 2, 1);
    co.tz[K - 1] = blocks;
  }
  co.desc.upload(d.data(), d.size(), s);
  HIPCHK(hipStreamSynchronize(s));
  co.tab = true;
}

// Per configuration (after the near-patch set-up; Ac still holds the coefficient near blocks):
// the FP16 blocks of A~ Z restricted to self and near pairs, E = R A~ Z, inv(E) by Newton-Schulz.
void pqn_ctx_impl::coarse_setup(Level& lv) {
  Precond& pc = lv.pc;
  CoarsePc& co = pc.co;
  co.on = false;
  coarse_tables(lv);
  hipStream_t s = stream;
  const int n = lv.n, n3 = 3 * n, M = lv.M, L = lv.L, nc = 3 * L;
  const long Mc = (long)kCoarseB * M;
  const size_t ncn = (size_t)nc * n3;
  // which far pairs take the close grid (centres closer than kCoarseClose radii)
  {
    std::vector<unsigned char> t1((size_t)M * M, 1), t2((size_t)M * M, 1);
    for (int i = 0; i < M; ++i) {
      std::vector<char> nb(M, 0);
      nb[i] = 1;
      for (int sl = 0; sl < h_npart[i]; ++sl) nb[h_partners[(size_t)i * kMaxNear + sl]] = 1;
      for (int j = 0; j < M; ++j) {
        if (nb[j]) continue;
        const double dx = centers[3 * j] - centers[3 * i], dy = centers[3 * j + 1] - centers[3 * i + 1],
                     dz = centers[3 * j + 2] - centers[3 * i + 2];
        const bool close = dx * dx + dy * dy + dz * dz < (kCoarseClose * a) * (kCoarseClose * a);
        (close ? t1 : t2)[(size_t)i * M + j] = 0;
      }
    }
    co.t1.upload(t1.data(), t1.size(), s);
    co.t2.upload(t2.data(), t2.size(), s);
    HIPCHK(hipStreamSynchronize(s));  // t1 and t2 are released after this
  }
  // near low columns, slot by slot
  std::vector<long> acs;
  for (int i = 0; i < M; ++i)
    for (int sl = 0; sl < h_npart[i]; ++sl) acs.push_back(pc.aco[i] + (long)sl * (long)ncn);
  const int nslots = (int)acs.size();
  DevArray<long> dacs;
  if (nslots > 0) {
    co.NL.alloc((size_t)nslots * kCoarseB * n3);
    dacs.upload(acs.data(), acs.size(), s);
    hipLaunchKernelGGL(k_low_cols, dim3(nblocks((long)nslots * kCoarseB * n3)), dim3(256), 0, s, pc.Ac.p, dacs.p,
                       nslots, n3, L, co.NL.p);
  }
  // blocks of A~ Z (self and near): sphere i's row holds D Z, then its slots' NL
  {
    std::vector<int> bp(M + 1, 0), bc;
    std::vector<const double*> src;
    std::vector<double> sg;
    int g = 0;
    for (int i = 0; i < M; ++i) {
      bp[i] = (int)bc.size();
      bc.push_back(i);
      src.push_back(co.DZ.p);
      sg.push_back(1.0);
      for (int sl = 0; sl < h_npart[i]; ++sl, ++g) {
        bc.push_back(h_partners[(size_t)i * kMaxNear + sl]);
        src.push_back(co.NL.p + (size_t)g * kCoarseB * n3);
        sg.push_back(1.0);
      }
    }
    bp[M] = (int)bc.size();
    const long nb = (long)bc.size();
    co.nblk = (int)nb;
    co.ld = (n3 + 63) / 64 * 64;
    co.bptr.upload(bp.data(), bp.size(), s);
    co.bcol.upload(bc.data(), bc.size(), s);
    co.B16.alloc((size_t)nb * kCoarseB * co.ld);
    co.bscale.alloc((size_t)nb);
    co.bpart.alloc((size_t)nb * kMaxRhs * n3);
    DevArray<const double*> dsrc;
    DevArray<double> dsg;
    dsrc.upload(src.data(), src.size(), s);
    dsg.upload(sg.data(), sg.size(), s);
    hipLaunchKernelGGL(k_block_absmax, dim3(nb), dim3(256), 0, s, dsrc.p, (long)kCoarseB * n3, co.bscale.p);
    hipLaunchKernelGGL(k_blocks_f16, dim3(nblocks(nb * (long)kCoarseB * co.ld)), dim3(256), 0, s, dsrc.p, dsg.p,
                       co.bscale.p, n3, kCoarseB, co.ld, nb, co.B16.p);
    HIPCHK(hipStreamSynchronize(s));  // dsrc is released after this
  }
  // E = R A~ Z by columns: diagonal blocks, near blocks R NL (one 27 x 27 product per slot),
  // far blocks on the coarse source grid
  co.E.alloc((size_t)Mc * Mc);
  hipLaunchKernelGGL(k_eself_fill, dim3(nblocks((long)M * kCoarseB * kCoarseB)), dim3(256), 0, s, co.ES.p, M, Mc,
                     co.E.p);
  if (nslots > 0) {
    std::vector<GemmDesc> gn;
    int ngn = 0, g = 0;
    for (int i = 0; i < M; ++i)
      for (int sl = 0; sl < h_npart[i]; ++sl, ++g) {
        const int j = h_partners[(size_t)i * kMaxNear + sl];
        push_gemm(gn, ngn, kCoarseB, kCoarseB, n3, co.R.p, n3, co.NL.p + (size_t)g * kCoarseB * n3, n3,
                  co.E.p + (size_t)j * kCoarseB * Mc + (size_t)i * kCoarseB, kCoarseB, 0, (int)Mc, 1, kCoarseB, 0, 0,
                  0);
      }
    DescPack dp;
    const size_t on = dp.add(gn);
    char* base = push_desc_pack(dp.host);
    launch_gemm64_multi(s, (const GemmDesc*)(base + on), (int)gn.size(), ngn);
  }
  if (n > 64 * kCfbMaxWaves) throw Error(PQN_ERR_INVALID, "precond_coarse supports at most 512 nodes per sphere");
  const int cfb_threads = 64 * ((n + 63) / 64);
  const int cfb_nodes = std::max(co.ncs1, co.ncs - co.ncs1);  // the larger of the two grids
  const size_t cfb_lds = sizeof(double) * ((size_t)(6 + kCoarseL) * cfb_nodes + (size_t)cfb_threads * (kCfbChunk + 1));
  if (cfb_lds > 65536)
    HIPCHK(hipFuncSetAttribute((const void*)k_coarse_far_blocks, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)cfb_lds));
  hipLaunchKernelGGL(k_coarse_far_blocks, dim3(M * M), dim3(cfb_threads), cfb_lds, s, ctr.p, lv.off.p, cls.p, co.t1.p,
                     co.offc.p, co.wc.p, co.Yc.p, co.Tlow.p, n, co.ncs, co.ncs1, M, a, co.E.p);
  // inv(E): Newton-Schulz X <- X (2I - E X). The residual squares at every step, so once it
  // is below sqrt(kCoarseTol / 10) one more step is taken without a new residual (its
  // estimate, the square, is what ns_res reports). The start is the previous configuration's
  // inverse when there is one of the same size whose residual on this E is at most
  // kCoarseWarm (the spheres move little between the configurations of a time-stepping run);
  // otherwise, and when the iteration from it does not reach kCoarseTol, it is the inverse of
  // E's block diagonal.
  co.X.alloc((size_t)Mc * Mc);
  co.X2.alloc((size_t)Mc * Mc);
  co.W.alloc((size_t)Mc * Mc);
  co.res.alloc((size_t)Mc);
  std::vector<double> resp(Mc);
  auto residual = [&]() {  // W = E X and the RMS column residual of I - W
    launch_gemm64_big(s, (int)Mc, (int)Mc, (int)Mc, co.E.p, (int)Mc, 0, co.X.p, 0, (int)Mc, co.W.p, 0, (int)Mc, 0,
                      (int)Mc, 1, 1);
    hipLaunchKernelGGL(k_col_residual, dim3((unsigned)Mc), dim3(256), 0, s, co.W.p, Mc, co.res.p);
    HIPCHK(hipMemcpyAsync(resp.data(), co.res.p, resp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double tot = 0.0;
    for (double v : resp) tot += v;
    return std::isfinite(tot) ? std::sqrt(tot / Mc) : 1e300;
  };
  auto iterate = [&](double res) {  // from X, whose residual is res, with W = E X
    for (int step = 0;; ++step) {
      if (res <= kCoarseTol || step == kCoarseMaxSteps) return res;
      const bool last = res * res <= 0.1 * kCoarseTol;
      hipLaunchKernelGGL(k_diag_minus, dim3((unsigned)Mc), dim3(256), 0, s, co.W.p, (int)Mc, 2.0);
      launch_gemm64_big(s, (int)Mc, (int)Mc, (int)Mc, co.X.p, (int)Mc, 0, co.W.p, 0, (int)Mc, co.X2.p, 0, (int)Mc,
                        0, (int)Mc, 1, 1);
      std::swap(co.X.p, co.X2.p);
      ++co.ns_iters;
      if (last) return res * res;
      res = residual();
    }
  };
  co.ns_iters = 0;
  bool warm = co.have_x && co.x_mc == Mc;
  co.have_x = false;
  double res = 1e300;
  if (warm) {
    res = residual();
    if (res <= kCoarseWarm) res = iterate(res);
    warm = res <= kCoarseTol;
  }
  if (!warm) {
    hipLaunchKernelGGL(k_blockdiag, dim3(nblocks(Mc * Mc)), dim3(256), 0, s, co.X0.p, Mc, co.X.p);
    res = iterate(residual());
  }
  co.ns_res = res;
  co.warm = warm;
  pc_coarse_steps += co.ns_iters;
  pc_coarse_warm += warm ? 1 : 0;
  if (res > kCoarseKeep) return;  // the coarse level stays off for this configuration
  co.Ei.alloc((size_t)Mc * Mc);
  hipLaunchKernelGGL(k_to_f32, dim3(nblocks(Mc * Mc)), dim3(256), 0, s, co.X.p, Mc * Mc, co.Ei.p);
  HIPCHK(hipStreamSynchronize(s));  // dacs and the descriptor staging are released/reused after this
  co.have_x = true;
  co.x_mc = Mc;
  co.on = true;
}

// The coarse pre-correction of an application, on the gathered input vC: c = inv(E) R v
// (into ccI and ccC), then vC <- v - A~ Z c. The caller's D^{-1} GEMM is followed by
// y += Z c, so that the result is Z c + P_f (v - A~ Z c).
void pqn_ctx_impl::coarse_pre(MvGroup& gr) {
  Level& lv = *gr.lv;
  CoarsePc& co = lv.pc.co;
  hipStream_t s = stream;
  const int n = lv.n, n3 = 3 * n, M = lv.M, N = lv.N, K = gr.K;
  const int Mc = kCoarseB * M;
  launch_gemm64_multi_big(s, co.desc.p + 2 * (K - 1), 1, co.tr[K - 1]);
  const dim3 gm((Mc + 255) / 256, (Mc + kCmvCols - 1) / kCmvCols);
#define CMV(KK) hipLaunchKernelGGL(k_coarse_mv<KK>, gm, dim3(256), 0, s, co.Ei.p, co.cr.p, Mc, co.cpart.p)
  switch (K) {
    case 1: CMV(1); break;
    case 2: CMV(2); break;
    case 3: CMV(3); break;
    case 4: CMV(4); break;
    case 5: CMV(5); break;
    default: CMV(6); break;
  }
#undef CMV
  hipLaunchKernelGGL(k_coarse_mv_sum, dim3(nblocks((long)Mc * K)), dim3(256), 0, s, co.cpart.p, (int)gm.y, Mc, M, K,
                     co.ccI.p, co.ccC.p);
  // self and near of A~ z1 from the FP16 blocks of A~ Z
  const int rchunks = (n3 + 255) / 256;
  const dim3 gb(co.nblk * rchunks);
#define CBK(KK)                                                                                                  \
  hipLaunchKernelGGL(k_bsr_block<KK>, gb, dim3(256), 0, s, co.B16.p, co.bscale.p, co.bcol.p, co.ccI.p, n3, kCoarseB, \
                     co.ld, rchunks, co.bpart.p)
  switch (K) {
    case 1: CBK(1); break;
    case 2: CBK(2); break;
    case 3: CBK(3); break;
    case 4: CBK(4); break;
    case 5: CBK(5); break;
    default: CBK(6); break;
  }
#undef CBK
  // far of A~ z1: the coarse density at the coarse source grid, summed by the far kernel
  hipLaunchKernelGGL(k_coarse_qc, dim3(nblocks((long)M * co.ncs * 3 * K)), dim3(256), 0, s, co.Yc.p, co.ccI.p, co.ncs,
                     M, K, co.qc.p);
  launch_pack_coarse(s, pc_prec, K, co.qc.p, co.offc.p, co.wc.p, co.ncs, M * co.ncs, co.src.p);
  OPtrs fp{};
  for (int r = 0; r < K; ++r) fp.p[r] = lv.wk(r).far_part.p;
  // the level's source chunks (with fewer, e.g. 6 of 24, the launch has too few waves to
  // balance: 1.22 against 0.90 ms for six densities at 216 spheres on one 6x12 grid; with
  // the two grids, 12 or 8 chunks gave 51.2-51.7 against 51.0-51.2 ms per six-force-set
  // pass, although their partials are two or three times fewer)
  launch_far_coarse(s, pc_prec, K, co.src.p, lv.off.p, ctr.p, co.t1.p, co.t2.p, n, co.ncs, co.ncs1, M, N, lv.spc,
                    lv.nchunks, 3.0 / (4.0 * kPi * a), fp);
  hipLaunchKernelGGL(k_coarse_resid, dim3(nblocks((long)K * M * n3)), dim3(256), 0, s, lv.pc.vC.p, co.bpart.p,
                     co.bptr.p, fp, lv.nchunks, K, n, M, N);
}

// ------------------------------------------------------------ application

// Every group's densities through its own level's preconditioner: one segmented launch
// per phase when the groups are single densities of different contexts (the suspensions
// of a batch), else one application per group.
void pqn_ctx_impl::precond_apply_groups(std::vector<MvGroup>& groups) {
  bool multi = groups.size() > 1;
  for (MvGroup& gr : groups) multi = multi && gr.K == 1 && !gr.lv->pc.co.on;
  if (!multi) {
    for (MvGroup& gr : groups) gr.c->precond_apply(gr);
    return;
  }
  hipStream_t s = stream;
  std::vector<PcDesc> pd;
  std::vector<GemmDesc> gd;
  int wg = 0, ngd = 0;
  long el = 0;
  for (MvGroup& gr : groups) {
    pqn_ctx_impl& c = *gr.c;
    Level& lv = *gr.lv;
    Precond& pc = lv.pc;
    if (pc.epoch != c.config_epoch) throw Error(PQN_ERR_STATE, "internal: preconditioner not set up");
    const int n3 = 3 * lv.n;
    const int rchunks = (n3 + 255) / 256;
    pd.push_back(PcDesc{pc.B16.p, pc.bscale.p, pc.bcol.p, pc.bptr.p, gr.in[0], gr.out[0], pc.vC.p, pc.wI.p, pc.yI.p,
                        pc.part.p, lv.n, lv.N, lv.M, 3 * lv.L, pc.ld, rchunks, wg, el});
    wg += pc.nblk * rchunks;
    el += (long)lv.M * n3;
    // the suspension's K = 1 GEMMs (y, then w when it has blocks), shifted to this launch
    for (int q = 0; q < (pc.nblk > 0 ? 2 : 1); ++q) {
      GemmDesc d = pc.adesc_h[q];
      d.start = ngd;
      ngd += q == 0 ? pc.aty[0] : pc.atw[0];
      gd.push_back(d);
    }
  }
  DescPack dp;
  const size_t od = dp.add(pd), og = dp.add(gd);
  char* base = push_desc_pack(dp.host);
  const PcDesc* dd = (const PcDesc*)(base + od);
  const int nd = (int)pd.size();
  stage_begin(kStagePrecond);
  hipLaunchKernelGGL(k_pc_gather_multi, dim3(nblocks(el)), dim3(256), 0, s, dd, nd, el);
  launch_gemm64_multi_big(s, (const GemmDesc*)(base + og), (int)gd.size(), ngd);
  if (wg > 0) hipLaunchKernelGGL(k_bsr_block_multi, dim3(wg), dim3(256), 0, s, dd, nd);
  hipLaunchKernelGGL(k_pc_sum_multi, dim3(nblocks(el)), dim3(256), 0, s, dd, nd, el);
  stage_end(kStagePrecond);
  ++pc_applies;
}

void pqn_ctx_impl::precond_apply(MvGroup& gr) {
  Level& lv = *gr.lv;
  Precond& pc = lv.pc;
  if (pc.epoch != config_epoch) throw Error(PQN_ERR_STATE, "internal: preconditioner not set up");
  hipStream_t s = stream;
  const int n = lv.n, n3 = 3 * n, nc = 3 * lv.L, M = lv.M, N = lv.N, K = gr.K;
  QPtrs vin{};
  OPtrs out{};
  for (int r = 0; r < K; ++r) {
    vin.p[r] = gr.in[r];
    out.p[r] = gr.out[r];
  }
  stage_begin(kStagePrecond);
  hipLaunchKernelGGL(k_pc_gather, dim3(nblocks((long)K * M * n3)), dim3(256), 0, s, vin, K, n, M, N, pc.vC.p);
  // two levels: c = inv(E) R v, vC <- v - A~ Z c; below, y += Z c after y = D^{-1} vC
  CoarsePc& co = pc.co;
  if (co.on) coarse_pre(gr);
  // y = D^{-1} v and (with blocks) w = TD v; out may be the input: v is not read after the
  // gather. With the side stream on, y (matrix cores) runs there beside the block product
  // (HBM), and the sum waits for both.
  const GemmDesc* ad = pc.adesc.p + 3 * (K - 1);
  const bool ov = cfg.side_stream && !cfg.profile && pc.nblk > 0;
  if (ov) {
    hipStream_t sa = side_stream();
    HIPCHK(hipEventRecord(ev_in, s));
    HIPCHK(hipStreamWaitEvent(sa, ev_in, 0));
    launch_gemm64_multi_big(sa, ad, 1, pc.aty[K - 1]);
    if (co.on) launch_gemm64_multi_big(sa, co.desc.p + 2 * (K - 1) + 1, 1, co.tz[K - 1]);
    HIPCHK(hipEventRecord(ev_side, sa));
    launch_gemm64_multi_big(s, ad + 2, 1, pc.atw[K - 1]);
  } else {
    launch_gemm64_multi_big(s, ad, pc.nblk > 0 ? 2 : 1, pc.aty[K - 1] + (pc.nblk > 0 ? pc.atw[K - 1] : 0));
    if (co.on) launch_gemm64_multi_big(s, co.desc.p + 2 * (K - 1) + 1, 1, co.tz[K - 1]);
  }
  if (pc.nblk > 0) {
    const int rchunks = (n3 + 255) / 256;
    const dim3 g(pc.nblk * rchunks);
#define BSRK(KK) \
  hipLaunchKernelGGL(k_bsr_block<KK>, g, dim3(256), 0, s, pc.B16.p, pc.bscale.p, pc.bcol.p, pc.wI.p, n3, nc, pc.ld, \
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
  }
  if (ov) HIPCHK(hipStreamWaitEvent(s, ev_side, 0));
  hipLaunchKernelGGL(k_pc_sum, dim3(nblocks((long)M * K * n3)), dim3(256), 0, s, pc.yI.p, pc.part.p, pc.bptr.p, K, n,
                     M, N, out);
  stage_end(kStagePrecond);
  ++pc_applies;
}

}  // namespace bipqn
