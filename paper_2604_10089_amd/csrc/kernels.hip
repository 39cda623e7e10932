// Device kernels of the mobility product (one HIP translation unit).
//
// Vector layout: surface fields are SoA [3][N] doubles, node index
// t = sphere * n + local node, local node = theta_row * n_phi + phi_col.
#include "kernels.hpp"

namespace bipqn {

// --------------------------------------------------------------- packing
//
// Far-tile sources for K densities sharing one geometry pass. FP32 record of a
// node: {o.x, o.y, o.z, wq_0.x, wq_0.y, wq_0.z, wq_1.x, ...} padded to a
// multiple of 4 floats; FP64 record padded to a multiple of 2 doubles.

template <int K>
__global__ __launch_bounds__(256) void k_pack32(QPtrs q, const double* __restrict__ off,
                                                const double* __restrict__ w, int n, int N, float* __restrict__ src) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  constexpr int S = src32_stride(K);
  const int k = t % n;
  const double wk = w[k];
  float* d = src + (size_t)t * S;
  d[0] = (float)off[3 * k];
  d[1] = (float)off[3 * k + 1];
  d[2] = (float)off[3 * k + 2];
#pragma unroll
  for (int r = 0; r < K; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) d[3 + 3 * r + c] = (float)(wk * q.p[r][(size_t)c * N + t]);
#pragma unroll
  for (int e = 3 + 3 * K; e < S; ++e) d[e] = 0.f;
}

template <int K>
__global__ __launch_bounds__(256) void k_pack64(QPtrs q, const double* __restrict__ off,
                                                const double* __restrict__ w, int n, int N, double* __restrict__ src) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  constexpr int S = src64_stride(K);
  const int k = t % n;
  const double wk = w[k];
  double* d = src + (size_t)t * S;
  d[0] = off[3 * k];
  d[1] = off[3 * k + 1];
  d[2] = off[3 * k + 2];
#pragma unroll
  for (int r = 0; r < K; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) d[3 + 3 * r + c] = wk * q.p[r][(size_t)c * N + t];
#pragma unroll
  for (int e = 3 + 3 * K; e < S; ++e) d[e] = 0.0;
}

// Far sources on the coarse far-source grid: record of coarse node k of sphere j
// from the synthesised coarse densities qc[(j * nc + k) * 3K + 3r + c] (the
// degree-truncated densities at the coarse nodes) with the coarse weights.
template <int K>
__global__ __launch_bounds__(256) void k_pack_coarse(const double* __restrict__ qc, const double* __restrict__ off,
                                                     const double* __restrict__ w, int nc, int Nc, int fp32,
                                                     void* __restrict__ src) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= Nc) return;
  constexpr int C = 3 * K;
  const int k = t % nc;
  const double wk = w[k];
  const double* q = qc + (size_t)t * C;
  if (fp32) {
    constexpr int S = src32_stride(K);
    float* d = (float*)src + (size_t)t * S;
    d[0] = (float)off[3 * k];
    d[1] = (float)off[3 * k + 1];
    d[2] = (float)off[3 * k + 2];
#pragma unroll
    for (int e = 0; e < C; ++e) d[3 + e] = (float)(wk * q[e]);
#pragma unroll
    for (int e = 3 + C; e < S; ++e) d[e] = 0.f;
  } else {
    constexpr int S = src64_stride(K);
    double* d = (double*)src + (size_t)t * S;
    d[0] = off[3 * k];
    d[1] = off[3 * k + 1];
    d[2] = off[3 * k + 2];
#pragma unroll
    for (int e = 0; e < C; ++e) d[3 + e] = wk * q[e];
#pragma unroll
    for (int e = 3 + C; e < S; ++e) d[e] = 0.0;
  }
}

// 1/sqrt(x) in FP64 for finite x > 0 (squared distances of distinct points):
// the hardware estimate y0 refined once by the second-order expansion of
// (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + ..., e = 1 - x y0^2. Six VALU
// instructions; the library rsqrt adds a class test and two selects for zero,
// infinite and denormal arguments, which cannot occur here.
__device__ __forceinline__ double rsqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(y * e, fma(e, 0.375, 0.5), y);
}

// One source sphere j of the FP64 pair sum: nodes [k0, k1) of its records (ns per sphere),
// added to the target's accumulator when the pair is active (cls 0).
template <int K>
__device__ __forceinline__ void far64_tile(int j, int k0, int k1, const double* __restrict__ src,
                                           const double* __restrict__ ctr, const unsigned char* __restrict__ cls,
                                           int ns, int M, bool valid, int i, double px, double py, double pz,
                                           double ox, double oy, double oz, double (&acc)[K][3]) {
  constexpr int S = src64_stride(K);
  const bool act = valid && cls[i * M + j] == 0;
  if (!__any(act)) return;
  const double Xx = act ? (px - ctr[3 * j]) + ox : 1.0e4;
  const double Xy = act ? (py - ctr[3 * j + 1]) + oy : 0.0;
  const double Xz = act ? (pz - ctr[3 * j + 2]) + oz : 0.0;
  double sm[K][3];
#pragma unroll
  for (int r = 0; r < K; ++r) sm[r][0] = sm[r][1] = sm[r][2] = 0.0;
  const double* sp = src + (size_t)j * ns * S;
  // r.y = Ct - r^2 / 2 (as in the FP32 tile); (w r).q for K >= 2
  const double Ct = 0.5 * (Xx * Xx + Xy * Xy + Xz * Xz - (sp[0] * sp[0] + sp[1] * sp[1] + sp[2] * sp[2]));
#pragma unroll 2
  for (int kk = k0; kk < k1; ++kk) {
    const double* e = sp + (size_t)kk * S;
    const double rx = Xx - e[0], ry = Xy - e[1], rz = Xz - e[2];
    const double r2 = fma(rx, rx, fma(ry, ry, rz * rz));
    const double ri = rsqrt_pos(r2);
    const double ri2 = ri * ri;
    const double rn = fma(-0.5, r2, Ct);
    const double wgt = rn * ri * ri2 * ri2;
    if constexpr (K == 1) {
      const double c = wgt * fma(rx, e[3], fma(ry, e[4], rz * e[5]));
      sm[0][0] = fma(c, rx, sm[0][0]);
      sm[0][1] = fma(c, ry, sm[0][1]);
      sm[0][2] = fma(c, rz, sm[0][2]);
    } else {
      const double wx = wgt * rx, wy = wgt * ry, wz = wgt * rz;
#pragma unroll
      for (int r = 0; r < K; ++r) {
        const double c = fma(wx, e[3 + 3 * r], fma(wy, e[4 + 3 * r], wz * e[5 + 3 * r]));
        sm[r][0] = fma(c, rx, sm[r][0]);
        sm[r][1] = fma(c, ry, sm[r][1]);
        sm[r][2] = fma(c, rz, sm[r][2]);
      }
    }
  }
  if (act)
#pragma unroll
    for (int r = 0; r < K; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[r][c] += sm[r][c];
}

// ----------------------------------------------------------- far pair sum
//
// u_r(x) += 3/(4 pi a) sum_y r (r.wq_r,y)(r.o_y)/|r|^5, r = x - y, for every
// density r < K, over source spheres j != i that are not near sphere i. One
// thread owns TPT targets; the grid's y dimension splits the source spheres
// into chunks. The source stream is wave-uniform, so its loads go through the
// scalar unit and its values enter the VALU as scalar operands; r, |r|^-5 and
// r.o are shared by the K densities. Target positions are taken relative to
// the source sphere's centre, X = (c_i - c_j) + o_x, formed in FP64 and
// rounded once, so r = X - o_y carries no large-coordinate cancellation. Each
// sphere's contribution (one tile) is summed in the pair precision and added
// to an FP64 accumulator.

// Workgroups are handed to the eight XCDs in turn (block b to XCD b mod 8).
// Block b takes work item xcd_item(b) so that each XCD runs one contiguous
// eighth of the item list: items next to each other in the list read the same
// sources, which then stay in that XCD's L2. The grid has 8 * per blocks;
// items past the end exit at once.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_item(int b, int per) { return (b % kXcds) * per + b / kXcds; }

// One source sphere j (ns source nodes per sphere), nodes [k0, k1), against TPT
// targets per thread: the tile is summed in FP32 and added to the FP64
// accumulators of active targets.
template <int TPT, int K>
__device__ __forceinline__ void far32_tile(int j, int k0, int k1, const float* __restrict__ src,
                                           const double* __restrict__ ctr, const unsigned char* __restrict__ cls,
                                           int ns, int M, const bool (&valid)[TPT], const int (&ti)[TPT],
                                           const double (&px)[TPT], const double (&py)[TPT], const double (&pz)[TPT],
                                           const double (&ox)[TPT], const double (&oy)[TPT],
                                           const double (&oz)[TPT], double (&acc)[TPT][K][3]) {
  constexpr int S = src32_stride(K);
  const double cjx = ctr[3 * j], cjy = ctr[3 * j + 1], cjz = ctr[3 * j + 2];
  const float* sp = src + (size_t)j * ns * S;
  // |y|^2 of the sphere's source offsets (all a^2 up to rounding), from its first node
  const double a2 = (double)sp[0] * sp[0] + (double)sp[1] * sp[1] + (double)sp[2] * sp[2];
  bool act[TPT];
  int any = 0;
#pragma unroll
  for (int u = 0; u < TPT; ++u) {
    act[u] = valid[u] && cls[ti[u] * M + j] == 0;
    any |= act[u];
  }
  if (!__any(any)) return;
  // r.y = (|X|^2 - |y|^2 - |r|^2) / 2 with r = X - y: one FMA per pair from the
  // target constant Ct = (|X|^2 - a^2) / 2 instead of a dot product. Rounding:
  // Ct and r^2 are O(|X|^2) while r.y is O(|X| a), so the relative error of r.y
  // grows like |X| / a (at most ~20 here), on the far pairs whose terms decay
  // like 1/|X|^2; the operator's mixed-vs-FP64 error is unchanged (2.4e-8).
  float Xx[TPT], Xy[TPT], Xz[TPT], Ct[TPT], sm[TPT][K][3];
#pragma unroll
  for (int u = 0; u < TPT; ++u) {
    Xx[u] = act[u] ? (float)((px[u] - cjx) + ox[u]) : 1.0e4f;
    Xy[u] = act[u] ? (float)((py[u] - cjy) + oy[u]) : 0.0f;
    Xz[u] = act[u] ? (float)((pz[u] - cjz) + oz[u]) : 0.0f;
    Ct[u] = (float)(0.5 * ((double)Xx[u] * Xx[u] + (double)Xy[u] * Xy[u] + (double)Xz[u] * Xz[u] - a2));
#pragma unroll
    for (int r = 0; r < K; ++r) sm[u][r][0] = sm[u][r][1] = sm[u][r][2] = 0.0f;
  }
#pragma unroll 8
  for (int kk = k0; kk < k1; ++kk) {
    const float* e = sp + (size_t)kk * S;
    const float sx = e[0], sy = e[1], sz = e[2];
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
      const float rx = Xx[u] - sx, ry = Xy[u] - sy, rz = Xz[u] - sz;
      const float r2 = fmaf(rx, rx, fmaf(ry, ry, rz * rz));
      const float ri = __builtin_amdgcn_rsqf(r2);
      const float ri2 = ri * ri;
      const float rn = fmaf(-0.5f, r2, Ct[u]);
      const float wgt = rn * ri * ri2 * ri2;
      if constexpr (K == 1) {
        const float rq = fmaf(rx, e[3], fmaf(ry, e[4], rz * e[5]));
        const float c = wgt * rq;
        sm[u][0][0] = fmaf(c, rx, sm[u][0][0]);
        sm[u][0][1] = fmaf(c, ry, sm[u][0][1]);
        sm[u][0][2] = fmaf(c, rz, sm[u][0][2]);
      } else {
        // the weight folded into r once: (w r).q costs one multiply per density less
        const float wx = wgt * rx, wy = wgt * ry, wz = wgt * rz;
#pragma unroll
        for (int r = 0; r < K; ++r) {
          const float c = fmaf(wx, e[3 + 3 * r], fmaf(wy, e[4 + 3 * r], wz * e[5 + 3 * r]));
          sm[u][r][0] = fmaf(c, rx, sm[u][r][0]);
          sm[u][r][1] = fmaf(c, ry, sm[u][r][1]);
          sm[u][r][2] = fmaf(c, rz, sm[u][r][2]);
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < TPT; ++u)
    if (act[u])
#pragma unroll
      for (int r = 0; r < K; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[u][r][c] += (double)sm[u][r][c];
}

// Block = 256 threads owning 256 TPT consecutive targets; every wave streams
// the whole chunk of source spheres.
template <int TPT, int K>
__device__ __forceinline__ void far32_body(int tb, int chunk, const float* __restrict__ src,
                                           const double* __restrict__ off, const double* __restrict__ ctr,
                                           const unsigned char* __restrict__ cls, int n, int ns, int M, int N,
                                           int spc, double scale, const OPtrs& part) {
  const int j0 = chunk * spc;
  const int j1 = min(M, j0 + spc);
  int ti[TPT];
  bool valid[TPT];
  double px[TPT], py[TPT], pz[TPT], ox[TPT], oy[TPT], oz[TPT];
  double acc[TPT][K][3];
#pragma unroll
  for (int u = 0; u < TPT; ++u) {
    const int t = tb * 256 * TPT + u * 256 + threadIdx.x;
    valid[u] = t < N;
    const int tt = valid[u] ? t : N - 1;
    const int i = tt / n;
    const int k = tt - i * n;
    ti[u] = i;
    px[u] = ctr[3 * i];
    py[u] = ctr[3 * i + 1];
    pz[u] = ctr[3 * i + 2];
    ox[u] = off[3 * k];
    oy[u] = off[3 * k + 1];
    oz[u] = off[3 * k + 2];
#pragma unroll
    for (int r = 0; r < K; ++r) acc[u][r][0] = acc[u][r][1] = acc[u][r][2] = 0.0;
  }
  for (int j = j0; j < j1; ++j)
    far32_tile<TPT, K>(j, 0, ns, src, ctr, cls, ns, M, valid, ti, px, py, pz, ox, oy, oz, acc);
#pragma unroll
  for (int u = 0; u < TPT; ++u) {
    const int t = tb * 256 * TPT + u * 256 + threadIdx.x;
    if (valid[u])
#pragma unroll
      for (int r = 0; r < K; ++r) {
        double* pb = part.p[r] + (size_t)chunk * 3 * N;
        pb[t] = scale * acc[u][r][0];
        pb[N + t] = scale * acc[u][r][1];
        pb[2 * N + t] = scale * acc[u][r][2];
      }
  }
}

// Split layout: block = 4 waves on the same 64 targets; the chunk's source
// nodes (spheres j0..j1 flattened) are cut into four equal ranges, one per
// wave, and the four FP64 partial sums are added in wave order through LDS
// (one density at a time, so the buffer stays at 9 x 64 doubles). For the same
// number of chunk partials the grid has four times as many, four times
// shorter, waves, which evens out the last wave of the launch.
template <int K>
__device__ __forceinline__ void far32_split_body(int tb, int chunk, const float* __restrict__ src,
                                                 const double* __restrict__ off, const double* __restrict__ ctr,
                                                 const unsigned char* __restrict__ cls, int n, int ns, int M, int N,
                                                 int spc, double scale, const OPtrs& part, double* __restrict__ lds) {
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int j0 = chunk * spc;
  const int j1 = min(M, j0 + spc);
  const int t = tb * 64 + lane;
  int ti[1];
  bool valid[1];
  double px[1], py[1], pz[1], ox[1], oy[1], oz[1];
  double acc[1][K][3];
  valid[0] = t < N;
  {
    const int tt = valid[0] ? t : N - 1;
    const int i = tt / n;
    const int k = tt - i * n;
    ti[0] = i;
    px[0] = ctr[3 * i];
    py[0] = ctr[3 * i + 1];
    pz[0] = ctr[3 * i + 2];
    ox[0] = off[3 * k];
    oy[0] = off[3 * k + 1];
    oz[0] = off[3 * k + 2];
  }
#pragma unroll
  for (int r = 0; r < K; ++r) acc[0][r][0] = acc[0][r][1] = acc[0][r][2] = 0.0;
  const int len = (j1 - j0) * ns;
  const int s0 = j0 * ns + (wv * len) / 4, s1 = j0 * ns + ((wv + 1) * len) / 4;
  for (int s = s0; s < s1;) {
    const int j = s / ns;
    const int k0 = s - j * ns, k1 = min(ns, s1 - j * ns);
    far32_tile<1, K>(j, k0, k1, src, ctr, cls, ns, M, valid, ti, px, py, pz, ox, oy, oz, acc);
    s = j * ns + k1;
  }
#pragma unroll
  for (int r = 0; r < K; ++r) {
    if (wv > 0)
#pragma unroll
      for (int c = 0; c < 3; ++c) lds[((wv - 1) * 3 + c) * 64 + lane] = acc[0][r][c];
    __syncthreads();
    if (wv == 0 && valid[0]) {
      double* pb = part.p[r] + (size_t)chunk * 3 * N;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double v = ((acc[0][r][c] + lds[c * 64 + lane]) + lds[(3 + c) * 64 + lane]) + lds[(6 + c) * 64 + lane];
        pb[(size_t)c * N + t] = scale * v;
      }
    }
    __syncthreads();
  }
}

template <int K>
__global__ __launch_bounds__(256) void k_far32s(const float* __restrict__ src, const double* __restrict__ off,
                                                const double* __restrict__ ctr, const unsigned char* __restrict__ cls,
                                                int n, int ns, int M, int N, int spc, double scale, OPtrs part,
                                                int ntb, int total, int per) {
  __shared__ double lds[9 * 64];
  // issue priority over waves of kernels running beside it (near tiles, GEMMs on the side stream)
  __builtin_amdgcn_s_setprio(3);
  const int item = xcd_item(blockIdx.x, per);
  if (item >= total) return;  // uniform over the block: no barrier is skipped by part of it
  far32_split_body<K>(item % ntb, item / ntb, src, off, ctr, cls, n, ns, M, N, spc, scale, part, lds);
}

// Work item = chunk * ntb + target block (chunk-major: an XCD takes whole chunks).
template <int TPT, int K>
__global__ __launch_bounds__(256) void k_far32(const float* __restrict__ src, const double* __restrict__ off,
                                               const double* __restrict__ ctr, const unsigned char* __restrict__ cls,
                                               int n, int ns, int M, int N, int spc, double scale, OPtrs part,
                                               int ntb, int total, int per) {
  __builtin_amdgcn_s_setprio(3);  // as in k_far32s
  const int item = xcd_item(blockIdx.x, per);
  if (item >= total) return;
  far32_body<TPT, K>(item % ntb, item / ntb, src, off, ctr, cls, n, ns, M, N, spc, scale, part);
}

// Many suspensions in one launch: block b takes work item b of a list ordered
// by decreasing cost (instance, target block, source chunk); the hardware
// dispatches blocks in order, so the largest tiles start first.
template <int TPT>
__global__ __launch_bounds__(256) void k_far32_multi(const FarDesc* __restrict__ desc, int ndesc) {
  const int item = blockIdx.x;
  int d = 0;
  while (d + 1 < ndesc && desc[d + 1].item0 <= item) ++d;
  const FarDesc D = desc[d];
  if (D.live && !*D.live) return;  // uniform over the block
  const int local = item - D.item0;
  const int tb = local % D.ntb, chunk = local / D.ntb;
  OPtrs part;
  part.p[0] = D.part;
  if constexpr (TPT == 0) {
    __shared__ double lds[9 * 64];
    far32_split_body<1>(tb, chunk, (const float*)D.src, D.off, D.ctr, D.cls, D.n, D.n, D.M, D.N, D.spc, D.scale,
                        part, lds);
  } else {
    far32_body<TPT, 1>(tb, chunk, (const float*)D.src, D.off, D.ctr, D.cls, D.n, D.n, D.M, D.N, D.spc, D.scale,
                       part);
  }
}

template <int K>
__device__ __forceinline__ void far64_body(int tb, int chunk, const double* __restrict__ src,
                                           const double* __restrict__ off, const double* __restrict__ ctr,
                                           const unsigned char* __restrict__ cls, int n, int ns, int M, int N,
                                           int spc, double scale, const OPtrs& part,
                                           const unsigned char* __restrict__ cls2 = nullptr, int ns1 = 0) {
  // FP64 pair sum, one target per thread. With cls2 set, sphere j's records are two source
  // grids (nodes [0, ns1) and [ns1, ns)), the first summed for the pairs active in cls, the
  // second for those active in cls2 (the coarse level's two far grids).
  const int t = tb * 256 + threadIdx.x;
  const bool valid = t < N;
  const int tt = valid ? t : N - 1;
  const int i = tt / n;
  const int k = tt - i * n;
  const double px = ctr[3 * i], py = ctr[3 * i + 1], pz = ctr[3 * i + 2];
  const double ox = off[3 * k], oy = off[3 * k + 1], oz = off[3 * k + 2];
  const int j0 = chunk * spc;
  const int j1 = min(M, j0 + spc);
  double acc[K][3];
#pragma unroll
  for (int r = 0; r < K; ++r) acc[r][0] = acc[r][1] = acc[r][2] = 0.0;
  for (int j = j0; j < j1; ++j) {
    if (cls2) {
      far64_tile<K>(j, 0, ns1, src, ctr, cls, ns, M, valid, i, px, py, pz, ox, oy, oz, acc);
      far64_tile<K>(j, ns1, ns, src, ctr, cls2, ns, M, valid, i, px, py, pz, ox, oy, oz, acc);
    } else {
      far64_tile<K>(j, 0, ns, src, ctr, cls, ns, M, valid, i, px, py, pz, ox, oy, oz, acc);
    }
  }
  if (valid)
#pragma unroll
    for (int r = 0; r < K; ++r) {
      double* pb = part.p[r] + (size_t)chunk * 3 * N;
      pb[t] = scale * acc[r][0];
      pb[N + t] = scale * acc[r][1];
      pb[2 * N + t] = scale * acc[r][2];
    }
}

// The FP32 pair sum over two source grids per sphere (as far64_body with cls2), one target
// per thread.
template <int K>
__device__ __forceinline__ void far32c_body(int tb, int chunk, const float* __restrict__ src,
                                            const double* __restrict__ off, const double* __restrict__ ctr,
                                            const unsigned char* __restrict__ cls,
                                            const unsigned char* __restrict__ cls2, int n, int ns, int ns1, int M,
                                            int N, int spc, double scale, const OPtrs& part) {
  const int j0 = chunk * spc;
  const int j1 = min(M, j0 + spc);
  int ti[1];
  bool valid[1];
  double px[1], py[1], pz[1], ox[1], oy[1], oz[1];
  double acc[1][K][3];
  const int t = tb * 256 + threadIdx.x;
  valid[0] = t < N;
  {
    const int tt = valid[0] ? t : N - 1;
    const int i = tt / n;
    const int k = tt - i * n;
    ti[0] = i;
    px[0] = ctr[3 * i];
    py[0] = ctr[3 * i + 1];
    pz[0] = ctr[3 * i + 2];
    ox[0] = off[3 * k];
    oy[0] = off[3 * k + 1];
    oz[0] = off[3 * k + 2];
  }
#pragma unroll
  for (int r = 0; r < K; ++r) acc[0][r][0] = acc[0][r][1] = acc[0][r][2] = 0.0;
  for (int j = j0; j < j1; ++j) {
    far32_tile<1, K>(j, 0, ns1, src, ctr, cls, ns, M, valid, ti, px, py, pz, ox, oy, oz, acc);
    far32_tile<1, K>(j, ns1, ns, src, ctr, cls2, ns, M, valid, ti, px, py, pz, ox, oy, oz, acc);
  }
  if (valid[0])
#pragma unroll
    for (int r = 0; r < K; ++r) {
      double* pb = part.p[r] + (size_t)chunk * 3 * N;
      pb[t] = scale * acc[0][r][0];
      pb[N + t] = scale * acc[0][r][1];
      pb[2 * N + t] = scale * acc[0][r][2];
    }
}

template <int K>
__global__ __launch_bounds__(256) void k_far64(const double* __restrict__ src, const double* __restrict__ off,
                                               const double* __restrict__ ctr, const unsigned char* __restrict__ cls,
                                               int n, int ns, int M, int N, int spc, double scale, OPtrs part,
                                               int ntb, int total, int per) {
  const int item = xcd_item(blockIdx.x, per);
  if (item >= total) return;
  far64_body<K>(item % ntb, item / ntb, src, off, ctr, cls, n, ns, M, N, spc, scale, part);
}

// The same pair sums launched by the preconditioner's coarse level (far pairs of its
// coarse operator, sources on its two coarse grids: the pairs active in cls on the first
// ns1 records of a sphere, those active in cls2 on the rest): kernels of their own, so that
// profiles keep them apart from the operator's far launches.
template <int K>
__global__ __launch_bounds__(256) void k_far32c(const float* __restrict__ src, const double* __restrict__ off,
                                                const double* __restrict__ ctr, const unsigned char* __restrict__ cls,
                                                const unsigned char* __restrict__ cls2, int n, int ns, int ns1, int M,
                                                int N, int spc, double scale, OPtrs part, int ntb, int total,
                                                int per) {
  const int item = xcd_item(blockIdx.x, per);
  if (item >= total) return;
  far32c_body<K>(item % ntb, item / ntb, src, off, ctr, cls, cls2, n, ns, ns1, M, N, spc, scale, part);
}

template <int K>
__global__ __launch_bounds__(256) void k_far64c(const double* __restrict__ src, const double* __restrict__ off,
                                                const double* __restrict__ ctr, const unsigned char* __restrict__ cls,
                                                const unsigned char* __restrict__ cls2, int n, int ns, int ns1, int M,
                                                int N, int spc, double scale, OPtrs part, int ntb, int total,
                                                int per) {
  const int item = xcd_item(blockIdx.x, per);
  if (item >= total) return;
  far64_body<K>(item % ntb, item / ntb, src, off, ctr, cls, n, ns, M, N, spc, scale, part, cls2, ns1);
}

__global__ __launch_bounds__(256) void k_far64_multi(const FarDesc* __restrict__ desc, int ndesc) {
  const int item = blockIdx.x;
  int d = 0;
  while (d + 1 < ndesc && desc[d + 1].item0 <= item) ++d;
  const FarDesc D = desc[d];
  if (D.live && !*D.live) return;
  const int local = item - D.item0;
  const int tb = local % D.ntb, chunk = local / D.ntb;
  OPtrs part;
  part.p[0] = D.part;
  far64_body<1>(tb, chunk, (const double*)D.src, D.off, D.ctr, D.cls, D.n, D.n, D.M, D.N, D.spc, D.scale, part);
}

// ---------------------------------------------------------- near pair sum
//
// For each target x on sphere i and near partner j: the sum over the upsampled
// nodes f of sphere j of w_f K(x, y_f) (q_f - q_j(x*)), x* the foot point of x
// on sphere j and q_j(x*) the degree-p harmonic expansion of the density there
// (constant-density subtraction). For K >= 2 densities the subtracted part is
// applied after the loop as (sum_f w_f K(x, y_f)) q_j(x*): the 3x3 kernel
// moment is shared by all densities.
//
// Grid (near pair, 64-target chunk), block = kNearWaves waves on the same 64
// targets. Wave w takes the w-th share of the source nodes and the harmonic
// orders m = w (mod kNearWaves) of the foot-point expansion; the partial sums
// meet in LDS and are added in wave order, so results do not depend on timing.
// Within a wave the source records and coefficients are uniform (scalar loads).
// The upsampled densities of the K densities are interleaved per node,
// qup[(j * nup + f) * 3K + 3r + c], so one node's values are one contiguous
// scalar-load stream.

constexpr int kNearWaves = 4;

// Partial foot-point values: orders m = wv (mod kNearWaves) of sum_lm c_lm Y_lm(x*).
// cj: the coefficients of the source sphere, [3K][L] (density r, component c at row 3r + c).
template <int K>
__device__ __forceinline__ void foot_part(int p, double ct, double st, double cp, double sp,
                                          const double* __restrict__ shab, const double* __restrict__ cj, int L,
                                          int wv, double (&f)[K][3]) {
  double pmm = sqrt(1.0 / (4.0 * kPi));
  double cm = 1.0, sm = 0.0;
  for (int m = 0; m <= p; ++m) {
    if (m > 0) {
      pmm *= shab[2 * sh_index(m, m, 0)] * st;
      const double c2 = cm * cp - sm * sp, s2 = sm * cp + cm * sp;
      cm = c2;
      sm = s2;
    }
    if (m % kNearWaves != wv) continue;
    const double fac = m == 0 ? 1.0 : sqrt(2.0);
    const double yc = fac * cm, ys = fac * sm;
    double plm2 = 0.0, plm1 = pmm;
    for (int l = m; l <= p; ++l) {
      const int ic = sh_index(l, m, 0);
      if (l > m) {
        const double pl = shab[2 * ic] * (ct * plm1 - shab[2 * ic + 1] * plm2);
        plm2 = plm1;
        plm1 = pl;
      }
      const double vc = plm1 * yc;
#pragma unroll
      for (int r = 0; r < K; ++r) {
        const double* cx = cj + (size_t)(3 * r) * L + ic;
        f[r][0] = fma(vc, cx[0], f[r][0]);
        f[r][1] = fma(vc, cx[L], f[r][1]);
        f[r][2] = fma(vc, cx[2 * L], f[r][2]);
      }
      if (m > 0) {
        const double vs = plm1 * ys;
#pragma unroll
        for (int r = 0; r < K; ++r) {
          const double* cx = cj + (size_t)(3 * r) * L + ic + 1;
          f[r][0] = fma(vs, cx[0], f[r][0]);
          f[r][1] = fma(vs, cx[L], f[r][1]);
          f[r][2] = fma(vs, cx[2 * L], f[r][2]);
        }
      }
    }
  }
}

// lds: kNearWaves * 3K * 64 doubles.
template <int K>
__device__ __forceinline__ void near_body(int pair, int chunk, const double* __restrict__ ctr,
                                          const double* __restrict__ off, const double4* __restrict__ offup,
                                          const double* __restrict__ shab, const double* __restrict__ qup,
                                          const double* __restrict__ coef,
                                          const int* __restrict__ npairs, int n, int M, int N, int nup, int p, int L,
                                          double scale, const OPtrs& near_part, double* __restrict__ lds) {
  constexpr int C = 3 * K;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int i = npairs[3 * pair], j = npairs[3 * pair + 1], slot = npairs[3 * pair + 2];
  const int k = chunk * 64 + lane;
  const bool valid = k < n;
  const int kk = valid ? k : n - 1;
  const int t = i * n + kk;
  const double Xx = (ctr[3 * i] + off[3 * kk]) - ctr[3 * j];
  const double Xy = (ctr[3 * i + 1] + off[3 * kk + 1]) - ctr[3 * j + 1];
  const double Xz = (ctr[3 * i + 2] + off[3 * kk + 2]) - ctr[3 * j + 2];
  double f[K][3];
  {
    const double rho = sqrt(Xx * Xx + Xy * Xy);
    const double R = sqrt(rho * rho + Xz * Xz);
    const double ct = Xz / R, st = rho / R;
    const double cp = rho > 0.0 ? Xx / rho : 1.0, sp = rho > 0.0 ? Xy / rho : 0.0;
#pragma unroll
    for (int r = 0; r < K; ++r) f[r][0] = f[r][1] = f[r][2] = 0.0;
    foot_part<K>(p, ct, st, cp, sp, shab, coef + (size_t)j * C * L, L, wv, f);
#pragma unroll
    for (int r = 0; r < K; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) lds[(wv * C + 3 * r + c) * 64 + lane] = f[r][c];
  }
  __syncthreads();
  if constexpr (K == 1) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double v = lds[c * 64 + lane];
#pragma unroll
      for (int w = 1; w < kNearWaves; ++w) v += lds[(w * C + c) * 64 + lane];
      f[0][c] = v;
    }
  }
  const int f0 = (wv * nup) / kNearWaves, f1 = ((wv + 1) * nup) / kNearWaves;
  // r.o = Ct - r^2 / 2 with Ct = (|X|^2 - |o|^2) / 2 (all upsampled nodes lie
  // on the sphere): one FMA per pair instead of a dot product. Ct and r^2 are
  // O(|X|^2) while r.o is O(|X| a), so the rounding grows like |X| / a: below
  // 3 for near targets at the default near gap (0.5 a).
  const double4 o0 = offup[0];
  const double Ct = 0.5 * (Xx * Xx + Xy * Xy + Xz * Xz - (o0.x * o0.x + o0.y * o0.y + o0.z * o0.z));
  double a[K][3];
#pragma unroll
  for (int r = 0; r < K; ++r) a[r][0] = a[r][1] = a[r][2] = 0.0;
  double mxx = 0.0, mxy = 0.0, mxz = 0.0, myy = 0.0, myz = 0.0, mzz = 0.0;
#pragma unroll 2
  for (int fi = f0; fi < f1; ++fi) {
    const double4 o = offup[fi];
    const double rx = Xx - o.x, ry = Xy - o.y, rz = Xz - o.z;
    const double r2 = fma(rx, rx, fma(ry, ry, rz * rz));
    const double ri = rsqrt_pos(r2);
    const double ri2 = ri * ri;
    const double rn = fma(-0.5, r2, Ct);
    const double wgt = o.w * rn * ri * ri2 * ri2;
    if constexpr (K == 1) {
      const double* qx = qup + ((size_t)j * nup + fi) * 3;
      const double dqx = qx[0] - f[0][0], dqy = qx[1] - f[0][1], dqz = qx[2] - f[0][2];
      const double c = wgt * fma(rx, dqx, fma(ry, dqy, rz * dqz));
      a[0][0] = fma(c, rx, a[0][0]);
      a[0][1] = fma(c, ry, a[0][1]);
      a[0][2] = fma(c, rz, a[0][2]);
    } else {
      const double wx = wgt * rx, wy = wgt * ry, wz = wgt * rz;
      mxx = fma(wx, rx, mxx);
      mxy = fma(wx, ry, mxy);
      mxz = fma(wx, rz, mxz);
      myy = fma(wy, ry, myy);
      myz = fma(wy, rz, myz);
      mzz = fma(wz, rz, mzz);
#pragma unroll
      for (int r = 0; r < K; ++r) {
        const double* qx = qup + ((size_t)j * nup + fi) * C + 3 * r;
        const double d = fma(wx, qx[0], fma(wy, qx[1], wz * qx[2]));
        a[r][0] = fma(d, rx, a[r][0]);
        a[r][1] = fma(d, ry, a[r][1]);
        a[r][2] = fma(d, rz, a[r][2]);
      }
    }
  }
  __syncthreads();  // every wave has read the foot-point partials
  if constexpr (K > 1) {
#pragma unroll
    for (int r = 0; r < K; ++r) {
      double q3[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double v = lds[(3 * r + c) * 64 + lane];
#pragma unroll
        for (int w = 1; w < kNearWaves; ++w) v += lds[(w * C + 3 * r + c) * 64 + lane];
        q3[c] = v;
      }
      a[r][0] -= fma(mxx, q3[0], fma(mxy, q3[1], mxz * q3[2]));
      a[r][1] -= fma(mxy, q3[0], fma(myy, q3[1], myz * q3[2]));
      a[r][2] -= fma(mxz, q3[0], fma(myz, q3[1], mzz * q3[2]));
    }
    __syncthreads();  // foot-point partials consumed: the buffer takes the results
  }
#pragma unroll
  for (int r = 0; r < K; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) lds[(wv * C + 3 * r + c) * 64 + lane] = a[r][c];
  __syncthreads();
  if (wv == 0 && valid) {
#pragma unroll
    for (int r = 0; r < K; ++r) {
      double* pb = near_part.p[r] + (size_t)slot * 3 * N;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double v = lds[(3 * r + c) * 64 + lane];
#pragma unroll
        for (int w = 1; w < kNearWaves; ++w) v += lds[(w * C + 3 * r + c) * 64 + lane];
        pb[(size_t)c * N + t] = scale * v;
      }
    }
  }
}

// Work item = pair * nch + target chunk; the pair list is ordered by source
// sphere, so an XCD's contiguous share re-reads the same upsampled densities.
template <int K>
__global__ __launch_bounds__(64 * kNearWaves) void k_near64(const double* __restrict__ ctr,
                                                            const double* __restrict__ off,
                                                            const double4* __restrict__ offup,
                                                            const double* __restrict__ shab,
                                                            const double* __restrict__ qup,
                                                            const double* __restrict__ coef,
                                                            const int* __restrict__ npairs, int n, int M, int N,
                                                            int nup, int p, int L, double scale, OPtrs near_part,
                                                            int nch, int total, int per) {
  __shared__ double lds[kNearWaves * 3 * K * 64];
  const int item = xcd_item(blockIdx.x, per);
  if (item >= total) return;  // uniform over the block
  near_body<K>(item / nch, item % nch, ctr, off, offup, shab, qup, coef, npairs, n, M, N, nup, p, L, scale, near_part,
               lds);
}

// ------------------------------------------------------------------ GEMM
//
// C(r, col) = sum_k A(r, k) * B(k, col), FP64, 32x32 output tiles,
// A(r, k) = A[r * lda + k] (at = 0) or A[k * lda + r] (at = 1),
// B(k, col) = B[col * ldb + k] (k contiguous) and C(r, col) stored at
// C[(r / rb) * rbs + (r % rb) * rs + (col / cb) * cbs + (col % cb) * ldc]: one
// kernel covers the per-sphere block products on the SoA field layout and the
// node-interleaved layouts (rs = 1 and cb >= Cn give C[(r / rb) rbs + col ldc + r % rb]).

constexpr int GBM = 32, GBN = 32, GBK = 16;
constexpr int kGemmSplitBelow = 2048;  // tiles per launch below which k is split over 4 waves
constexpr int GLS = GBK + 1;            // padded k stride of the LDS tiles (spreads the banks)

typedef double gemm_acc4 __attribute__((ext_vector_type(4)));

// One workgroup of GW waves per 32x32 output tile, on the FP64 matrix cores:
// each wave holds the tile as 2x2 blocks of 16x16 accumulated by
// V_MFMA_F64_16X16X4F64 (lane l supplies A(l%16, l/16) and B(l/16, l%16) of a
// 16x4 by 4x16 step and holds D(l/16 + 4j, l%16), j < 4). Wave w accumulates
// the k-blocks w, w + GW, ...; with GW = 4 (launches with few tiles: short and
// wide products, K up to 288) the partial tiles are added in wave order
// through LDS. Tile loads run along k, so consecutive lanes read consecutive
// addresses of A rows and B columns.
template <int GW>
__device__ __forceinline__ void gemm_tile(int bx, int by, int R, int Cn, int K, const double* __restrict__ A,
                                          int lda, const double* __restrict__ B, int ldb, double* __restrict__ C,
                                          int rb, long rbs, int ldc, int rs, int cb, long cbs, int at) {
  // per wave: A and B slices [32][GLS]; reused for the partial tiles [32][33]
  __shared__ double sh[GW][2 * GBM * GLS];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double* As = sh[wv];
  double* Bs = sh[wv] + GBM * GLS;
  const int r0 = bx * GBM, c0 = by * GBN;
  const int li = lane & 15, lk = lane >> 4;
  gemm_acc4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = gemm_acc4{0.0, 0.0, 0.0, 0.0};
  const int nkb = (K + GBK - 1) / GBK;
  const int steps = (nkb + GW - 1) / GW;  // same count for every wave (barriers)
  for (int st = 0; st < steps; ++st) {
    const int k0 = (st * GW + wv) * GBK;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = lane + e * 64;  // 0..511: k fastest
      const int kk = idx % GBK, rc = idx / GBK;
      const int gk = k0 + kk;
      const int gc = c0 + rc;
      if (!at) {
        const int gr = r0 + rc;
        As[rc * GLS + kk] = (gr < R && gk < K) ? A[(size_t)gr * lda + gk] : 0.0;
      }
      Bs[rc * GLS + kk] = (gc < Cn && gk < K) ? B[(size_t)gc * ldb + gk] : 0.0;
    }
    if (at) {
      // A stored by columns: rows fastest, so consecutive lanes read consecutive addresses
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int idx = lane + e * 64;
        const int rc = idx % GBM, kk = idx / GBM;
        const int gr = r0 + rc, gk = k0 + kk;
        As[rc * GLS + kk] = (gr < R && gk < K) ? A[(size_t)gk * lda + gr] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < GBK / 4; ++k4) {
      double av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        av[i] = As[(16 * i + li) * GLS + 4 * k4 + lk];
        bv[i] = Bs[(16 * i + li) * GLS + 4 * k4 + lk];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // element (i, j, q) of the lane: tile row 16 i + lk + 4 q, tile column 16 j + li
  double* part = &sh[0][0];  // (GW - 1) x [32][33] doubles fit in sh
  if (GW > 1 && wv > 0)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          part[((wv - 1) * GBM + 16 * i + lk + 4 * q) * (GBN + 1) + 16 * j + li] = acc[i][j][q];
  if (GW > 1) __syncthreads();
  if (wv == 0) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int tr = 16 * i + lk + 4 * q;
        const int gr = r0 + tr;
        if (gr >= R) continue;
        const size_t rowbase = (size_t)(gr / rb) * rbs + (size_t)(gr % rb) * rs;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int tc = 16 * j + li;
          const int gc = c0 + tc;
          double v = acc[i][j][q];
#pragma unroll
          for (int w = 1; w < GW; ++w) v += part[((w - 1) * GBM + tr) * (GBN + 1) + tc];
          if (gc < Cn) C[rowbase + (size_t)(gc / cb) * cbs + (size_t)(gc % cb) * ldc] = v;
        }
      }
  }
}

// 64x64 output tiles for large products (R and Cn in the hundreds or more, as in the
// preconditioner set-up): four waves, each a 32x32 quadrant of 2x2 16x16 MFMA blocks as
// above, share the LDS slices of A (64 x 16) and B (64 x 16), which halves the loads per
// flop of the 32x32 tiles; the next slices are loaded into registers while the MFMAs run
// on the current ones.
__device__ __forceinline__ void gemm_tile_big(int bx, int by, int R, int Cn, int K, const double* __restrict__ A,
                                              int lda, const double* __restrict__ B, int ldb, double* __restrict__ C,
                                              int rb, long rbs, int ldc, int rs, int cb, long cbs, int at_acc) {
  // at_acc bit 0: A stored by columns; bit 1: C += A B instead of C = A B
  const int at = at_acc & 1, accum = at_acc & 2;
  __shared__ double As[2 * GBM * GLS], Bs[2 * GBN * GLS];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const int r0 = bx * 2 * GBM, c0 = by * 2 * GBN;
  const int qr = (wv >> 1) * GBM, qc = (wv & 1) * GBN;
  const int li = lane & 15, lk = lane >> 4;
  gemm_acc4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = gemm_acc4{0.0, 0.0, 0.0, 0.0};
  double ra[4], rbv[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = t + e * 256;  // 0..1023
      {
        const int kk = at ? idx / (2 * GBM) : idx % GBK, rc = at ? idx % (2 * GBM) : idx / GBK;
        const int gr = r0 + rc, gk = k0 + kk;
        ra[e] = (gr < R && gk < K) ? (at ? A[(size_t)gk * lda + gr] : A[(size_t)gr * lda + gk]) : 0.0;
      }
      const int kk = idx % GBK, rc = idx / GBK;
      const int gc = c0 + rc, gk = k0 + kk;
      rbv[e] = (gc < Cn && gk < K) ? B[(size_t)gc * ldb + gk] : 0.0;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = t + e * 256;
      {
        const int kk = at ? idx / (2 * GBM) : idx % GBK, rc = at ? idx % (2 * GBM) : idx / GBK;
        As[rc * GLS + kk] = ra[e];
      }
      Bs[(idx / GBK) * GLS + idx % GBK] = rbv[e];
    }
  };
  const int nkb = (K + GBK - 1) / GBK;
  if (nkb > 0) {
    load(0);
    store();
  }
  __syncthreads();
  for (int kb = 0; kb < nkb; ++kb) {
    if (kb + 1 < nkb) load((kb + 1) * GBK);  // in flight during the MFMAs below
#pragma unroll
    for (int k4 = 0; k4 < GBK / 4; ++k4) {
      double av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        av[i] = As[(qr + 16 * i + li) * GLS + 4 * k4 + lk];
        bv[i] = Bs[(qc + 16 * i + li) * GLS + 4 * k4 + lk];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
    if (kb + 1 < nkb) store();
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int gr = r0 + qr + 16 * i + lk + 4 * q;
      if (gr >= R) continue;
      const size_t rowbase = (size_t)(gr / rb) * rbs + (size_t)(gr % rb) * rs;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int gc = c0 + qc + 16 * j + li;
        if (gc < Cn) {
          double* c = C + rowbase + (size_t)(gc / cb) * cbs + (size_t)(gc % cb) * ldc;
          *c = accum ? *c + acc[i][j][q] : acc[i][j][q];
        }
      }
    }
}

__global__ __launch_bounds__(256) void k_gemm64_big(int R, int Cn, int K, const double* __restrict__ A, int lda,
                                                    long Az, const double* __restrict__ B, long Bz, int ldb,
                                                    double* __restrict__ C, long Cz, int rb, long rbs, int ldc,
                                                    int at) {
  gemm_tile_big(blockIdx.x, blockIdx.y, R, Cn, K, A + (size_t)blockIdx.z * Az, lda, B + (size_t)blockIdx.z * Bz,
                ldb, C + (size_t)blockIdx.z * Cz, rb, rbs, ldc, 1, Cn, 0, at);
}

template <int GW>
__global__ __launch_bounds__(64 * GW) void k_gemm64(int R, int Cn, int K, const double* __restrict__ A, int lda,
                                                    long Az, const double* __restrict__ B, long Bz, int ldb,
                                                    double* __restrict__ C, long Cz, int rb, long rbs, int ldc,
                                                    int at) {
  gemm_tile<GW>(blockIdx.x, blockIdx.y, R, Cn, K, A + (size_t)blockIdx.z * Az, lda, B + (size_t)blockIdx.z * Bz, ldb,
                C + (size_t)blockIdx.z * Cz, rb, rbs, ldc, 1, Cn, 0, at);
}

// ------------------------------------------------- completion and slip RHS
//
// rhs(x) = u_s(x) - V[F,T](x), V the Stokeslet + rotlet field of every sphere:
// V = 1/(8 pi mu) sum_j F_j/|r| + r (r.F_j)/|r|^3 + T_j x r/|r|^3, r = x - c_j.
// u_s = -s (e - (e.n) n) where n.e > 0 (Janus half-cap slip), else 0.

__global__ __launch_bounds__(256) void k_rhs(const double* __restrict__ ctr, const double* __restrict__ FT,
                                             const double* __restrict__ axes, const double* __restrict__ off,
                                             int n, int M, int N, double a, double mu, double slip,
                                             double* __restrict__ rhs) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= N) return;
  const int i = t / n, k = t - i * n;
  const double x = ctr[3 * i] + off[3 * k], y = ctr[3 * i + 1] + off[3 * k + 1], z = ctr[3 * i + 2] + off[3 * k + 2];
  double ux = 0.0, uy = 0.0, uz = 0.0;
  if (FT) {
    for (int j = 0; j < M; ++j) {
      const double rx = x - ctr[3 * j], ry = y - ctr[3 * j + 1], rz = z - ctr[3 * j + 2];
      const double r2 = rx * rx + ry * ry + rz * rz;
      const double ri = 1.0 / sqrt(r2);
      const double ri3 = ri * ri * ri;
      const double* f = FT + 6 * j;
      const double rf = rx * f[0] + ry * f[1] + rz * f[2];
      ux += f[0] * ri + rx * rf * ri3 + (f[4] * rz - f[5] * ry) * ri3;
      uy += f[1] * ri + ry * rf * ri3 + (f[5] * rx - f[3] * rz) * ri3;
      uz += f[2] * ri + rz * rf * ri3 + (f[3] * ry - f[4] * rx) * ri3;
    }
    const double s = -1.0 / (8.0 * kPi * mu);
    ux *= s;
    uy *= s;
    uz *= s;
  }
  if (axes) {
    const double nx = off[3 * k] / a, ny = off[3 * k + 1] / a, nz = off[3 * k + 2] / a;
    const double ex = axes[3 * i], ey = axes[3 * i + 1], ez = axes[3 * i + 2];
    const double en = ex * nx + ey * ny + ez * nz;
    if (en > 0.0) {
      ux -= slip * (ex - en * nx);
      uy -= slip * (ey - en * ny);
      uz -= slip * (ez - en * nz);
    }
  }
  rhs[t] = ux;
  rhs[N + t] = uy;
  rhs[2 * N + t] = uz;
}

// ------------------------------------------ rigid moments and projection

// mom[j] = (sum w q, sum w o x q) over the nodes of sphere j (one block each).
__device__ __forceinline__ void moments_body(int j, const double* __restrict__ q, const double* __restrict__ off,
                                             const double* __restrict__ w, int n, int N, double* __restrict__ mom) {
  double m[6] = {0, 0, 0, 0, 0, 0};
  for (int k = threadIdx.x; k < n; k += 256) {
    const int t = j * n + k;
    const double qx = w[k] * q[t], qy = w[k] * q[N + t], qz = w[k] * q[2 * N + t];
    const double ox = off[3 * k], oy = off[3 * k + 1], oz = off[3 * k + 2];
    m[0] += qx;
    m[1] += qy;
    m[2] += qz;
    m[3] += oy * qz - oz * qy;
    m[4] += oz * qx - ox * qz;
    m[5] += ox * qy - oy * qx;
  }
  __shared__ double red[6][256];
#pragma unroll
  for (int c = 0; c < 6; ++c) red[c][threadIdx.x] = m[c];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
#pragma unroll
      for (int c = 0; c < 6; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 6) mom[6 * j + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_moments(const double* __restrict__ q, const double* __restrict__ off,
                                                 const double* __restrict__ w, int n, int N,
                                                 double* __restrict__ mom) {
  moments_body(blockIdx.x, q, off, w, n, N, mom);
}

// UO[j] = -(f/(4 pi a^2), 3 t/(8 pi a^4)): the rigid motion -P_j[q].
__global__ void k_rigid_velocity(const double* __restrict__ mom, int M, double a, double* __restrict__ UO) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  const double s1 = -1.0 / (4.0 * kPi * a * a), s2 = -3.0 / (8.0 * kPi * a * a * a * a);
  for (int c = 0; c < 3; ++c) {
    UO[6 * j + c] = s1 * mom[6 * j + c];
    UO[6 * j + 3 + c] = s2 * mom[6 * j + 3 + c];
  }
}

// y = q/2 + sum(self partials) + sum(far partials) + sum(near partials) + P[q],
// one thread per (component, node): element e = c * N + t.
__device__ __forceinline__ void combine_elem(int e, const double* __restrict__ q, const double* __restrict__ selfo,
                                             int nself, const double* __restrict__ far_part, int nchunks,
                                             const double* __restrict__ near_part, const int* __restrict__ npart,
                                             const double* __restrict__ mom, const double* __restrict__ off, int n,
                                             int N, double a, double* __restrict__ y) {
  const int c = e / N, t = e - c * N;
  const int i = t / n, k = t - i * n;
  const double s1 = 1.0 / (4.0 * kPi * a * a), s2 = 3.0 / (8.0 * kPi * a * a * a * a);
  const double* mj = mom + 6 * i;
  const double ox = off[3 * k], oy = off[3 * k + 1], oz = off[3 * k + 2];
  double P;
  if (c == 0)
    P = s1 * mj[0] + s2 * (mj[4] * oz - mj[5] * oy);
  else if (c == 1)
    P = s1 * mj[1] + s2 * (mj[5] * ox - mj[3] * oz);
  else
    P = s1 * mj[2] + s2 * (mj[3] * oy - mj[4] * ox);
  double v = 0.5 * q[e] + P;
  for (int h = 0; h < nself; ++h) v += selfo[(size_t)h * 3 * N + e];
  for (int h = 0; h < nchunks; ++h) v += far_part[(size_t)h * 3 * N + e];
  const int np = npart[i];
  for (int h = 0; h < np; ++h) v += near_part[(size_t)h * 3 * N + e];
  y[e] = v;
}

__global__ __launch_bounds__(256) void k_combine(const double* __restrict__ q, const double* __restrict__ selfo,
                                                 int nself, const double* __restrict__ far_part, int nchunks,
                                                 const double* __restrict__ near_part, const int* __restrict__ npart,
                                                 const double* __restrict__ mom, const double* __restrict__ off,
                                                 int n, int N, double a, double* __restrict__ y) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < 3 * N) combine_elem(e, q, selfo, nself, far_part, nchunks, near_part, npart, mom, off, n, N, a, y);
}

// ---------------------------------------------------------------- Arnoldi

// partial[v][b] = sum over block b's slice of V_v . w (grid: blocks x vectors).
__global__ __launch_bounds__(256) void k_dots(const double* __restrict__ V, long ldv, const double* __restrict__ w,
                                              long len, double* __restrict__ partial) {
  const int v = blockIdx.y;
  const double* x = V + (size_t)v * ldv;
  double s = 0.0;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < len; e += (long)gridDim.x * 256) s = fma(x[e], w[e], s);
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(size_t)v * gridDim.x + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_dots_finish(const double* __restrict__ partial, int nb,
                                                     double* __restrict__ out) {
  const int v = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) s += partial[(size_t)v * nb + b];
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[v] = red[0];
}

// w = beta * w + alpha * sum_v h[v] V_v   (h on the device).
__global__ __launch_bounds__(256) void k_combo(double* __restrict__ w, double beta, const double* __restrict__ V,
                                               long ldv, int nvec, const double* __restrict__ h, double alpha,
                                               long len) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= len) return;
  double s = 0.0;
  for (int v = 0; v < nvec; ++v) s = fma(h[v], V[(size_t)v * ldv + e], s);
  w[e] = (beta == 0.0 ? 0.0 : beta * w[e]) + alpha * s;
}

__global__ __launch_bounds__(256) void k_scale_copy(double* __restrict__ y, const double* __restrict__ x,
                                                    double s, long len) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e < len) y[e] = s * x[e];
}

// y = a * x + b * y
__global__ __launch_bounds__(256) void k_axpby(double* __restrict__ y, const double* __restrict__ x, double a,
                                               double b, long len) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e < len) y[e] = a * x[e] + b * y[e];
}

// ----------------------------------------------- many suspensions at once
//
// Every per-iteration kernel of the batched GMRES has a segmented form: one
// launch covers all systems; a descriptor table gives each system's pointers
// and sizes, and `start` is the first block (or element, or vector) of that
// system in the launch. Blocks find their system by binary search.

template <class D>
__device__ __forceinline__ int find_seg(const D* __restrict__ d, int nd, int idx) {
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].start <= idx)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <int GW>
__global__ __launch_bounds__(64 * GW) void k_gemm64_multi(const GemmDesc* __restrict__ d, int nd) {
  const int b = blockIdx.x;
  const GemmDesc D = d[find_seg(d, nd, b)];
  if (D.live && !*D.live) return;  // uniform over the block, before any barrier
  const int local = b - D.start;
  gemm_tile<GW>(local % D.tr, local / D.tr, D.R, D.Cn, D.K, D.A, D.lda, D.B, D.ldb, D.C, D.rb, D.rbs, D.ldc, D.rs,
                D.cb, D.cbs, D.at);
}

// Segmented launch of 64x64 tiles (descriptors built with 64-row tiles: tr = ceil(R / 64)).
__global__ __launch_bounds__(256) void k_gemm64_multi_big(const GemmDesc* __restrict__ d, int nd) {
  const int b = blockIdx.x;
  const GemmDesc D = d[find_seg(d, nd, b)];
  if (D.live && !*D.live) return;  // uniform over the block, before any barrier
  const int local = b - D.start;
  gemm_tile_big(local % D.tr, local / D.tr, D.R, D.Cn, D.K, D.A, D.lda, D.B, D.ldb, D.C, D.rb, D.rbs, D.ldc, D.rs,
                D.cb, D.cbs, D.at);
}

__global__ __launch_bounds__(256) void k_pack_multi(const PackDesc* __restrict__ d, int nd, int fp32) {
  const int g = blockIdx.x * 256 + threadIdx.x;
  const PackDesc D = d[find_seg(d, nd, g)];
  const int t = g - D.start;
  if (t < 0 || t >= D.N || (D.live && !*D.live)) return;
  const int k = t % D.n;
  const double wk = D.w[k];
  if (fp32) {
    float* e = (float*)D.src + (size_t)t * src32_stride(1);
    e[0] = (float)D.off[3 * k];
    e[1] = (float)D.off[3 * k + 1];
    e[2] = (float)D.off[3 * k + 2];
    for (int c = 0; c < 3; ++c) e[3 + c] = (float)(wk * D.q[(size_t)c * D.N + t]);
    e[6] = e[7] = 0.f;
  } else {
    double* e = (double*)D.src + (size_t)t * src64_stride(1);
    e[0] = D.off[3 * k];
    e[1] = D.off[3 * k + 1];
    e[2] = D.off[3 * k + 2];
    for (int c = 0; c < 3; ++c) e[3 + c] = wk * D.q[(size_t)c * D.N + t];
  }
}

__global__ __launch_bounds__(64 * kNearWaves) void k_near64_multi(const NearDesc* __restrict__ d, int nd) {
  __shared__ double lds[kNearWaves * 3 * 64];
  const int b = blockIdx.x;
  const NearDesc D = d[find_seg(d, nd, b)];
  if (D.live && !*D.live) return;
  const int local = b - D.start;
  OPtrs np{};
  np.p[0] = D.part;
  near_body<1>(local / D.nch, local % D.nch, D.ctr, D.off, D.offup, D.shab, D.qup, D.coef, D.pairs, D.n, D.M, D.N,
               D.nup, D.p, D.L, D.scale, np, lds);
}

__global__ __launch_bounds__(256) void k_moments_multi(const MomDesc* __restrict__ d, int nd) {
  const MomDesc D = d[find_seg(d, nd, blockIdx.x)];
  if (D.live && !*D.live) return;
  moments_body(blockIdx.x - D.start, D.q, D.off, D.w, D.n, D.N, D.mom);
}

__global__ __launch_bounds__(256) void k_combine_multi(const CombDesc* __restrict__ d, int nd) {
  const int g = blockIdx.x * 256 + threadIdx.x;
  const CombDesc D = d[find_seg(d, nd, g)];
  const int e = g - D.start;
  if (e < 0 || e >= 3 * D.N || (D.live && !*D.live)) return;
  combine_elem(e, D.q, D.selfo, 3, D.far, D.nchunks, D.near, D.npart, D.mom, D.off, D.n, D.N, D.a, D.y);
}

// partial[v][b] for the vectors of every system (grid: nb x total vectors)
__global__ __launch_bounds__(256) void k_dots_multi(const DotDesc* __restrict__ d, int nd) {
  const DotDesc D = d[find_seg(d, nd, blockIdx.y)];
  if (D.live && !*D.live) return;
  const int v = blockIdx.y - D.start;
  const double* x = D.V + (size_t)v * D.ldv;
  double s = 0.0;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < D.len; e += (long)gridDim.x * 256) s = fma(x[e], D.w[e], s);
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) D.partial[(size_t)v * gridDim.x + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_dots_finish_multi(const DotDesc* __restrict__ d, int nd, int nb) {
  const DotDesc D = d[find_seg(d, nd, blockIdx.x)];
  if (D.live && !*D.live) return;
  const int v = blockIdx.x - D.start;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) s += D.partial[(size_t)v * nb + b];
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) D.out[v] = red[0];
}

// w = beta w + alpha sum_v h[v] V_v for every system (elementwise, segmented)
__global__ __launch_bounds__(256) void k_combo_multi(const ComboDesc* __restrict__ d, int nd) {
  const int g = blockIdx.x * 256 + threadIdx.x;
  const ComboDesc D = d[find_seg(d, nd, g)];
  const long e = g - D.start;
  if (e < 0 || e >= D.len || (D.live && !*D.live)) return;
  double s = 0.0;
  for (int v = 0; v < D.nvec; ++v) s = fma(D.h[v], D.V[(size_t)v * D.ldv + e], s);
  D.w[e] = (D.beta == 0.0 ? 0.0 : D.beta * D.w[e]) + D.alpha * s;
}

// One GMRES step per active system (one thread each): Hessenberg column k from the
// two CGS2 passes, the earlier Givens rotations applied to it, a new rotation, the
// residual estimate |g_{k+1}| and the end test (converged, or cycle full / iteration
// cap). A system that goes on gets inv_hn = 1/|w| for the normalisation of V[k+1];
// one that ends keeps V[k+1] unnormalised (hn kept), as the host loop does.
__global__ void k_gmres_step(GmSys* __restrict__ sys, double* __restrict__ hess, const double* __restrict__ hbuf,
                             int hs, int m, int ns) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  GmSys S = sys[i];
  if (!S.active) return;
  const int k = S.k;
  double* H = hess + (size_t)i * gm_stride(m);
  double* cs = H + (size_t)(m + 1) * m;
  double* sn = cs + m;
  double* g = sn + m;
  const double* hb = hbuf + (size_t)i * hs;
  if (k == 0) g[0] = S.bnorm;  // cold start: the residual is the right-hand side
  for (int r = 0; r <= k; ++r) H[r * m + k] = hb[r] + hb[m + 1 + r];
  const double hn = sqrt(fmax(0.0, hb[2 * (m + 1)]));
  H[(k + 1) * m + k] = hn;
  for (int r = 0; r < k; ++r) {
    const double t0 = cs[r] * H[r * m + k] + sn[r] * H[(r + 1) * m + k];
    H[(r + 1) * m + k] = -sn[r] * H[r * m + k] + cs[r] * H[(r + 1) * m + k];
    H[r * m + k] = t0;
  }
  const double den = sqrt(H[k * m + k] * H[k * m + k] + hn * hn);
  S.its += 1;
  if (!(den > 0.0) || !isfinite(den) || !isfinite(hn)) {
    S.err = 1;
    S.active = 0;
    sys[i] = S;
    return;
  }
  cs[k] = H[k * m + k] / den;
  sn[k] = H[(k + 1) * m + k] / den;
  H[k * m + k] = den;
  H[(k + 1) * m + k] = 0.0;
  g[k + 1] = -sn[k] * g[k];
  g[k] = cs[k] * g[k];
  S.relres = fabs(g[k + 1]) / S.bnorm;
  const bool conv = fabs(g[k + 1]) <= S.tol * S.bnorm || hn == 0.0;
  const bool full = (k + 1 == m) || S.its >= S.max_iter;
  S.hn = hn;
  if (!conv && !full) {
    S.inv_hn = 1.0 / hn;
    S.k = k + 1;
  } else {
    S.active = 0;
    S.conv = conv ? 1 : 0;
  }
  sys[i] = S;
}

// w *= s for every segment whose system is still active (segmented, elementwise).
__global__ __launch_bounds__(256) void k_scale_multi(const ScaleDesc* __restrict__ d, int nd) {
  const int g = blockIdx.x * 256 + threadIdx.x;
  const ScaleDesc D = d[find_seg(d, nd, g)];
  const long e = g - D.start;
  if (e < 0 || e >= D.len || (D.live && !*D.live)) return;
  D.w[e] *= *D.s;
}

// ------------------------------------------------------------- launchers

static inline unsigned nblk(long n, int b = 256) { return (unsigned)((n + b - 1) / b); }

template <int K>
static void pack_k(hipStream_t s, int prec, const QPtrs& q, const double* off, const double* w, int n, int N,
                   void* src) {
  if (prec == 1)
    hipLaunchKernelGGL(k_pack32<K>, dim3(nblk(N)), dim3(256), 0, s, q, off, w, n, N, (float*)src);
  else
    hipLaunchKernelGGL(k_pack64<K>, dim3(nblk(N)), dim3(256), 0, s, q, off, w, n, N, (double*)src);
}

void launch_pack_coarse(hipStream_t s, int prec, int K, const double* qc, const double* off, const double* w, int nc,
                        int Nc, void* src) {
  const int f = prec == 1 ? 1 : 0;
  switch (K) {
    case 1: hipLaunchKernelGGL(k_pack_coarse<1>, dim3(nblk(Nc)), dim3(256), 0, s, qc, off, w, nc, Nc, f, src); break;
    case 2: hipLaunchKernelGGL(k_pack_coarse<2>, dim3(nblk(Nc)), dim3(256), 0, s, qc, off, w, nc, Nc, f, src); break;
    case 3: hipLaunchKernelGGL(k_pack_coarse<3>, dim3(nblk(Nc)), dim3(256), 0, s, qc, off, w, nc, Nc, f, src); break;
    case 4: hipLaunchKernelGGL(k_pack_coarse<4>, dim3(nblk(Nc)), dim3(256), 0, s, qc, off, w, nc, Nc, f, src); break;
    case 5: hipLaunchKernelGGL(k_pack_coarse<5>, dim3(nblk(Nc)), dim3(256), 0, s, qc, off, w, nc, Nc, f, src); break;
    default: hipLaunchKernelGGL(k_pack_coarse<6>, dim3(nblk(Nc)), dim3(256), 0, s, qc, off, w, nc, Nc, f, src); break;
  }
}

void launch_pack(hipStream_t s, int prec, int K, const QPtrs& q, const double* off, const double* w, int n, int N,
                 void* src) {
  switch (K) {
    case 1: pack_k<1>(s, prec, q, off, w, n, N, src); break;
    case 2: pack_k<2>(s, prec, q, off, w, n, N, src); break;
    case 3: pack_k<3>(s, prec, q, off, w, n, N, src); break;
    case 4: pack_k<4>(s, prec, q, off, w, n, N, src); break;
    case 5: pack_k<5>(s, prec, q, off, w, n, N, src); break;
    default: pack_k<6>(s, prec, q, off, w, n, N, src); break;
  }
}

template <int K>
static void far_k(hipStream_t s, int prec, int tpt, const void* src, const double* off, const double* ctr,
                  const unsigned char* cls, int n, int ns, int M, int N, int spc, int nchunks, double scale,
                  const OPtrs& part) {
  const int per_block = prec == 1 ? (tpt == 0 ? 64 : 256 * tpt) : 256;
  const int ntb = (int)nblk(N, per_block);
  const int total = ntb * nchunks, per = (total + kXcds - 1) / kXcds;
  const dim3 grid(per * kXcds);
  if (prec == 1) {
    if (tpt == 0)
      hipLaunchKernelGGL((k_far32s<K>), grid, dim3(256), 0, s, (const float*)src, off, ctr, cls, n, ns, M, N, spc,
                         scale, part, ntb, total, per);
    else if (tpt == 2)
      hipLaunchKernelGGL((k_far32<2, K>), grid, dim3(256), 0, s, (const float*)src, off, ctr, cls, n, ns, M, N, spc,
                         scale, part, ntb, total, per);
    else
      hipLaunchKernelGGL((k_far32<1, K>), grid, dim3(256), 0, s, (const float*)src, off, ctr, cls, n, ns, M, N, spc,
                         scale, part, ntb, total, per);
  } else {
    hipLaunchKernelGGL(k_far64<K>, grid, dim3(256), 0, s, (const double*)src, off, ctr, cls, n, ns, M, N, spc,
                       scale, part, ntb, total, per);
  }
}

void launch_far(hipStream_t s, int prec, int K, int tpt, const void* src, const double* off, const double* ctr,
                const unsigned char* cls, int n, int ns, int M, int N, int spc, int nchunks, double scale,
                const OPtrs& part) {
  const int t1 = tpt == 0 ? 0 : 1;  // two targets per thread only for K <= 2
  switch (K) {
    case 1: far_k<1>(s, prec, tpt, src, off, ctr, cls, n, ns, M, N, spc, nchunks, scale, part); break;
    case 2: far_k<2>(s, prec, tpt, src, off, ctr, cls, n, ns, M, N, spc, nchunks, scale, part); break;
    case 3: far_k<3>(s, prec, t1, src, off, ctr, cls, n, ns, M, N, spc, nchunks, scale, part); break;
    case 4: far_k<4>(s, prec, t1, src, off, ctr, cls, n, ns, M, N, spc, nchunks, scale, part); break;
    case 5: far_k<5>(s, prec, t1, src, off, ctr, cls, n, ns, M, N, spc, nchunks, scale, part); break;
    default: far_k<6>(s, prec, t1, src, off, ctr, cls, n, ns, M, N, spc, nchunks, scale, part); break;
  }
}

template <int K>
static void far_kc(hipStream_t s, int prec, const void* src, const double* off, const double* ctr,
                   const unsigned char* cls, const unsigned char* cls2, int n, int ns, int ns1, int M, int N, int spc,
                   int nchunks, double scale, const OPtrs& part) {
  const int ntb = (int)nblk(N, 256);
  const int total = ntb * nchunks, per = (total + kXcds - 1) / kXcds;
  const dim3 grid(per * kXcds);
  if (prec == 1)
    hipLaunchKernelGGL(k_far32c<K>, grid, dim3(256), 0, s, (const float*)src, off, ctr, cls, cls2, n, ns, ns1, M, N,
                       spc, scale, part, ntb, total, per);
  else
    hipLaunchKernelGGL(k_far64c<K>, grid, dim3(256), 0, s, (const double*)src, off, ctr, cls, cls2, n, ns, ns1, M, N,
                       spc, scale, part, ntb, total, per);
}

void launch_far_coarse(hipStream_t s, int prec, int K, const void* src, const double* off, const double* ctr,
                       const unsigned char* cls, const unsigned char* cls2, int n, int ns, int ns1, int M, int N,
                       int spc, int nchunks, double scale, const OPtrs& part) {
  switch (K) {
    case 1: far_kc<1>(s, prec, src, off, ctr, cls, cls2, n, ns, ns1, M, N, spc, nchunks, scale, part); break;
    case 2: far_kc<2>(s, prec, src, off, ctr, cls, cls2, n, ns, ns1, M, N, spc, nchunks, scale, part); break;
    case 3: far_kc<3>(s, prec, src, off, ctr, cls, cls2, n, ns, ns1, M, N, spc, nchunks, scale, part); break;
    case 4: far_kc<4>(s, prec, src, off, ctr, cls, cls2, n, ns, ns1, M, N, spc, nchunks, scale, part); break;
    case 5: far_kc<5>(s, prec, src, off, ctr, cls, cls2, n, ns, ns1, M, N, spc, nchunks, scale, part); break;
    default: far_kc<6>(s, prec, src, off, ctr, cls, cls2, n, ns, ns1, M, N, spc, nchunks, scale, part); break;
  }
}

void launch_far_multi(hipStream_t s, int prec, int tpt, const FarDesc* desc, int ndesc, int nitems) {
  if (nitems <= 0) return;
  if (prec == 1) {
    if (tpt == 0)
      hipLaunchKernelGGL(k_far32_multi<0>, dim3(nitems), dim3(256), 0, s, desc, ndesc);
    else if (tpt == 2)
      hipLaunchKernelGGL(k_far32_multi<2>, dim3(nitems), dim3(256), 0, s, desc, ndesc);
    else
      hipLaunchKernelGGL(k_far32_multi<1>, dim3(nitems), dim3(256), 0, s, desc, ndesc);
  } else {
    hipLaunchKernelGGL(k_far64_multi, dim3(nitems), dim3(256), 0, s, desc, ndesc);
  }
}

void launch_near(hipStream_t s, int K, int npairs_count, const double* ctr, const double* off, const double4* offup,
                 const double* shab, const double* qup, const double* coef, const int* npairs, int n, int M, int N,
                 int nup, int p, int L, double scale, const OPtrs& near_part) {
  if (npairs_count <= 0) return;
  const int nch = (n + 63) / 64, total = npairs_count * nch, per = (total + kXcds - 1) / kXcds;
  const dim3 g(per * kXcds);
#define NEARK(KK)                                                                                                \
  hipLaunchKernelGGL(k_near64<KK>, g, dim3(64 * kNearWaves), 0, s, ctr, off, offup, shab, qup, coef, npairs, n, M, \
                     N, nup, p, L, scale, near_part, nch, total, per)
  switch (K) {
    case 1: NEARK(1); break;
    case 2: NEARK(2); break;
    case 3: NEARK(3); break;
    case 4: NEARK(4); break;
    case 5: NEARK(5); break;
    default: NEARK(6); break;
  }
#undef NEARK
}

void launch_gemm64(hipStream_t s, int R, int Cn, int K, const double* A, int lda, long Az, const double* B, long Bz,
                   int ldb, double* C, long Cz, int rb, long rbs, int ldc, int batch, int at) {
  const dim3 g((R + GBM - 1) / GBM, (Cn + GBN - 1) / GBN, batch);
  if ((long)g.x * g.y * g.z < kGemmSplitBelow)
    hipLaunchKernelGGL(k_gemm64<4>, g, dim3(256), 0, s, R, Cn, K, A, lda, Az, B, Bz, ldb, C, Cz, rb, rbs, ldc, at);
  else
    hipLaunchKernelGGL(k_gemm64<1>, g, dim3(64), 0, s, R, Cn, K, A, lda, Az, B, Bz, ldb, C, Cz, rb, rbs, ldc, at);
}
void launch_gemm64_big(hipStream_t s, int R, int Cn, int K, const double* A, int lda, long Az, const double* B,
                       long Bz, int ldb, double* C, long Cz, int rb, long rbs, int ldc, int batch, int at) {
  const dim3 g((R + 2 * GBM - 1) / (2 * GBM), (Cn + 2 * GBN - 1) / (2 * GBN), batch);
  hipLaunchKernelGGL(k_gemm64_big, g, dim3(256), 0, s, R, Cn, K, A, lda, Az, B, Bz, ldb, C, Cz, rb, rbs, ldc, at);
}
void launch_gemm64_multi_big(hipStream_t s, const GemmDesc* d, int nd, int nblocks) {
  if (nblocks > 0) hipLaunchKernelGGL(k_gemm64_multi_big, dim3(nblocks), dim3(256), 0, s, d, nd);
}
void launch_rhs(hipStream_t s, const double* ctr, const double* FT, const double* axes, const double* off, int n,
                int M, int N, double a, double mu, double slip, double* rhs) {
  hipLaunchKernelGGL(k_rhs, dim3(nblk(N)), dim3(256), 0, s, ctr, FT, axes, off, n, M, N, a, mu, slip, rhs);
}
void launch_moments(hipStream_t s, const double* q, const double* off, const double* w, int n, int M, int N,
                    double* mom) {
  hipLaunchKernelGGL(k_moments, dim3(M), dim3(256), 0, s, q, off, w, n, N, mom);
}
void launch_rigid_velocity(hipStream_t s, const double* mom, int M, double a, double* UO) {
  hipLaunchKernelGGL(k_rigid_velocity, dim3(nblk(M, 64)), dim3(64), 0, s, mom, M, a, UO);
}
void launch_combine(hipStream_t s, const double* q, const double* selfo, int nself, const double* far_part,
                    int nchunks, const double* near_part, const int* npart, const double* mom, const double* off,
                    int n, int N, double a, double* y) {
  hipLaunchKernelGGL(k_combine, dim3(nblk(3L * N)), dim3(256), 0, s, q, selfo, nself, far_part, nchunks, near_part,
                     npart, mom, off, n, N, a, y);
}
void launch_dots(hipStream_t s, const double* V, long ldv, int nvec, const double* w, long len, int nb,
                 double* partial, double* out) {
  hipLaunchKernelGGL(k_dots, dim3(nb, nvec), dim3(256), 0, s, V, ldv, w, len, partial);
  hipLaunchKernelGGL(k_dots_finish, dim3(nvec), dim3(256), 0, s, partial, nb, out);
}
void launch_combo(hipStream_t s, double* w, double beta, const double* V, long ldv, int nvec, const double* h,
                  double alpha, long len) {
  hipLaunchKernelGGL(k_combo, dim3(nblk(len)), dim3(256), 0, s, w, beta, V, ldv, nvec, h, alpha, len);
}
void launch_scale_copy(hipStream_t s, double* y, const double* x, double a, long len) {
  hipLaunchKernelGGL(k_scale_copy, dim3(nblk(len)), dim3(256), 0, s, y, x, a, len);
}
void launch_axpby(hipStream_t s, double* y, const double* x, double a, double b, long len) {
  hipLaunchKernelGGL(k_axpby, dim3(nblk(len)), dim3(256), 0, s, y, x, a, b, len);
}

}  // namespace bipqn

namespace bipqn {
static inline unsigned nblk2(long n, int b = 256) { return (unsigned)((n + b - 1) / b); }
void launch_gemm64_multi(hipStream_t s, const GemmDesc* d, int nd, int nblocks) {
  if (nblocks <= 0) return;
  if (nblocks < kGemmSplitBelow)
    hipLaunchKernelGGL(k_gemm64_multi<4>, dim3(nblocks), dim3(256), 0, s, d, nd);
  else
    hipLaunchKernelGGL(k_gemm64_multi<1>, dim3(nblocks), dim3(64), 0, s, d, nd);
}
void launch_pack_multi(hipStream_t s, const PackDesc* d, int nd, int total, int fp32) {
  if (total > 0) hipLaunchKernelGGL(k_pack_multi, dim3(nblk2(total)), dim3(256), 0, s, d, nd, fp32);
}
void launch_near_multi(hipStream_t s, const NearDesc* d, int nd, int nblocks) {
  if (nblocks > 0) hipLaunchKernelGGL(k_near64_multi, dim3(nblocks), dim3(64 * kNearWaves), 0, s, d, nd);
}
void launch_moments_multi(hipStream_t s, const MomDesc* d, int nd, int nblocks) {
  if (nblocks > 0) hipLaunchKernelGGL(k_moments_multi, dim3(nblocks), dim3(256), 0, s, d, nd);
}
void launch_combine_multi(hipStream_t s, const CombDesc* d, int nd, int total) {
  if (total > 0) hipLaunchKernelGGL(k_combine_multi, dim3(nblk2(total)), dim3(256), 0, s, d, nd);
}
void launch_dots_multi(hipStream_t s, const DotDesc* d, int nd, int nvec_total, int nb) {
  if (nvec_total <= 0) return;
  hipLaunchKernelGGL(k_dots_multi, dim3(nb, nvec_total), dim3(256), 0, s, d, nd);
  hipLaunchKernelGGL(k_dots_finish_multi, dim3(nvec_total), dim3(256), 0, s, d, nd, nb);
}
void launch_combo_multi(hipStream_t s, const ComboDesc* d, int nd, int total) {
  if (total > 0) hipLaunchKernelGGL(k_combo_multi, dim3(nblk2(total)), dim3(256), 0, s, d, nd);
}
void launch_gmres_step(hipStream_t s, GmSys* sys, double* hess, const double* hbuf, int hs, int m, int ns) {
  if (ns > 0) hipLaunchKernelGGL(k_gmres_step, dim3(nblk2(ns, 64)), dim3(64), 0, s, sys, hess, hbuf, hs, m, ns);
}
void launch_scale_multi(hipStream_t s, const ScaleDesc* d, int nd, int total) {
  if (total > 0) hipLaunchKernelGGL(k_scale_multi, dim3(nblk2(total)), dim3(256), 0, s, d, nd);
}
}  // namespace bipqn
