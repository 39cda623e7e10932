// Device kernels of the mobility product (one HIP translation unit).
//
// Vector layout: surface fields are SoA [3][N] doubles, node index
// t = sphere * n + local node, local node = theta_row * n_phi + phi_col.
#include "kernels.hpp"

namespace bipqn {

// --------------------------------------------------------------- packing

// Far-tile sources: {o.x, o.y, o.z, wq.x} {wq.y, wq.z, 0, 0} per node, FP32.
__global__ __launch_bounds__(256) void k_pack32(const double* __restrict__ q, const double* __restrict__ off,
                                                const double* __restrict__ w, int n, int N,
                                                float4* __restrict__ src) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int k = t % n;
  const double wk = w[k];
  src[2 * t] = make_float4((float)off[3 * k], (float)off[3 * k + 1], (float)off[3 * k + 2], (float)(wk * q[t]));
  src[2 * t + 1] = make_float4((float)(wk * q[N + t]), (float)(wk * q[2 * N + t]), 0.f, 0.f);
}

// FP64 sources: {o.x, o.y, o.z, wq.x, wq.y, wq.z, 0, 0} per node.
__global__ __launch_bounds__(256) void k_pack64(const double* __restrict__ q, const double* __restrict__ off,
                                                const double* __restrict__ w, int n, int N,
                                                double2* __restrict__ src) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int k = t % n;
  const double wk = w[k];
  src[4 * t] = make_double2(off[3 * k], off[3 * k + 1]);
  src[4 * t + 1] = make_double2(off[3 * k + 2], wk * q[t]);
  src[4 * t + 2] = make_double2(wk * q[N + t], wk * q[2 * N + t]);
  src[4 * t + 3] = make_double2(0.0, 0.0);
}

// ----------------------------------------------------------- far pair sum
//
// u(x) += 3/(4 pi a) sum_y r (r.wq_y)(r.o_y)/|r|^5, r = x - y, over source
// spheres j != i that are not near sphere i. One thread owns TPT targets; the
// grid's y dimension splits the source spheres into chunks. The source node
// stream is wave-uniform, so its loads go through the scalar unit and its
// values enter the VALU as scalar operands. Target positions are taken
// relative to the source sphere's centre, X = (c_i - c_j) + o_x, formed in
// FP64 and rounded once, so r = X - o_y carries no large-coordinate
// cancellation. Each sphere's contribution (one tile) is summed in the pair
// precision and added to an FP64 accumulator.

template <int TPT>
__global__ __launch_bounds__(256) void k_far32(const float4* __restrict__ src, const double* __restrict__ off,
                                               const double* __restrict__ ctr, const unsigned char* __restrict__ cls,
                                               int n, int M, int N, int spc, double scale,
                                               double* __restrict__ part) {
  const int j0 = blockIdx.y * spc;
  const int j1 = min(M, j0 + spc);
  int ti[TPT];
  bool valid[TPT];
  double px[TPT], py[TPT], pz[TPT];
  double ax[TPT], ay[TPT], az[TPT];
#pragma unroll
  for (int u = 0; u < TPT; ++u) {
    const int t = blockIdx.x * 256 * TPT + u * 256 + threadIdx.x;
    valid[u] = t < N;
    const int tt = valid[u] ? t : N - 1;
    const int i = tt / n;
    const int k = tt - i * n;
    ti[u] = i;
    px[u] = ctr[3 * i] + 0.0;
    py[u] = ctr[3 * i + 1];
    pz[u] = ctr[3 * i + 2];
    // keep the offset separately to form (c_i - c_j) + o_x per tile
    ax[u] = off[3 * k];
    ay[u] = off[3 * k + 1];
    az[u] = off[3 * k + 2];
  }
  double ox[TPT], oy[TPT], oz[TPT];
#pragma unroll
  for (int u = 0; u < TPT; ++u) {
    ox[u] = ax[u];
    oy[u] = ay[u];
    oz[u] = az[u];
    ax[u] = ay[u] = az[u] = 0.0;
  }
  for (int j = j0; j < j1; ++j) {
    const double cjx = ctr[3 * j], cjy = ctr[3 * j + 1], cjz = ctr[3 * j + 2];
    bool act[TPT];
    int any = 0;
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
      act[u] = valid[u] && cls[ti[u] * M + j] == 0;
      any |= act[u];
    }
    if (!__any(any)) continue;
    float Xx[TPT], Xy[TPT], Xz[TPT], sx[TPT], sy[TPT], sz[TPT];
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
      Xx[u] = act[u] ? (float)((px[u] - cjx) + ox[u]) : 1.0e4f;
      Xy[u] = act[u] ? (float)((py[u] - cjy) + oy[u]) : 0.0f;
      Xz[u] = act[u] ? (float)((pz[u] - cjz) + oz[u]) : 0.0f;
      sx[u] = sy[u] = sz[u] = 0.0f;
    }
    const float4* s = src + 2 * (size_t)j * n;
#pragma unroll 4
    for (int kk = 0; kk < n; ++kk) {
      const float4 a = s[2 * kk];
      const float4 b = s[2 * kk + 1];
#pragma unroll
      for (int u = 0; u < TPT; ++u) {
        const float rx = Xx[u] - a.x, ry = Xy[u] - a.y, rz = Xz[u] - a.z;
        const float r2 = fmaf(rx, rx, fmaf(ry, ry, rz * rz));
        const float ri = __builtin_amdgcn_rsqf(r2);
        const float ri2 = ri * ri;
        const float rn = fmaf(rx, a.x, fmaf(ry, a.y, rz * a.z));
        const float rq = fmaf(rx, a.w, fmaf(ry, b.x, rz * b.y));
        const float c = rn * rq * ri * ri2 * ri2;
        sx[u] = fmaf(c, rx, sx[u]);
        sy[u] = fmaf(c, ry, sy[u]);
        sz[u] = fmaf(c, rz, sz[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
      if (act[u]) {
        ax[u] += (double)sx[u];
        ay[u] += (double)sy[u];
        az[u] += (double)sz[u];
      }
    }
  }
  double* pb = part + (size_t)blockIdx.y * 3 * N;
#pragma unroll
  for (int u = 0; u < TPT; ++u) {
    const int t = blockIdx.x * 256 * TPT + u * 256 + threadIdx.x;
    if (valid[u]) {
      pb[t] = scale * ax[u];
      pb[N + t] = scale * ay[u];
      pb[2 * N + t] = scale * az[u];
    }
  }
}

__global__ __launch_bounds__(256) void k_far64(const double2* __restrict__ src, const double* __restrict__ off,
                                               const double* __restrict__ ctr, const unsigned char* __restrict__ cls,
                                               int n, int M, int N, int spc, double scale,
                                               double* __restrict__ part) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  const bool valid = t < N;
  const int tt = valid ? t : N - 1;
  const int i = tt / n;
  const int k = tt - i * n;
  const double px = ctr[3 * i], py = ctr[3 * i + 1], pz = ctr[3 * i + 2];
  const double ox = off[3 * k], oy = off[3 * k + 1], oz = off[3 * k + 2];
  const int j0 = blockIdx.y * spc;
  const int j1 = min(M, j0 + spc);
  double ax = 0.0, ay = 0.0, az = 0.0;
  for (int j = j0; j < j1; ++j) {
    const bool act = valid && cls[i * M + j] == 0;
    if (!__any(act)) continue;
    const double Xx = act ? (px - ctr[3 * j]) + ox : 1.0e4;
    const double Xy = act ? (py - ctr[3 * j + 1]) + oy : 0.0;
    const double Xz = act ? (pz - ctr[3 * j + 2]) + oz : 0.0;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    const double2* s = src + 4 * (size_t)j * n;
#pragma unroll 2
    for (int kk = 0; kk < n; ++kk) {
      const double2 a = s[4 * kk], b = s[4 * kk + 1], c2 = s[4 * kk + 2];
      const double rx = Xx - a.x, ry = Xy - a.y, rz = Xz - b.x;
      const double r2 = fma(rx, rx, fma(ry, ry, rz * rz));
      const double ri = rsqrt(r2);
      const double ri2 = ri * ri;
      const double rn = fma(rx, a.x, fma(ry, a.y, rz * b.x));
      const double rq = fma(rx, b.y, fma(ry, c2.x, rz * c2.y));
      const double c = rn * rq * ri * ri2 * ri2;
      sx = fma(c, rx, sx);
      sy = fma(c, ry, sy);
      sz = fma(c, rz, sz);
    }
    if (act) {
      ax += sx;
      ay += sy;
      az += sz;
    }
  }
  if (valid) {
    double* pb = part + (size_t)blockIdx.y * 3 * N;
    pb[t] = scale * ax;
    pb[N + t] = scale * ay;
    pb[2 * N + t] = scale * az;
  }
}

// ---------------------------------------------------------- near pair sum
//
// For each target and each near partner sphere j (grid y = partner slot):
// sum over the upsampled nodes f of sphere j of w_f K(x, y_f)(q_f - q_j(x*)),
// x* the foot point of x on sphere j, q_j(x*) evaluated from the degree-p
// harmonic coefficients of the density (constant-density subtraction).

__global__ __launch_bounds__(256) void k_near64(const double* __restrict__ ctr, const double* __restrict__ off,
                                                const double4* __restrict__ offup, const double* __restrict__ qup,
                                                const double* __restrict__ coef, const int* __restrict__ partners,
                                                const int* __restrict__ npart, int n, int M, int N, int nup, int p,
                                                int L, double scale, double* __restrict__ near_part) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int slot = blockIdx.y;
  if (t >= N) return;
  const int i = t / n;
  if (slot >= npart[i]) return;
  const int j = partners[i * kMaxNear + slot];
  const int k = t - i * n;
  const double Xx = (ctr[3 * i] + off[3 * k]) - ctr[3 * j];
  const double Xy = (ctr[3 * i + 1] + off[3 * k + 1]) - ctr[3 * j + 1];
  const double Xz = (ctr[3 * i + 2] + off[3 * k + 2]) - ctr[3 * j + 2];
  const double rho = sqrt(Xx * Xx + Xy * Xy);
  const double R = sqrt(rho * rho + Xz * Xz);
  const double ct = Xz / R, st = rho / R;
  const double cp = rho > 0.0 ? Xx / rho : 1.0, sp = rho > 0.0 ? Xy / rho : 0.0;
  const size_t ML = (size_t)M * L;
  const double* cx = coef + (size_t)j * L;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  real_sh_visit(p, ct, st, cp, sp, [&](int idx, double y) {
    fx = fma(y, cx[idx], fx);
    fy = fma(y, cx[ML + idx], fy);
    fz = fma(y, cx[2 * ML + idx], fz);
  });
  const size_t MU = (size_t)M * nup;
  const double* qx = qup + (size_t)j * nup;
  double ax = 0.0, ay = 0.0, az = 0.0;
  for (int f = 0; f < nup; ++f) {
    const double4 o = offup[f];
    const double rx = Xx - o.x, ry = Xy - o.y, rz = Xz - o.z;
    const double r2 = fma(rx, rx, fma(ry, ry, rz * rz));
    const double ri = rsqrt(r2);
    const double ri2 = ri * ri;
    const double dqx = qx[f] - fx, dqy = qx[MU + f] - fy, dqz = qx[2 * MU + f] - fz;
    const double rn = fma(rx, o.x, fma(ry, o.y, rz * o.z));
    const double rq = o.w * fma(rx, dqx, fma(ry, dqy, rz * dqz));
    const double c = rn * rq * ri * ri2 * ri2;
    ax = fma(c, rx, ax);
    ay = fma(c, ry, ay);
    az = fma(c, rz, az);
  }
  double* pb = near_part + (size_t)slot * 3 * N;
  pb[t] = scale * ax;
  pb[N + t] = scale * ay;
  pb[2 * N + t] = scale * az;
}

// Same sum, organised by near sphere pair: grid (pair, 64-target chunk). All
// lanes of a wave share the source sphere j, so the upsampled source stream and
// the harmonic coefficients of q_j are wave-uniform (scalar loads).
__global__ __launch_bounds__(64) void k_near64p(const double* __restrict__ ctr, const double* __restrict__ off,
                                                const double4* __restrict__ offup, const double* __restrict__ qup,
                                                const double* __restrict__ coef, const int* __restrict__ npairs,
                                                int n, int M, int N, int nup, int p, int L, double scale,
                                                double* __restrict__ near_part) {
  const int i = npairs[3 * blockIdx.x], j = npairs[3 * blockIdx.x + 1], slot = npairs[3 * blockIdx.x + 2];
  const int k = blockIdx.y * 64 + threadIdx.x;
  const bool valid = k < n;
  const int kk = valid ? k : n - 1;
  const int t = i * n + kk;
  const double Xx = (ctr[3 * i] + off[3 * kk]) - ctr[3 * j];
  const double Xy = (ctr[3 * i + 1] + off[3 * kk + 1]) - ctr[3 * j + 1];
  const double Xz = (ctr[3 * i + 2] + off[3 * kk + 2]) - ctr[3 * j + 2];
  const double rho = sqrt(Xx * Xx + Xy * Xy);
  const double R = sqrt(rho * rho + Xz * Xz);
  const double ct = Xz / R, st = rho / R;
  const double cp = rho > 0.0 ? Xx / rho : 1.0, sp = rho > 0.0 ? Xy / rho : 0.0;
  const size_t ML = (size_t)M * L;
  const double* cx = coef + (size_t)j * L;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  real_sh_visit(p, ct, st, cp, sp, [&](int idx, double y) {
    fx = fma(y, cx[idx], fx);
    fy = fma(y, cx[ML + idx], fy);
    fz = fma(y, cx[2 * ML + idx], fz);
  });
  const size_t MU = (size_t)M * nup;
  const double* qx = qup + (size_t)j * nup;
  double ax = 0.0, ay = 0.0, az = 0.0;
#pragma unroll 2
  for (int f = 0; f < nup; ++f) {
    const double4 o = offup[f];
    const double rx = Xx - o.x, ry = Xy - o.y, rz = Xz - o.z;
    const double r2 = fma(rx, rx, fma(ry, ry, rz * rz));
    const double ri = rsqrt(r2);
    const double ri2 = ri * ri;
    const double dqx = qx[f] - fx, dqy = qx[MU + f] - fy, dqz = qx[2 * MU + f] - fz;
    const double rn = fma(rx, o.x, fma(ry, o.y, rz * o.z));
    const double rq = o.w * fma(rx, dqx, fma(ry, dqy, rz * dqz));
    const double c = rn * rq * ri * ri2 * ri2;
    ax = fma(c, rx, ax);
    ay = fma(c, ry, ay);
    az = fma(c, rz, az);
  }
  if (valid) {
    double* pb = near_part + (size_t)slot * 3 * N;
    pb[t] = scale * ax;
    pb[N + t] = scale * ay;
    pb[2 * N + t] = scale * az;
  }
}

// ------------------------------------------------------------------ GEMM
//
// C(r, col) = sum_k A[r * lda + k] * B(k, col), FP64, 64x64 tiles, BK = 16.
// B(k, col) = B[z * Bz + (k / kb) * kbs + col * ldb + k % kb] and
// C(r, col) is stored at C[z * Cz + (r / rb) * rbs + col * ldc + r % rb]: one
// kernel covers the per-sphere block products on the SoA field layout.

constexpr int GBM = 32, GBN = 32, GBK = 16;

// One wave per 32x32 output tile, 4x4 outputs per lane (rows ty+8e, cols tx+8f).
__global__ __launch_bounds__(64) void k_gemm64(int R, int Cn, int K, const double* __restrict__ A, int lda, long Az,
                                               const double* __restrict__ B, long Bz, int kb, long kbs, int ldb,
                                               double* __restrict__ C, long Cz, int rb, long rbs, int ldc) {
  __shared__ double As[GBK][GBM + 1];
  __shared__ double Bs[GBK][GBN + 1];
  const int tid = threadIdx.x;
  const int tx = tid % 8, ty = tid / 8;
  const int r0 = blockIdx.x * GBM, c0 = blockIdx.y * GBN;
  A += (size_t)blockIdx.z * Az;
  B += (size_t)blockIdx.z * Bz;
  C += (size_t)blockIdx.z * Cz;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += GBK) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = tid + e * 64;         // 0..511
      const int ar = idx / GBK, ak = idx % GBK;
      const int gr = r0 + ar, gk = k0 + ak;
      As[ak][ar] = (gr < R && gk < K) ? A[(size_t)gr * lda + gk] : 0.0;
      const int bk = idx / GBN, bc = idx % GBN;
      const int gk2 = k0 + bk, gc = c0 + bc;
      Bs[bk][bc] = (gk2 < K && gc < Cn) ? B[(size_t)(gk2 / kb) * kbs + (size_t)gc * ldb + gk2 % kb] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GBK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        a[e] = As[kk][ty + 8 * e];
        b[e] = Bs[kk][tx + 8 * e];
      }
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int f = 0; f < 4; ++f) acc[e][f] = fma(a[e], b[f], acc[e][f]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int gr = r0 + ty + 8 * e;
    if (gr >= R) continue;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const int gc = c0 + tx + 8 * f;
      if (gc < Cn) C[(size_t)(gr / rb) * rbs + (size_t)gc * ldc + gr % rb] = acc[e][f];
    }
  }
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
__global__ __launch_bounds__(256) void k_moments(const double* __restrict__ q, const double* __restrict__ off,
                                                 const double* __restrict__ w, int n, int N,
                                                 double* __restrict__ mom) {
  const int j = blockIdx.x;
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

// y = q/2 + sum(self partials) + sum(far partials) + sum(near partials) + P[q].
__global__ __launch_bounds__(256) void k_combine(const double* __restrict__ q, const double* __restrict__ selfo,
                                                 int nself, const double* __restrict__ far_part, int nchunks,
                                                 const double* __restrict__ near_part, const int* __restrict__ npart,
                                                 const double* __restrict__ mom, const double* __restrict__ off,
                                                 int n, int N, double a, double* __restrict__ y) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= N) return;
  const int i = t / n, k = t - i * n;
  const double s1 = 1.0 / (4.0 * kPi * a * a), s2 = 3.0 / (8.0 * kPi * a * a * a * a);
  const double* mj = mom + 6 * i;
  const double ox = off[3 * k], oy = off[3 * k + 1], oz = off[3 * k + 2];
  const double P[3] = {s1 * mj[0] + s2 * (mj[4] * oz - mj[5] * oy), s1 * mj[1] + s2 * (mj[5] * ox - mj[3] * oz),
                       s1 * mj[2] + s2 * (mj[3] * oy - mj[4] * ox)};
  const int np = npart[i];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const size_t e = (size_t)c * N + t;
    double v = 0.5 * q[e] + P[c];
    for (int h = 0; h < nself; ++h) v += selfo[(size_t)h * 3 * N + e];
    for (int h = 0; h < nchunks; ++h) v += far_part[(size_t)h * 3 * N + e];
    for (int h = 0; h < np; ++h) v += near_part[(size_t)h * 3 * N + e];
    y[e] = v;
  }
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

// ------------------------------------------------------------- launchers

static inline unsigned nblk(long n, int b = 256) { return (unsigned)((n + b - 1) / b); }

void launch_pack32(hipStream_t s, const double* q, const double* off, const double* w, int n, int N, float4* src) {
  hipLaunchKernelGGL(k_pack32, dim3(nblk(N)), dim3(256), 0, s, q, off, w, n, N, src);
}
void launch_pack64(hipStream_t s, const double* q, const double* off, const double* w, int n, int N, double2* src) {
  hipLaunchKernelGGL(k_pack64, dim3(nblk(N)), dim3(256), 0, s, q, off, w, n, N, src);
}
void launch_far32(hipStream_t s, int tpt, const float4* src, const double* off, const double* ctr,
                  const unsigned char* cls, int n, int M, int N, int spc, int nchunks, double scale, double* part) {
  if (tpt == 2)
    hipLaunchKernelGGL(k_far32<2>, dim3(nblk(N, 512), nchunks), dim3(256), 0, s, src, off, ctr, cls, n, M, N, spc,
                       scale, part);
  else
    hipLaunchKernelGGL(k_far32<1>, dim3(nblk(N, 256), nchunks), dim3(256), 0, s, src, off, ctr, cls, n, M, N, spc,
                       scale, part);
}
void launch_far64(hipStream_t s, const double2* src, const double* off, const double* ctr, const unsigned char* cls,
                  int n, int M, int N, int spc, int nchunks, double scale, double* part) {
  hipLaunchKernelGGL(k_far64, dim3(nblk(N), nchunks), dim3(256), 0, s, src, off, ctr, cls, n, M, N, spc, scale,
                     part);
}
void launch_near64(hipStream_t s, int max_slots, const double* ctr, const double* off, const double4* offup,
                   const double* qup, const double* coef, const int* partners, const int* npart, int n, int M, int N,
                   int nup, int p, int L, double scale, double* near_part) {
  if (max_slots <= 0) return;
  hipLaunchKernelGGL(k_near64, dim3(nblk(N), max_slots), dim3(256), 0, s, ctr, off, offup, qup, coef, partners,
                     npart, n, M, N, nup, p, L, scale, near_part);
}
void launch_gemm64(hipStream_t s, int R, int Cn, int K, const double* A, int lda, long Az, const double* B, long Bz,
                   int kb, long kbs, int ldb, double* C, long Cz, int rb, long rbs, int ldc, int batch) {
  hipLaunchKernelGGL(k_gemm64, dim3((R + GBM - 1) / GBM, (Cn + GBN - 1) / GBN, batch), dim3(64), 0, s, R, Cn, K, A,
                     lda, Az, B, Bz, kb, kbs, ldb, C, Cz, rb, rbs, ldc);
}
void launch_near64p(hipStream_t s, int npairs_count, const double* ctr, const double* off, const double4* offup,
                    const double* qup, const double* coef, const int* npairs, int n, int M, int N, int nup, int p,
                    int L, double scale, double* near_part) {
  if (npairs_count <= 0) return;
  hipLaunchKernelGGL(k_near64p, dim3(npairs_count, (n + 63) / 64), dim3(64), 0, s, ctr, off, offup, qup, coef,
                     npairs, n, M, N, nup, p, L, scale, near_part);
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
  hipLaunchKernelGGL(k_combine, dim3(nblk(N)), dim3(256), 0, s, q, selfo, nself, far_part, nchunks, near_part, npart,
                     mom, off, n, N, a, y);
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
