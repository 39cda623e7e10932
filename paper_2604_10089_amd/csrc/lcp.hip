// LCP layer on the device: contacts, A = D^T M D products, and the PQN solvers.
//
// The quasi-Newton iterations run in single-workgroup kernels (n contacts and
// r memory pairs are small: ~10^2 and <= 32); the host only sequences them
// around the mobility solves and reads a few flags per iteration.
#include "lcp.hpp"

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

namespace bipqn {

constexpr int kT = 256;  // threads of the single-workgroup kernels (4 waves)

// sigma: scale of the initial metric B0 = sigma I (0 = not yet set; the first
// step then uses H0 = I and sets sigma = p.Ap/p.p from its own product).
struct PqnScal {
  int r, conv, stationary, reset, ssn_steps, ssn_fail, have_prev, nonzero;
  int resets;  // steps of this solve that met the Alg. 2 edge cases (non-positive curvature or no descent)
  int nonpos;  // of those, steps with p.Ap <= 0: the operator is not positive definite along p
  int bad;     // k_check_lcp_inputs: an invalid pair or a non-finite entry of b or x
  double e, e_prev, eta, tol_abs, tol_rel, tau, sigma;
};

// One PQN engine's device workspace (vectors of length n, memory [kRmax][n]).
struct PqnDev {
  int n;
  double *b, *x, *Ax, *g, *p, *Ap, *xt, *xh, *w, *t1, *t2;
  double *U, *V, *S, *Y, *rho, *CiV;
  PqnScal* sc;
};

// Bi-PQN outer state: high-fidelity corrections (Uc, Vc) of B^(k) = A^ + Uc Uc^T - Vc Vc^T,
// the transferred low-fidelity secant pairs and A^ x.
struct BiDev {
  int n;
  double *Uc, *Vc, *Slow, *Ylow, *Alox, *Alos, *Bs, *tmp;
  int* cnt;  // [0] = rc (corrections), [1] = number of low pairs
};

// --------------------------------------------------------- block helpers

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

__device__ inline double block_min(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  return fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
}

__device__ inline double bdot(const double* a, const double* b, int n, double* red) {
  double s = 0.0;
  for (int e = threadIdx.x; e < n; e += kT) s = fma(a[e], b[e], s);
  return block_sum(s, red);
}

// Solve A X = B in place (A m x m, B m x nr, row-major, shared memory) by
// Gaussian elimination with partial pivoting; returns false if singular.
__device__ bool block_solve(double* A, int lda, double* B, int ldb, int m, int nr, double* fac, int* flag) {
  for (int k = 0; k < m; ++k) {
    if (threadIdx.x == 0) {
      int piv = k;
      double best = fabs(A[k * lda + k]);
      for (int i = k + 1; i < m; ++i)
        if (fabs(A[i * lda + k]) > best) {
          best = fabs(A[i * lda + k]);
          piv = i;
        }
      *flag = best > 0.0 ? 1 : 0;
      if (piv != k) {
        for (int j = 0; j < m; ++j) {
          double t = A[k * lda + j];
          A[k * lda + j] = A[piv * lda + j];
          A[piv * lda + j] = t;
        }
        for (int j = 0; j < nr; ++j) {
          double t = B[k * ldb + j];
          B[k * ldb + j] = B[piv * ldb + j];
          B[piv * ldb + j] = t;
        }
      }
    }
    __syncthreads();
    if (!*flag) return false;
    const double pv = A[k * lda + k];
    for (int i = k + 1 + threadIdx.x; i < m; i += kT) fac[i] = A[i * lda + k] / pv;
    __syncthreads();
    const int wA = m - k, wtot = wA + nr;
    for (int idx = threadIdx.x; idx < (m - k - 1) * wtot; idx += kT) {
      const int i = k + 1 + idx / wtot, c = idx % wtot;
      if (c < wA)
        A[i * lda + k + c] -= fac[i] * A[k * lda + k + c];
      else
        B[i * ldb + (c - wA)] -= fac[i] * B[k * ldb + (c - wA)];
    }
    __syncthreads();
  }
  for (int c = threadIdx.x; c < nr; c += kT)
    for (int k = m - 1; k >= 0; --k) {
      double v = B[k * ldb + c];
      for (int j = k + 1; j < m; ++j) v -= A[k * lda + j] * B[j * ldb + c];
      B[k * ldb + c] = v / A[k * lda + k];
    }
  __syncthreads();
  return true;
}

// BFGS append of the pair (s, y) to B = sigma I + U U^T - V V^T (or to a given B s):
// u = y/sqrt(y.s), v = B s/sqrt(s.B s); skipped when y.s <= 1e-12 |s||y| or s.B s <= 0.
// bs_given != nullptr supplies B s (Bi-PQN corrections); otherwise B s = sigma s + U(U^T s) - V(V^T s).
// When the memory is full it restarts from the identity.
__device__ void bfgs_append(int n, double* U, double* V, double* S, double* Y, double* rho, int* r_io,
                            const double* s, const double* y, const double* bs_given, double* bs_buf, double* red,
                            double* coefs, double sigma) {
  int r = *r_io;
  const double ys = bdot(y, s, n, red), ss = bdot(s, s, n, red), yy = bdot(y, y, n, red);
  if (!(ys > 1e-12 * sqrt(ss) * sqrt(yy))) return;
  if (r >= kRmax) r = 0;
  const double* bs = bs_given;
  if (!bs) {
    for (int a = 0; a < 2 * r; ++a) {
      const double* vec = a < r ? U + (size_t)a * n : V + (size_t)(a - r) * n;
      double d = bdot(vec, s, n, red);
      if (threadIdx.x == 0) coefs[a] = d;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n; e += kT) {
      double v = sigma * s[e];
      for (int a = 0; a < r; ++a) v = fma(U[(size_t)a * n + e], coefs[a], v);
      for (int a = 0; a < r; ++a) v = fma(-V[(size_t)a * n + e], coefs[r + a], v);
      bs_buf[e] = v;
    }
    __syncthreads();
    bs = bs_buf;
  }
  const double sbs = bdot(s, bs, n, red);
  if (!(sbs > 0.0)) {
    *r_io = r;
    return;
  }
  const double iu = 1.0 / sqrt(ys), iv = 1.0 / sqrt(sbs);
  for (int e = threadIdx.x; e < n; e += kT) {
    U[(size_t)r * n + e] = y[e] * iu;
    V[(size_t)r * n + e] = bs[e] * iv;
    if (S) S[(size_t)r * n + e] = s[e];
    if (Y) Y[(size_t)r * n + e] = y[e];
  }
  if (threadIdx.x == 0 && rho) rho[r] = 1.0 / ys;
  __syncthreads();
  *r_io = r + 1;
}

// ------------------------------------------------------------ contacts

// Pairs i < j with |c_i - c_j| - 2a <= delta, lexicographic. One workgroup:
// rows are taken 256 at a time, counted, scanned, then written.
__global__ __launch_bounds__(kT) void k_contacts(const double* __restrict__ ctr, int M, double a, double delta,
                                                 int cap, int* __restrict__ pairs, double* __restrict__ gaps,
                                                 int* __restrict__ count) {
  __shared__ int cnt[kT];
  int base = 0;
  for (int r0 = 0; r0 < M; r0 += kT) {
    const int i = r0 + threadIdx.x;
    int c = 0;
    if (i < M)
      for (int j = i + 1; j < M; ++j) {
        const double dx = ctr[3 * i] - ctr[3 * j], dy = ctr[3 * i + 1] - ctr[3 * j + 1],
                     dz = ctr[3 * i + 2] - ctr[3 * j + 2];
        if (sqrt(dx * dx + dy * dy + dz * dz) - 2.0 * a <= delta) ++c;
      }
    cnt[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
      int run = 0;
      for (int t = 0; t < kT; ++t) {
        const int v = cnt[t];
        cnt[t] = run;
        run += v;
      }
    }
    __syncthreads();
    int o = base + cnt[threadIdx.x];
    if (i < M)
      for (int j = i + 1; j < M; ++j) {
        const double dx = ctr[3 * i] - ctr[3 * j], dy = ctr[3 * i + 1] - ctr[3 * j + 1],
                     dz = ctr[3 * i + 2] - ctr[3 * j + 2];
        const double gp = sqrt(dx * dx + dy * dy + dz * dz) - 2.0 * a;
        if (gp <= delta) {
          if (o < cap) {
            pairs[2 * o] = i;
            pairs[2 * o + 1] = j;
            gaps[o] = gp;
          }
          ++o;
        }
      }
    __syncthreads();
    if (threadIdx.x == kT - 1) cnt[0] = o;  // last thread holds the running end
    __syncthreads();
    base = cnt[0];
    __syncthreads();
  }
  if (threadIdx.x == 0) *count = base;
}

// --------------------------------------------- contacts without allocation
//
// pqn_find_contacts_noalloc stages the contact kernel's count and list in this
// file-scope device array instead of buffers of the context (one copy per device,
// held until the process ends). Layout: the count at byte 0; gaps (double) from
// byte 256; pairs (two int) after the gaps. Host code never passes the array's name
// to a kernel or a copy: it uses the per-device address resolved at set-up.
constexpr int kNoAllocContacts = 32768;
constexpr size_t kScratchGaps = 256;
constexpr size_t kScratchPairs = kScratchGaps + sizeof(double) * kNoAllocContacts;
constexpr size_t kScratchBytes = kScratchPairs + 2 * sizeof(int) * kNoAllocContacts;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Resolve the array's address on `device` (current on the calling thread), once.
void contact_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) throw Error(PQN_ERR_DEVICE, "device ordinal beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* p = nullptr;
  HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw Error(PQN_ERR_DEVICE, "hipGetSymbolAddress returned a null address for the contact staging");
  g_scratch_ptr[device] = p;
}

pqn_status lcp_find_contacts_noalloc(pqn_ctx_impl& ctx, double delta, int cap, int* n_out, int* pairs,
                                     double* gaps) {
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (ctx.device >= 0 && ctx.device < kMaxDevices) base = g_scratch_ptr[ctx.device];
  }
  if (!base) throw Error(PQN_ERR_STATE, "contact staging not set up on this device");
  unsigned char* b = static_cast<unsigned char*>(base);
  int* count = reinterpret_cast<int*>(b);
  double* sgaps = reinterpret_cast<double*>(b + kScratchGaps);
  int* spairs = reinterpret_cast<int*>(b + kScratchPairs);
  // the kernel writes the count unconditionally and at most kNoAllocContacts entries
  hipLaunchKernelGGL(k_contacts, dim3(1), dim3(kT), 0, ctx.stream, ctx.ctr.p, ctx.M, ctx.a, delta, kNoAllocContacts,
                     spairs, sgaps, count);
  HIPCHK(hipGetLastError());
  int n = 0;
  HIPCHK(hipMemcpyAsync(&n, count, sizeof(int), hipMemcpyDeviceToHost, ctx.stream));
  HIPCHK(hipStreamSynchronize(ctx.stream));
  *n_out = n;
  if (n > kNoAllocContacts)
    throw Error(PQN_ERR_INVALID, "pqn_find_contacts_noalloc: " + std::to_string(n) +
                                     " contacts, more than its staging holds (32768)");
  if (n > cap) throw Error(PQN_ERR_INVALID, "pqn_find_contacts_noalloc: cap too small");
  if (n > 0) {
    HIPCHK(hipMemcpyAsync(pairs, spairs, 2 * (size_t)n * sizeof(int), hipMemcpyDeviceToHost, ctx.stream));
    HIPCHK(hipMemcpyAsync(gaps, sgaps, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
    HIPCHK(hipStreamSynchronize(ctx.stream));
  }
  return PQN_OK;
}

// FT = D x: force -x_l n_l on i, +x_l n_l on j (n_l = unit c_j - c_i), no torque.
__global__ __launch_bounds__(kT) void k_D_scatter(const double* __restrict__ ctr, const int* __restrict__ pairs,
                                                  const double* __restrict__ x, int n, int M,
                                                  double* __restrict__ FT) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= M) return;
  double f[3] = {0.0, 0.0, 0.0};
  for (int l = 0; l < n; ++l) {
    const int pi = pairs[2 * l], pj = pairs[2 * l + 1];
    if (pi != i && pj != i) continue;
    const double dx = ctr[3 * pj] - ctr[3 * pi], dy = ctr[3 * pj + 1] - ctr[3 * pi + 1],
                 dz = ctr[3 * pj + 2] - ctr[3 * pi + 2];
    const double inv = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
    const double sg = (pj == i) ? x[l] : -x[l];
    f[0] += sg * dx * inv;
    f[1] += sg * dy * inv;
    f[2] += sg * dz * inv;
  }
  FT[6 * i] = f[0];
  FT[6 * i + 1] = f[1];
  FT[6 * i + 2] = f[2];
  FT[6 * i + 3] = FT[6 * i + 4] = FT[6 * i + 5] = 0.0;
}

// out_l = n_l . (U_j - U_i)
__global__ __launch_bounds__(kT) void k_DT_gather(const double* __restrict__ ctr, const int* __restrict__ pairs,
                                                  const double* __restrict__ UO, int n, double* __restrict__ out) {
  const int l = blockIdx.x * kT + threadIdx.x;
  if (l >= n) return;
  const int pi = pairs[2 * l], pj = pairs[2 * l + 1];
  const double dx = ctr[3 * pj] - ctr[3 * pi], dy = ctr[3 * pj + 1] - ctr[3 * pi + 1],
               dz = ctr[3 * pj + 2] - ctr[3 * pi + 2];
  const double inv = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
  out[l] = inv * (dx * (UO[6 * pj] - UO[6 * pi]) + dy * (UO[6 * pj + 1] - UO[6 * pi + 1]) +
                  dz * (UO[6 * pj + 2] - UO[6 * pi + 2]));
}

// ------------------------------------------------------------ PQN engine

// Reset an engine: memory cleared; x, Ax either zero or kept (warm start);
// sigma0 = initial metric scale (0 = set by the first step).
__global__ __launch_bounds__(kT) void k_pqn_init(PqnDev d, int keep_x, double tol_abs, double tol_rel,
                                                 double sigma0) {
  for (int e = threadIdx.x; e < d.n; e += kT)
    if (!keep_x) d.x[e] = d.Ax[e] = 0.0;
  if (threadIdx.x == 0) {
    PqnScal z{};
    z.tol_abs = tol_abs;
    z.tol_rel = tol_rel;
    z.sigma = sigma0;
    *d.sc = z;
  }
}

// Replay secant pairs (columns of Sw, Yw) into the engine's memory (warm start).
__global__ __launch_bounds__(kT) void k_pqn_replay(PqnDev d, const double* __restrict__ Sw,
                                                   const double* __restrict__ Yw, int npairs) {
  __shared__ double red[4];
  __shared__ double coefs[2 * kRmax];
  __shared__ int r;
  if (threadIdx.x == 0) r = d.sc->r;
  __syncthreads();
  const int first = npairs > kRmax ? npairs - kRmax : 0;
  for (int k = first; k < npairs; ++k) {
    int rr = r;
    bfgs_append(d.n, d.U, d.V, d.S, d.Y, d.rho, &rr, Sw + (size_t)k * d.n, Yw + (size_t)k * d.n, nullptr, d.t1,
                red, coefs, d.sc->sigma > 0.0 ? d.sc->sigma : 1.0);
    __syncthreads();
    if (threadIdx.x == 0) r = rr;
    __syncthreads();
  }
  if (threadIdx.x == 0) d.sc->r = r;
}

// KKT check, x~ = x - H g (two-loop recursion, H0 = I), prox by semi-smooth
// Newton (Prop. 1, Alg. 3), p = x^ - x.
__global__ __launch_bounds__(kT) void k_pqn_prepare(PqnDev d, int jmax, double ssn_tol) {
  __shared__ double red[4];
  __shared__ double Jm[2 * kRmax * 2 * kRmax];
  __shared__ double Lv[2 * kRmax];
  __shared__ double Gm[kRmax * kRmax];
  __shared__ double Xm[kRmax * kRmax];
  __shared__ double z[2 * kRmax];
  __shared__ double fac[2 * kRmax];
  __shared__ double alpha[kRmax];
  __shared__ int flag, stop, conv;
  const int n = d.n;
  const int r = d.sc->r;
  // 1. gradient and KKT error (eq. (kkt-error))
  double s = 0.0;
  for (int e = threadIdx.x; e < n; e += kT) {
    const double g = d.Ax[e] + d.b[e];
    d.g[e] = g;
    const double m = fmin(d.x[e], g);
    s = fma(m, m, s);
  }
  const double err = sqrt(block_sum(s, red));
  if (threadIdx.x == 0) {
    PqnScal* sc = d.sc;
    const double mx = fmax(err, sc->e_prev);
    int c = err < sc->tol_abs;
    if (!c && sc->have_prev && mx > 0.0 && fabs(err - sc->e_prev) / mx < sc->tol_rel) c = 1;
    sc->e = err;
    if (!c) {
      sc->e_prev = err;
      sc->have_prev = 1;
    }
    sc->conv = c;
    sc->stationary = 0;
    conv = c;
  }
  __syncthreads();
  if (conv) return;
  // 2. two-loop recursion: t1 = H g
  for (int e = threadIdx.x; e < n; e += kT) d.t1[e] = d.g[e];
  __syncthreads();
  for (int i = r - 1; i >= 0; --i) {
    const double al = d.rho[i] * bdot(d.S + (size_t)i * n, d.t1, n, red);
    if (threadIdx.x == 0) alpha[i] = al;
    for (int e = threadIdx.x; e < n; e += kT) d.t1[e] = fma(-al, d.Y[(size_t)i * n + e], d.t1[e]);
    __syncthreads();
  }
  const double sigma = d.sc->sigma > 0.0 ? d.sc->sigma : 1.0;
  const double isig = 1.0 / sigma;
  for (int e = threadIdx.x; e < n; e += kT) d.t1[e] *= isig;   // H0 = I / sigma
  __syncthreads();
  for (int i = 0; i < r; ++i) {
    const double be = d.rho[i] * bdot(d.Y + (size_t)i * n, d.t1, n, red);
    __syncthreads();
    const double cf = alpha[i] - be;
    for (int e = threadIdx.x; e < n; e += kT) d.t1[e] = fma(cf, d.S[(size_t)i * n + e], d.t1[e]);
    __syncthreads();
  }
  for (int e = threadIdx.x; e < n; e += kT) d.xt[e] = d.x[e] - d.t1[e];
  __syncthreads();
  // 3. weighted prox (D = sigma I): x^ = (x~ + C^{-1} V a~ - U a / sigma)_+, C = sigma I + U U^T
  if (r == 0) {
    for (int e = threadIdx.x; e < n; e += kT) d.xh[e] = fmax(d.xt[e], 0.0);
  } else {
    // Gm = sigma I + U^T U, Xm = U^T V; Xm <- Gm^{-1} Xm; CiV = (V - U Xm)/sigma (Woodbury)
    for (int ent = threadIdx.x; ent < 2 * r * r; ent += kT) {
      const int which = ent / (r * r), ab = ent % (r * r), a = ab / r, b = ab % r;
      const double* u = d.U + (size_t)a * n;
      const double* v = which == 0 ? d.U + (size_t)b * n : d.V + (size_t)b * n;
      double t = 0.0;
      for (int e = 0; e < n; ++e) t = fma(u[e], v[e], t);
      if (which == 0)
        Gm[a * r + b] = t + (a == b ? sigma : 0.0);
      else
        Xm[a * r + b] = t;
    }
    __syncthreads();
    block_solve(Gm, r, Xm, r, r, r, fac, &flag);
    for (int e = threadIdx.x; e < n; e += kT)
      for (int c = 0; c < r; ++c) {
        double v = d.V[(size_t)c * n + e];
        for (int a = 0; a < r; ++a) v = fma(-d.U[(size_t)a * n + e], Xm[a * r + c], v);
        d.CiV[(size_t)c * n + e] = v * isig;
      }
    for (int k = threadIdx.x; k < 2 * r; k += kT) z[k] = 0.0;
    __syncthreads();
    const int m2 = 2 * r;
    int steps = 0;
    for (int j = 0; j < jmax; ++j) {
      ++steps;
      // w = x~ + CiV a~ - U a / sigma; t2 = x~ + CiV a~; x^ = w_+; Lambda = [w > 0]
      for (int e = threadIdx.x; e < n; e += kT) {
        double t2 = d.xt[e];
        for (int c = 0; c < r; ++c) t2 = fma(d.CiV[(size_t)c * n + e], z[r + c], t2);
        double ua = 0.0;
        for (int a = 0; a < r; ++a) ua = fma(d.U[(size_t)a * n + e], z[a], ua);
        const double w = t2 - ua * isig;
        d.t2[e] = t2;
        d.w[e] = w;
        d.xh[e] = fmax(w, 0.0);
      }
      __syncthreads();
      // L~ = [a + U^T (t2 - x^); a~ + V^T (x~ - x^)] and its Jacobian (printed J_L)
      for (int ent = threadIdx.x; ent < m2 * m2 + m2; ent += kT) {
        if (ent < m2) {
          const bool top = ent < r;
          const double* u = top ? d.U + (size_t)ent * n : d.V + (size_t)(ent - r) * n;
          double t = 0.0;
          for (int e = 0; e < n; ++e) t = fma(u[e], (top ? d.t2[e] : d.xt[e]) - d.xh[e], t);
          Lv[ent] = z[ent] + t;
        } else {
          const int q = ent - m2, row = q / m2, col = q % m2;
          const bool rtop = row < r, ctop = col < r;
          const double* u = rtop ? d.U + (size_t)row * n : d.V + (size_t)(row - r) * n;
          const double* v = ctop ? d.U + (size_t)col * n : d.CiV + (size_t)(col - r) * n;
          double t = 0.0;
          if (rtop && !ctop) {
            for (int e = 0; e < n; ++e) t = fma(u[e] * (d.w[e] > 0.0 ? 0.0 : 1.0), v[e], t);
          } else {
            for (int e = 0; e < n; ++e) t = fma(u[e] * (d.w[e] > 0.0 ? 1.0 : 0.0), v[e], t);
          }
          if (ctop) t *= isig;      // columns D^{-1} U
          if (!rtop && !ctop) t = -t;
          Jm[row * m2 + col] = t + (row == col ? 1.0 : 0.0);
        }
      }
      __syncthreads();
      const bool ok = block_solve(Jm, m2, Lv, 1, m2, 1, fac, &flag);
      if (threadIdx.x == 0) {
        double dn = 0.0, zn = 0.0;
        if (ok)
          for (int k = 0; k < m2; ++k) {
            z[k] -= Lv[k];
            dn += Lv[k] * Lv[k];
            zn += z[k] * z[k];
          }
        stop = !ok || sqrt(dn) <= ssn_tol * fmax(1.0, sqrt(zn));
        if (!ok) d.sc->ssn_fail += 1;
      }
      __syncthreads();
      if (stop) break;
    }
    for (int e = threadIdx.x; e < n; e += kT) {
      double w = d.xt[e];
      for (int c = 0; c < r; ++c) w = fma(d.CiV[(size_t)c * n + e], z[r + c], w);
      double ua = 0.0;
      for (int a = 0; a < r; ++a) ua = fma(d.U[(size_t)a * n + e], z[a], ua);
      d.xh[e] = fmax(w - ua * isig, 0.0);
    }
    if (threadIdx.x == 0) d.sc->ssn_steps += steps;
  }
  __syncthreads();
  // 4. search direction
  double nz = 0.0;
  for (int e = threadIdx.x; e < n; e += kT) {
    const double pe = d.xh[e] - d.x[e];
    d.p[e] = pe;
    nz += pe != 0.0 ? 1.0 : 0.0;
  }
  nz = block_sum(nz, red);
  if (threadIdx.x == 0) d.sc->stationary = nz == 0.0;
}

// Optimal over-relaxation (Alg. 2) and the updates x += eta p, A x += eta A p,
// then the BFGS update with s = eta p, y = eta A p.
__device__ double step_size_block(const double* g, const double* x, const double* p, const double* Ap, int n,
                                  double* red, int* reset) {
  const double pAp = bdot(p, Ap, n, red);
  const double gp = bdot(p, g, n, red);
  double lim = INFINITY;
  for (int e = threadIdx.x; e < n; e += kT)
    if (p[e] < 0.0) lim = fmin(lim, -x[e] / p[e]);
  lim = block_min(lim, red);
  if (!(pAp > 0.0)) {
    *reset = 2;
    return 1.0;
  }
  const double eta1 = -gp / pAp;
  if (!(eta1 > 0.0)) {
    *reset = 1;
    return 1.0;
  }
  *reset = 0;
  return fmin(eta1, lim);
}

__global__ __launch_bounds__(kT) void k_pqn_accept(PqnDev d) {
  __shared__ double red[4];
  __shared__ double coefs[2 * kRmax];
  const int n = d.n;
  int reset = 0;
  double sigma = d.sc->sigma;
  if (!(sigma > 0.0)) {
    // first step: the metric scale is the curvature of this step's own product
    const double pAp = bdot(d.p, d.Ap, n, red), pp = bdot(d.p, d.p, n, red);
    sigma = pAp > 0.0 ? pAp / pp : 1.0;
  }
  const double eta = step_size_block(d.g, d.x, d.p, d.Ap, n, red, &reset);
  for (int e = threadIdx.x; e < n; e += kT) {
    d.x[e] = fmax(fma(eta, d.p[e], d.x[e]), 0.0);
    d.Ax[e] = fma(eta, d.Ap[e], d.Ax[e]);
    d.xt[e] = eta * d.p[e];   // s
    d.xh[e] = eta * d.Ap[e];  // y
  }
  __syncthreads();
  int r = reset ? 0 : d.sc->r;
  bfgs_append(n, d.U, d.V, d.S, d.Y, d.rho, &r, d.xt, d.xh, nullptr, d.t1, red, coefs, sigma);
  if (threadIdx.x == 0) {
    d.sc->sigma = sigma;
    d.sc->r = r;
    d.sc->eta = eta;
    d.sc->reset = reset;
    d.sc->resets += reset != 0;
    d.sc->nonpos += reset == 2;
  }
}

// BB-PGD (eq. (spectralStepSize), eta = 1): KKT check, tau_bb, x+ = (x - tau g)_+.
// t1/t2 keep the previous x and A x; the product of the new x is the next A x.
__global__ __launch_bounds__(kT) void k_bb_prepare(PqnDev d, double tau0) {
  __shared__ double red[4];
  __shared__ int conv;
  const int n = d.n;
  double s = 0.0;
  for (int e = threadIdx.x; e < n; e += kT) {
    const double g = d.Ax[e] + d.b[e];
    d.g[e] = g;
    const double m = fmin(d.x[e], g);
    s = fma(m, m, s);
  }
  const double err = sqrt(block_sum(s, red));
  if (threadIdx.x == 0) {
    PqnScal* sc = d.sc;
    const double mx = fmax(err, sc->e_prev);
    int c = err < sc->tol_abs;
    if (!c && sc->have_prev && mx > 0.0 && fabs(err - sc->e_prev) / mx < sc->tol_rel) c = 1;
    sc->e = err;
    sc->conv = c;
    conv = c;
  }
  __syncthreads();
  if (conv) return;
  double tau = d.sc->have_prev ? d.sc->tau : tau0;
  if (d.sc->have_prev) {
    double dxdx = 0.0, dxdg = 0.0;
    for (int e = threadIdx.x; e < n; e += kT) {
      const double dx = d.x[e] - d.t1[e], dg = d.Ax[e] - d.t2[e];
      dxdx = fma(dx, dx, dxdx);
      dxdg = fma(dx, dg, dxdg);
    }
    dxdx = block_sum(dxdx, red);
    dxdg = block_sum(dxdg, red);
    if (dxdg > 0.0) tau = dxdx / dxdg;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n; e += kT) {
    d.t1[e] = d.x[e];
    d.t2[e] = d.Ax[e];
    d.x[e] = fmax(d.x[e] - tau * d.g[e], 0.0);
  }
  if (threadIdx.x == 0) {
    d.sc->tau = tau;
    d.sc->e_prev = err;
    d.sc->have_prev = 1;
  }
}

// Low-rank correction: out = base + Uc (Uc^T v) - Vc (Vc^T v).
__global__ __launch_bounds__(kT) void k_lowrank(BiDev B, const double* __restrict__ base,
                                                const double* __restrict__ v, double* __restrict__ out) {
  __shared__ double red[4];
  __shared__ double cf[2 * kRmax];
  const int n = B.n, rc = B.cnt[0];
  for (int a = 0; a < 2 * rc; ++a) {
    const double* u = a < rc ? B.Uc + (size_t)a * n : B.Vc + (size_t)(a - rc) * n;
    const double t = bdot(u, v, n, red);
    if (threadIdx.x == 0) cf[a] = t;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n; e += kT) {
    double o = base ? base[e] : 0.0;
    for (int a = 0; a < rc; ++a) o = fma(B.Uc[(size_t)a * n + e], cf[a], o);
    for (int a = 0; a < rc; ++a) o = fma(-B.Vc[(size_t)a * n + e], cf[rc + a], o);
    out[e] = o;
  }
}

// Bi-PQN outer step, first half: gradient, KKT check, subproblem data
// c = A x + b - B x with B x = A^ x + corrections (eq. (pqnSubproblem)).
// Writes the inner engine's b (= c), x and A x (= B x).
__global__ __launch_bounds__(kT) void k_bi_prepare(PqnDev o, BiDev B, PqnDev in) {
  __shared__ double red[4];
  __shared__ double cf[2 * kRmax];
  __shared__ int conv;
  const int n = o.n, rc = B.cnt[0];
  double s = 0.0;
  for (int e = threadIdx.x; e < n; e += kT) {
    const double g = o.Ax[e] + o.b[e];
    o.g[e] = g;
    const double m = fmin(o.x[e], g);
    s = fma(m, m, s);
  }
  const double err = sqrt(block_sum(s, red));
  if (threadIdx.x == 0) {
    PqnScal* sc = o.sc;
    const double mx = fmax(err, sc->e_prev);
    int c = err < sc->tol_abs;
    if (!c && sc->have_prev && mx > 0.0 && fabs(err - sc->e_prev) / mx < sc->tol_rel) c = 1;
    sc->e = err;
    if (!c) {
      sc->e_prev = err;
      sc->have_prev = 1;
    }
    sc->conv = c;
    conv = c;
  }
  __syncthreads();
  if (conv) return;
  for (int a = 0; a < 2 * rc; ++a) {
    const double* u = a < rc ? B.Uc + (size_t)a * n : B.Vc + (size_t)(a - rc) * n;
    const double t = bdot(u, o.x, n, red);
    if (threadIdx.x == 0) cf[a] = t;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n; e += kT) {
    double bx = B.Alox[e];
    for (int a = 0; a < rc; ++a) bx = fma(B.Uc[(size_t)a * n + e], cf[a], bx);
    for (int a = 0; a < rc; ++a) bx = fma(-B.Vc[(size_t)a * n + e], cf[rc + a], bx);
    in.b[e] = o.g[e] - bx;
    in.x[e] = o.x[e];
    in.Ax[e] = bx;
  }
}

// p = x^ - x (inner result minus outer iterate); flags a zero step.
__global__ __launch_bounds__(kT) void k_bi_direction(PqnDev o, PqnDev in) {
  __shared__ double red[4];
  double nz = 0.0;
  for (int e = threadIdx.x; e < o.n; e += kT) {
    const double pe = in.x[e] - o.x[e];
    o.p[e] = pe;
    nz += pe != 0.0 ? 1.0 : 0.0;
  }
  nz = block_sum(nz, red);
  if (threadIdx.x == 0) o.sc->stationary = nz == 0.0;
}

// Bi-PQN outer step, second half (after the high-fidelity product A p):
// eta* (Alg. 2), A^ s = eta (A^ x^ - A^ x) (App. E.2), BFGS correction of
// B^(k) with B^(k) s = A^ s + corrections, secant transfer of the subproblem
// pairs Y <- Y^ + u (u.S^) - v (v.S^), and x, A x, A^ x updates.
__global__ __launch_bounds__(kT) void k_bi_accept(PqnDev o, BiDev B, PqnDev in) {
  __shared__ double red[4];
  __shared__ double cf[4 * kRmax];
  const int n = o.n;
  int reset = 0;
  const double eta = step_size_block(o.g, o.x, o.p, o.Ap, n, red, &reset);
  int rc = B.cnt[0];
  // A^ x^ = B x^ - corrections(x^), with B x^ the inner engine's final A x
  for (int a = 0; a < 2 * rc; ++a) {
    const double* u = a < rc ? B.Uc + (size_t)a * n : B.Vc + (size_t)(a - rc) * n;
    const double t1 = bdot(u, in.x, n, red);
    const double t2 = bdot(u, o.p, n, red);
    if (threadIdx.x == 0) {
      cf[a] = t1;
      cf[2 * kRmax + a] = eta * t2;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n; e += kT) {
    double alxh = in.Ax[e];
    double cs = 0.0;
    for (int a = 0; a < rc; ++a) {
      alxh = fma(-B.Uc[(size_t)a * n + e], cf[a], alxh);
      cs = fma(B.Uc[(size_t)a * n + e], cf[2 * kRmax + a], cs);
    }
    for (int a = 0; a < rc; ++a) {
      alxh = fma(B.Vc[(size_t)a * n + e], cf[rc + a], alxh);
      cs = fma(-B.Vc[(size_t)a * n + e], cf[2 * kRmax + rc + a], cs);
    }
    const double alos = eta * (alxh - B.Alox[e]);
    B.Alos[e] = alos;
    B.Bs[e] = reset ? alos : alos + cs;
    o.xt[e] = eta * o.p[e];   // s
    o.xh[e] = eta * o.Ap[e];  // y
  }
  __syncthreads();
  // subproblem pairs S^, Y^ (dropped after a memory reset)
  const int nlow = reset ? 0 : min(in.sc->r, kRmax);
  if (reset) rc = 0;
  int rnew = rc;
  bfgs_append(n, B.Uc, B.Vc, nullptr, nullptr, nullptr, &rnew, o.xt, o.xh, B.Bs, nullptr, red, cf, 1.0);
  const bool added = rnew == rc + 1 || (rc >= kRmax && rnew == 1);
  const double* u = added ? B.Uc + (size_t)(rnew - 1) * n : nullptr;
  const double* v = added ? B.Vc + (size_t)(rnew - 1) * n : nullptr;
  for (int k = 0; k < nlow; ++k) {
    const double* sh = in.S + (size_t)k * n;
    const double* yh = in.Y + (size_t)k * n;
    double us = 0.0, vs = 0.0;
    if (added) {
      us = bdot(u, sh, n, red);
      vs = bdot(v, sh, n, red);
    }
    for (int e = threadIdx.x; e < n; e += kT) {
      B.Slow[(size_t)k * n + e] = sh[e];
      B.Ylow[(size_t)k * n + e] = added ? yh[e] + u[e] * us - v[e] * vs : yh[e];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < n; e += kT) {
    o.x[e] = fmax(fma(eta, o.p[e], o.x[e]), 0.0);
    o.Ax[e] = fma(eta, o.Ap[e], o.Ax[e]);
    B.Alox[e] += B.Alos[e];
  }
  if (threadIdx.x == 0) {
    B.cnt[0] = rnew;
    B.cnt[1] = nlow;
    o.sc->eta = eta;
    o.sc->reset = reset;
    o.sc->resets += reset != 0;
    o.sc->nonpos += reset == 2;
  }
}

// y += eta * x with eta read from the device (recurrence of M D x for the step).
__global__ void k_axpy_dev(double* __restrict__ y, const double* __restrict__ x, const PqnScal* __restrict__ sc,
                           int len) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < len) y[e] = fma(sc->eta, x[e], y[e]);
}

// Nonzero test of a vector (Bi-PQN: whether x^(0) needs a high-fidelity product).
__global__ __launch_bounds__(kT) void k_nonzero(const double* __restrict__ x, int n, PqnScal* sc) {
  __shared__ double red[4];
  double c = 0.0;
  for (int e = threadIdx.x; e < n; e += kT) c += x[e] != 0.0 ? 1.0 : 0.0;
  c = block_sum(c, red);
  if (threadIdx.x == 0) sc->nonzero = c > 0.0;
}

// KKT error of x = 0: |min(0, b)|_2 (into sc->e).
__global__ __launch_bounds__(kT) void k_kkt_zero(const double* __restrict__ b, int n, PqnScal* sc) {
  __shared__ double red[4];
  double s = 0.0;
  for (int e = threadIdx.x; e < n; e += kT) {
    const double m = fmin(0.0, b[e]);
    s = fma(m, m, s);
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) sc->e = sqrt(s);
}

// Inputs handed over in device memory: pairs in range with i != j, b and x finite
// (else sc->bad); x projected on x >= 0 in place; sc->nonzero = x has a positive entry.
__global__ __launch_bounds__(kT) void k_check_lcp_inputs(const int* __restrict__ pairs, const double* __restrict__ b,
                                                         double* __restrict__ x, int n, int M, PqnScal* sc) {
  __shared__ double red[4];
  double bad = 0.0, nz = 0.0;
  for (int e = threadIdx.x; e < n; e += kT) {
    const int i = pairs[2 * e], j = pairs[2 * e + 1];
    if (i < 0 || j < 0 || i >= M || j >= M || i == j || !isfinite(b[e]) || !isfinite(x[e])) bad += 1.0;
    const double v = fmax(x[e], 0.0);
    x[e] = v;
    nz += v > 0.0 ? 1.0 : 0.0;
  }
  bad = block_sum(bad, red);
  nz = block_sum(nz, red);
  if (threadIdx.x == 0) {
    sc->bad = bad > 0.0;
    sc->nonzero = nz > 0.0;
  }
}

// KKT error |min(x, A x + b)|_2 (into sc->e).
__global__ __launch_bounds__(kT) void k_kkt(const double* __restrict__ x, const double* __restrict__ Ax,
                                            const double* __restrict__ b, int n, PqnScal* sc) {
  __shared__ double red[4];
  double s = 0.0;
  for (int e = threadIdx.x; e < n; e += kT) {
    const double m = fmin(x[e], Ax[e] + b[e]);
    s = fma(m, m, s);
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) sc->e = sqrt(s);
}

// Forward Euler of centres and Rodrigues rotation of the Janus axes.
__global__ void k_euler(double* __restrict__ ctr, double* __restrict__ axes, const double* __restrict__ Unc,
                        const double* __restrict__ MDx, int M, double dt, int has_axes) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  double U[6];
  for (int c = 0; c < 6; ++c) U[c] = Unc[6 * i + c] + (MDx ? MDx[6 * i + c] : 0.0);
  for (int c = 0; c < 3; ++c) ctr[3 * i + c] += dt * U[c];
  if (!has_axes) return;
  const double wn = sqrt(U[3] * U[3] + U[4] * U[4] + U[5] * U[5]);
  const double th = wn * dt;
  if (th == 0.0) return;
  const double k[3] = {U[3] / wn, U[4] / wn, U[5] / wn};
  const double e[3] = {axes[3 * i], axes[3 * i + 1], axes[3 * i + 2]};
  const double ke = k[0] * e[0] + k[1] * e[1] + k[2] * e[2];
  const double kxe[3] = {k[1] * e[2] - k[2] * e[1], k[2] * e[0] - k[0] * e[2], k[0] * e[1] - k[1] * e[0]};
  const double c = cos(th), s = sin(th);
  for (int q = 0; q < 3; ++q) axes[3 * i + q] = e[q] * c + kxe[q] * s + k[q] * ke * (1.0 - c);
}

// ------------------------------------------------------- host-side driver

struct Engine {
  DevArray<double> vec, mem;
  DevArray<PqnScal> sc;
  PqnDev d{};
  void alloc(int n) {
    vec.alloc((size_t)11 * n);
    mem.alloc((size_t)5 * kRmax * n + kRmax);
    sc.alloc(1);
    double* v = vec.p;
    d.n = n;
    d.b = v;
    d.x = v + n;
    d.Ax = v + 2 * n;
    d.g = v + 3 * n;
    d.p = v + 4 * n;
    d.Ap = v + 5 * n;
    d.xt = v + 6 * n;
    d.xh = v + 7 * n;
    d.w = v + 8 * n;
    d.t1 = v + 9 * n;
    d.t2 = v + 10 * n;
    double* m = mem.p;
    d.U = m;
    d.V = m + (size_t)kRmax * n;
    d.S = m + (size_t)2 * kRmax * n;
    d.Y = m + (size_t)3 * kRmax * n;
    d.CiV = m + (size_t)4 * kRmax * n;
    d.rho = m + (size_t)5 * kRmax * n;
    d.sc = sc.p;
  }
};

struct LcpState {
  int cap = 0;
  DevArray<int> pairs, cpairs, ccount;
  DevArray<double> cgaps;
  // engines: outer (the solve itself), mid (the middle level of recursive Bi-PQN),
  // inner (the lowest-fidelity Mono-PQN subproblems)
  Engine outer, mid, inner;
  DevArray<double> bivec;
  DevArray<int> bicnt;
  BiDev bi{}, bi2{};  // Bi-PQN state of the top level and of the middle level
  DevArray<double> MDx, MDp, Unc;
  void ensure(int n, int M) {
    if (n <= cap && MDx.p) return;
    cap = std::max(n, 1);
    pairs.alloc(2 * (size_t)cap);
    outer.alloc(cap);
    mid.alloc(cap);
    inner.alloc(cap);
    const size_t per = (size_t)(4 * kRmax + 4) * cap;
    bivec.alloc(2 * per);
    bicnt.alloc(4);
    BiDev* bs[2] = {&bi, &bi2};
    for (int l = 0; l < 2; ++l) {
      BiDev& b = *bs[l];
      double* v = bivec.p + l * per;
      b.Uc = v;
      b.Vc = v + (size_t)kRmax * cap;
      b.Slow = v + (size_t)2 * kRmax * cap;
      b.Ylow = v + (size_t)3 * kRmax * cap;
      b.Alox = v + (size_t)4 * kRmax * cap;
      b.Alos = b.Alox + cap;
      b.Bs = b.Alos + cap;
      b.tmp = b.Bs + cap;
      b.cnt = bicnt.p + 2 * l;
    }
    MDx.alloc(6 * (size_t)M);
    MDp.alloc(6 * (size_t)M);
    Unc.alloc(6 * (size_t)M);
  }
  void set_n(int n) {
    outer.d.n = n;
    mid.d.n = n;
    inner.d.n = n;
    bi.n = n;
    bi2.n = n;
  }
};

void lcp_release(LcpState* st) { delete st; }

static LcpState& state(pqn_ctx_impl& ctx) {
  if (!ctx.lcp) ctx.lcp = new LcpState();
  return *ctx.lcp;
}

void lcp_check_pairs(pqn_ctx_impl& ctx, int n, const int32_t* pairs) {
  for (int l = 0; l < n; ++l) {
    const int i = pairs[2 * l], j = pairs[2 * l + 1];
    if (i < 0 || j < 0 || i >= ctx.M || j >= ctx.M || i == j)
      throw Error(PQN_ERR_INVALID, "contact pair with an invalid sphere index");
  }
}

int lcp_find_contacts(pqn_ctx_impl& ctx, double delta) {
  LcpState& st = state(ctx);
  const int cap = ctx.M * 12 + 16;  // more contacts than 6 per sphere cannot occur without overlap
  st.cpairs.alloc(2 * (size_t)cap);
  st.cgaps.alloc(cap);
  st.ccount.alloc(1);
  hipLaunchKernelGGL(k_contacts, dim3(1), dim3(kT), 0, ctx.stream, ctx.ctr.p, ctx.M, ctx.a, delta, cap,
                     st.cpairs.p, st.cgaps.p, st.ccount.p);
  int n = 0;
  HIPCHK(hipMemcpyAsync(&n, st.ccount.p, sizeof(int), hipMemcpyDeviceToHost, ctx.stream));
  HIPCHK(hipStreamSynchronize(ctx.stream));
  if (n > cap) throw Error(PQN_ERR_INVALID, "more contacts than 12 per sphere: overlapping spheres?");
  return n;
}

void lcp_copy_contacts(pqn_ctx_impl& ctx, int n, int32_t* pairs, double* gaps) {
  LcpState& st = state(ctx);
  if (n == 0) return;
  HIPCHK(hipMemcpyAsync(pairs, st.cpairs.p, 2 * (size_t)n * sizeof(int), hipMemcpyDeviceToHost, ctx.stream));
  HIPCHK(hipMemcpyAsync(gaps, st.cgaps.p, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  HIPCHK(hipStreamSynchronize(ctx.stream));
}

// One LCP product out = D^T M D v on the device; M D v also left in UO_out.
static void lcp_mvp(pqn_ctx_impl& ctx, Level& lv, int n, const int* pairs_dev, const double* v, double* out,
                    double* UO_out, int* gmres_its) {
  hipLaunchKernelGGL(k_D_scatter, dim3((ctx.M + kT - 1) / kT), dim3(kT), 0, ctx.stream, ctx.ctr.p, pairs_dev, v, n,
                     ctx.M, ctx.FT.p);
  pqn_mvp_stats ms{};
  ctx.mobility(lv, ctx.FT.p, nullptr, UO_out, &ms);
  hipLaunchKernelGGL(k_DT_gather, dim3((n + kT - 1) / kT), dim3(kT), 0, ctx.stream, ctx.ctr.p, pairs_dev, UO_out, n,
                     out);
  HIPCHK(hipGetLastError());
  if (gmres_its) *gmres_its += ms.gmres_iters;
}

pqn_status lcp_apply_host(pqn_ctx_impl& ctx, int n, const int32_t* pairs, const double* x, double* Ax,
                          int fidelity) {
  if (n == 0) return PQN_OK;
  LcpState& st = state(ctx);
  st.ensure(n, ctx.M);
  st.set_n(n);
  Level& lv = ctx.level(fidelity);
  HIPCHK(hipMemcpyAsync(st.pairs.p, pairs, 2 * (size_t)n * sizeof(int), hipMemcpyHostToDevice, ctx.stream));
  double* xd = st.outer.d.t1;
  double* yd = st.outer.d.t2;
  HIPCHK(hipMemcpyAsync(xd, x, (size_t)n * sizeof(double), hipMemcpyHostToDevice, ctx.stream));
  lcp_mvp(ctx, lv, n, st.pairs.p, xd, yd, ctx.UO.p, nullptr);
  HIPCHK(hipMemcpyAsync(Ax, yd, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  HIPCHK(hipStreamSynchronize(ctx.stream));
  ctx.end_far_timing();
  return PQN_OK;
}

struct SolveCounters {
  int mvp[3] = {0, 0, 0};  // LCP products per fidelity (PQN_HIFI, PQN_LOFI, PQN_LOFI2)
  double t[3] = {0.0, 0.0, 0.0};
  int gmres = 0;
};

static PqnScal read_scal(pqn_ctx_impl& ctx, const PqnScal* d) {
  PqnScal h{};
  HIPCHK(hipMemcpyAsync(&h, d, sizeof(PqnScal), hipMemcpyDeviceToHost, ctx.stream));
  HIPCHK(hipStreamSynchronize(ctx.stream));
  return h;
}

// Mono-PQN (Alg. 1) on an engine; mvp(v, out, md) computes out = A v (md: M D v or null).
// Returns whether it converged; the engine holds x, A x and the memory.
template <class Mvp>
static bool run_mono(pqn_ctx_impl& ctx, Engine& E, int k_max, const pqn_lcp_opts& o, Mvp&& mvp, double* MDx, int M,
                     int* iters) {
  bool conv = false;
  int k = 0;
  for (k = 0; k < k_max; ++k) {
    TraceRange trace_iter("pqn_iteration");
    hipLaunchKernelGGL(k_pqn_prepare, dim3(1), dim3(kT), 0, ctx.stream, E.d, o.j_max, o.ssn_tol);
    HIPCHK(hipGetLastError());
    PqnScal s = read_scal(ctx, E.d.sc);
    if (!std::isfinite(s.e)) throw Error(PQN_ERR_NUMERIC, "non-finite KKT error in PQN");
    if (s.conv || s.stationary) {
      conv = true;
      break;
    }
    mvp(E.d.p, E.d.Ap, MDx ? ctx.lcp->MDp.p : nullptr);
    hipLaunchKernelGGL(k_pqn_accept, dim3(1), dim3(kT), 0, ctx.stream, E.d);
    if (MDx)
      hipLaunchKernelGGL(k_axpy_dev, dim3((6 * M + 255) / 256), dim3(256), 0, ctx.stream, MDx, ctx.lcp->MDp.p,
                         E.d.sc, 6 * M);
    HIPCHK(hipGetLastError());
  }
  if (!conv) {
    // final KKT evaluation (no product needed: A x is carried by the recurrence)
    hipLaunchKernelGGL(k_pqn_prepare, dim3(1), dim3(kT), 0, ctx.stream, E.d, o.j_max, o.ssn_tol);
    PqnScal s = read_scal(ctx, E.d.sc);
    conv = s.conv;
  }
  if (iters) *iters += k;
  return conv;
}

static pqn_lcp_opts opts_or_default(const pqn_lcp_opts* o) {
  pqn_lcp_opts r{100, 50, 50, 1e-8, 1e-8, 1e-14, 0, 0};
  if (o) {
    if (o->k_max > 0) r.k_max = o->k_max;
    if (o->k_max_inner > 0) r.k_max_inner = o->k_max_inner;
    if (o->j_max > 0) r.j_max = o->j_max;
    if (o->kkt_tol_abs > 0) r.kkt_tol_abs = o->kkt_tol_abs;
    if (o->kkt_tol_rel > 0) r.kkt_tol_rel = o->kkt_tol_rel;
    if (o->ssn_tol > 0) r.ssn_tol = o->ssn_tol;
    if (o->printed_metric < 0 || o->printed_metric > 1) throw Error(PQN_ERR_INVALID, "printed_metric must be 0 or 1");
    r.printed_metric = o->printed_metric;
    if (o->recycle < 0 || o->recycle > 1) throw Error(PQN_ERR_INVALID, "recycle must be 0 or 1");
    r.recycle = o->recycle;
  }
  return r;
}

// Bi-PQN (Alg. 4) and its recursive form over up to three fidelities. Level d
// minimises 1/2 z.H_d z + c.z over z >= 0 from the iterate in its engine, with
// H_0 = A and, below, H_d = A_d + C_0 + ... + C_{d-1} (A_d the LCP product at
// fidelity d, C_e the BFGS corrections U U^T - V V^T of the enclosing Bi-PQN
// levels). A Bi-PQN level models H_d by A_{d+1} + C_0 + ... + C_d and solves
// each subproblem one level down; the lowest level is Mono-PQN. With two
// fidelities this is Alg. 4 as written (plus the model safeguard).
struct BiSolver {
  pqn_ctx_impl& ctx;
  LcpState& st;
  const pqn_lcp_opts& o;
  SolveCounters& cnt;
  int n, M, nf;     // nf fidelities: 2 = Bi-PQN, 3 = recursive Bi-PQN
  double* MDx;      // M D x of the top level (may be null)
  bool x0;          // the top level starts from the caller's x^(-1) (in its engine's x), not 0
  Level* lv[3];
  Engine* eng[3];   // engine of each level (eng[nf - 1] runs Mono-PQN)
  BiDev* bd[2];     // Bi-PQN state of each Bi-PQN level
  int ssn = 0, in_iters = 0;
  bool rejected = false;  // the top level finished as Mono-PQN on A

  // out = A_d v + C_0 v + ... + C_{nc-1} v (nc = d: H_d v); md (top level only)
  // receives M D v.
  void op(int d, const double* v, double* out, double* md, int nc = -1) {
    Timer t;
    if (nc < 0) nc = d;
    if (nc == 0) {
      lcp_mvp(ctx, *lv[d], n, st.pairs.p, v, out, md ? md : ctx.UO.p, &cnt.gmres);
    } else {
      const double* cur = bd[0]->tmp;
      lcp_mvp(ctx, *lv[d], n, st.pairs.p, v, bd[0]->tmp, ctx.UO.p, &cnt.gmres);
      for (int e = 0; e < nc; ++e) {
        double* dst = e == nc - 1 ? out : bd[e + 1]->tmp;
        hipLaunchKernelGGL(k_lowrank, dim3(1), dim3(kT), 0, ctx.stream, *bd[e], cur, v, dst);
        cur = dst;
      }
      HIPCHK(hipGetLastError());
    }
    HIPCHK(hipStreamSynchronize(ctx.stream));
    cnt.t[d] += t.ms();
    cnt.mvp[d] += 1;
  }

  // (small host-to-device copies from the stack: the stream is synchronised before
  // the source goes out of scope)
  void set_counts(BiDev& B, int rc, int nlow) {
    int h[2] = {rc, nlow};
    HIPCHK(hipMemcpyAsync(B.cnt, h, 2 * sizeof(int), hipMemcpyHostToDevice, ctx.stream));
    HIPCHK(hipStreamSynchronize(ctx.stream));
  }

  void set_pair_count(BiDev& B, int nlow) {
    HIPCHK(hipMemcpyAsync(B.cnt + 1, &nlow, sizeof(int), hipMemcpyHostToDevice, ctx.stream));
    HIPCHK(hipStreamSynchronize(ctx.stream));
  }

  // initial metric scale of a Mono-PQN solve: 1 = H0 = I as printed, 0 = set by its first step
  double sigma0() const { return o.printed_metric ? 1.0 : 0.0; }

  void init_scal(Engine& E, double tol_abs, double sigma) {
    PqnScal z{};
    z.tol_abs = tol_abs;
    z.tol_rel = o.kkt_tol_rel;
    z.sigma = sigma;
    HIPCHK(hipMemcpyAsync(E.d.sc, &z, sizeof(PqnScal), hipMemcpyHostToDevice, ctx.stream));
    HIPCHK(hipStreamSynchronize(ctx.stream));
  }

  struct Result {
    int resets = 0;  // Alg. 2 edge cases met on H_d (own steps and fallback)
    bool conv = false;
    double kkt = 0.0;
    int iters = 0;
  };

  // Mono-PQN on H_d from the iterate (x, H_d x) in its engine; level d - 1's stored
  // secant pairs (npairs of them) warm the memory.
  Result mono_level(int d, double tol, int k_lim, double& sigma, int npairs) {
    Engine& E = *eng[d];
    init_scal(E, tol, sigma);
    if (npairs > 0)
      hipLaunchKernelGGL(k_pqn_replay, dim3(1), dim3(kT), 0, ctx.stream, E.d, bd[d - 1]->Slow, bd[d - 1]->Ylow,
                         npairs);
    Result r;
    run_mono(ctx, E, k_lim, o, [&](const double* v, double* out, double*) { op(d, v, out, nullptr); },
             nullptr, M, &in_iters);
    PqnScal s = read_scal(ctx, E.d.sc);
    ssn += s.ssn_steps;
    sigma = s.sigma;
    r.resets = s.resets;
    r.conv = s.conv || s.stationary;
    r.kkt = s.e;
    return r;
  }

  // Model safeguard: level d continues as Mono-PQN on H_d from its current
  // iterate (keep_x), from the top level's x^(-1) (restart: x is still in the
  // engine, A x is evaluated again) or from 0.
  Result fallback(int d, double tol, int k_lim, bool keep_x, int k_done, int resets_before, bool restart = false) {
    Engine& E = *eng[d];
    const bool top = d == 0;
    if (top) rejected = true;
    hipLaunchKernelGGL(k_pqn_init, dim3(1), dim3(kT), 0, ctx.stream, E.d, keep_x || restart ? 1 : 0, tol,
                       o.kkt_tol_rel, sigma0());
    double* md = top ? MDx : nullptr;
    if (restart)
      op(d, E.d.x, E.d.Ax, md);  // md (if any) receives M D x^(-1)
    else if (md && !keep_x)
      HIPCHK(hipMemsetAsync(md, 0, 6 * (size_t)M * sizeof(double), ctx.stream));
    int it = 0;
    Result r;
    r.conv = run_mono(
        ctx, E, std::max(1, k_lim - k_done), o,
        [&](const double* v, double* out, double* mdv) { op(d, v, out, top ? mdv : nullptr); }, md, M, &it);
    PqnScal sm = read_scal(ctx, E.d.sc);
    ssn += sm.ssn_steps;
    r.kkt = sm.e;
    r.iters = k_done + it;
    r.resets = resets_before + sm.resets;
    return r;
  }

  // Bi-PQN at level d < nf - 1. Top level: from x = 0 with Alg. 4's initial solve
  // one level down. Nested: from the iterate the caller left in the engine
  // (b = c, x, A x = H_d x), with A_{d+1} x paid by one product, and with the
  // correction C_d its previous calls left (H_d - (A_{d+1} + C_0 + ... + C_{d-1})
  // = A_d - A_{d+1} does not depend on the enclosing corrections, so it stays
  // valid; the top level clears it once per solve).
  Result bi_level(int d, double tol, int k_lim, double& sigma) {
    const bool top = d == 0;
    Engine& E = *eng[d];
    Engine& I = *eng[d + 1];
    BiDev& B = *bd[d];
    const bool mono_in = d + 1 == nf - 1;
    auto solve_in = [&](double tol_in, double& sg, int npairs) {
      return mono_in ? mono_level(d + 1, tol_in, o.k_max_inner, sg, npairs) : bi_level(d + 1, tol_in, o.k_max_inner, sg);
    };
    if (top) {
      for (int l = 0; l < nf - 1; ++l) set_counts(*bd[l], 0, 0);
      // initial solve one level down from x^(-1) with tolerance 1e-2 x the model's KKT
      // error there (|min(0, b)| at x^(-1) = 0, where the model product is free)
      HIPCHK(hipMemcpyAsync(I.d.b, E.d.b, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, ctx.stream));
      if (x0) {
        HIPCHK(hipMemcpyAsync(I.d.x, E.d.x, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, ctx.stream));
        op(1, I.d.x, I.d.Ax, nullptr);  // no correction yet: A_1 x^(-1)
        hipLaunchKernelGGL(k_kkt, dim3(1), dim3(kT), 0, ctx.stream, I.d.x, I.d.Ax, I.d.b, n, E.d.sc);
      } else {
        hipLaunchKernelGGL(k_pqn_init, dim3(1), dim3(kT), 0, ctx.stream, I.d, 0, 0.0, 0.0, sigma0());
        hipLaunchKernelGGL(k_kkt_zero, dim3(1), dim3(kT), 0, ctx.stream, E.d.b, n, E.d.sc);
      }
      const double e0 = read_scal(ctx, E.d.sc).e;
      Result r0 = solve_in(std::max(1e-12, 1e-2 * e0), sigma, 0);
      if (r0.resets > 0) return fallback(d, tol, k_lim, false, 0, 0, x0);
      // x = x0, A^ x = its model product, stored pairs = its Mono-PQN memory
      init_scal(E, tol, 0.0);
      HIPCHK(hipMemcpyAsync(E.d.x, I.d.x, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, ctx.stream));
      HIPCHK(hipMemcpyAsync(B.Alox, I.d.Ax, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, ctx.stream));
      int nlow = 0;
      if (mono_in) {
        nlow = std::min(read_scal(ctx, I.d.sc).r, kRmax);
        if (nlow > 0) {
          HIPCHK(hipMemcpyAsync(B.Slow, I.d.S, (size_t)nlow * n * sizeof(double), hipMemcpyDeviceToDevice,
                                ctx.stream));
          HIPCHK(hipMemcpyAsync(B.Ylow, I.d.Y, (size_t)nlow * n * sizeof(double), hipMemcpyDeviceToDevice,
                                ctx.stream));
        }
      }
      set_counts(B, 0, nlow);
      hipLaunchKernelGGL(k_nonzero, dim3(1), dim3(kT), 0, ctx.stream, E.d.x, n, E.d.sc);
      if (read_scal(ctx, E.d.sc).nonzero)
        op(0, E.d.x, E.d.Ax, MDx);
      else
        HIPCHK(hipMemsetAsync(E.d.Ax, 0, (size_t)n * sizeof(double), ctx.stream));
    } else {
      init_scal(E, tol, 0.0);
      set_pair_count(B, 0);
      hipLaunchKernelGGL(k_nonzero, dim3(1), dim3(kT), 0, ctx.stream, E.d.x, n, E.d.sc);
      if (read_scal(ctx, E.d.sc).nonzero)
        op(d + 1, E.d.x, B.Alox, nullptr, d);  // A_{d+1} x + C_0 x + ... + C_{d-1} x
      else
        HIPCHK(hipMemsetAsync(B.Alox, 0, (size_t)n * sizeof(double), ctx.stream));
    }
    Result r;
    int k = 0;
    for (k = 0; k < k_lim; ++k) {
      TraceRange trace_iter(top ? "bi_pqn_outer_iteration" : "bi_pqn_nested_iteration");
      hipLaunchKernelGGL(k_bi_prepare, dim3(1), dim3(kT), 0, ctx.stream, E.d, B, I.d);
      PqnScal so = read_scal(ctx, E.d.sc);
      if (!std::isfinite(so.e)) throw Error(PQN_ERR_NUMERIC, "non-finite KKT error in Bi-PQN");
      r.kkt = so.e;
      if (so.conv) {
        r.conv = true;
        break;
      }
      // subproblem one level down, from x, warm-started with the stored pairs
      int hc[2];
      HIPCHK(hipMemcpyAsync(hc, B.cnt, 2 * sizeof(int), hipMemcpyDeviceToHost, ctx.stream));
      HIPCHK(hipStreamSynchronize(ctx.stream));
      Result ri = solve_in(std::max(1e-12, 1e-2 * so.e), sigma, hc[1]);
      if (ri.resets > 0) return fallback(d, tol, k_lim, true, k, read_scal(ctx, E.d.sc).resets);
      hipLaunchKernelGGL(k_bi_direction, dim3(1), dim3(kT), 0, ctx.stream, E.d, I.d);
      if (read_scal(ctx, E.d.sc).stationary) {
        r.conv = true;
        break;
      }
      op(d, E.d.p, E.d.Ap, top && MDx ? st.MDp.p : nullptr);
      hipLaunchKernelGGL(k_bi_accept, dim3(1), dim3(kT), 0, ctx.stream, E.d, B, I.d);
      if (top && MDx)
        hipLaunchKernelGGL(k_axpy_dev, dim3((6 * M + 255) / 256), dim3(256), 0, ctx.stream, MDx, st.MDp.p, E.d.sc,
                           6 * M);
      HIPCHK(hipGetLastError());
    }
    if (!r.conv) {
      hipLaunchKernelGGL(k_bi_prepare, dim3(1), dim3(kT), 0, ctx.stream, E.d, B, I.d);
      PqnScal sf = read_scal(ctx, E.d.sc);
      r.conv = sf.conv;
      r.kkt = sf.e;
    }
    r.iters = k;
    r.resets = read_scal(ctx, E.d.sc).resets;
    return r;
  }
};

// Reuse of earlier solutions across the products of one solve (pqn_lcp_opts.recycle) on
// every level of the context, for the duration of the solve; the stores start empty.
struct RecycleScope {
  std::vector<Level*> lv;
  RecycleScope(pqn_ctx_impl& ctx, bool on) {
    if (!on || (ctx.cfg.precision == PQN_MIXED && ctx.cfg.refine_sweeps > 0)) return;
    lv.push_back(&ctx.hi);
    if (ctx.has_lo) lv.push_back(&ctx.lo);
    if (ctx.has_lo2) lv.push_back(&ctx.lo2);
    for (Level* l : lv) {
      l->rc.active = true;
      l->rc.k = 0;
    }
  }
  ~RecycleScope() {
    for (Level* l : lv) {
      l->rc.active = false;
      l->rc.k = 0;
    }
  }
  RecycleScope(const RecycleScope&) = delete;
  RecycleScope& operator=(const RecycleScope&) = delete;
};

// Solve the LCP with b (device, length n) on the stored pairs. x ends in
// st.outer.d.x; MDx (if non-null) receives M D x.
static bool solve_device(pqn_ctx_impl& ctx, int n, int solver, const pqn_lcp_opts& o, double* MDx,
                         pqn_lcp_stats* stats, bool x0) {
  LcpState& st = *ctx.lcp;
  RecycleScope recycle_scope(ctx, o.recycle != 0);
  SolveCounters cnt;
  Level& hi = ctx.hi;
  const int M = ctx.M;
  auto mvp_hi = [&](const double* v, double* out, double* md) {
    Timer t;
    lcp_mvp(ctx, hi, n, st.pairs.p, v, out, md ? md : ctx.UO.p, &cnt.gmres);
    HIPCHK(hipStreamSynchronize(ctx.stream));
    cnt.t[0] += t.ms();
    cnt.mvp[0] += 1;
  };
  if (MDx) HIPCHK(hipMemsetAsync(MDx, 0, 6 * (size_t)M * sizeof(double), ctx.stream));
  bool conv = false;
  bool rejected = false;
  int iters = 0;
  int ssn = 0;
  double kkt = 0.0;
  hipLaunchKernelGGL(k_pqn_init, dim3(1), dim3(kT), 0, ctx.stream, st.outer.d, x0 ? 1 : 0, o.kkt_tol_abs,
                     o.kkt_tol_rel, o.printed_metric ? 1.0 : 0.0);
  // Mono-PQN and BB-PGD from x^(-1): A x^(-1) (and M D x^(-1)) by one product
  if (x0 && solver != PQN_BI && solver != PQN_BI_REC) mvp_hi(st.outer.d.x, st.outer.d.Ax, MDx);
  if (solver == PQN_MONO) {
    conv = run_mono(ctx, st.outer, o.k_max, o, mvp_hi, MDx, M, &iters);
    PqnScal s = read_scal(ctx, st.outer.d.sc);
    ssn = s.ssn_steps;
    kkt = s.e;
  } else if (solver == PQN_BBPGD) {
    const double tau0 = 3.0 * kPi * ctx.mu * ctx.a;  // inverse of twice the single-sphere mobility
    int k = 0;
    for (k = 0; k < o.k_max; ++k) {
      hipLaunchKernelGGL(k_bb_prepare, dim3(1), dim3(kT), 0, ctx.stream, st.outer.d, tau0);
      PqnScal s = read_scal(ctx, st.outer.d.sc);
      if (!std::isfinite(s.e)) throw Error(PQN_ERR_NUMERIC, "non-finite KKT error in BB-PGD");
      kkt = s.e;
      if (s.conv) {
        conv = true;
        break;
      }
      mvp_hi(st.outer.d.x, st.outer.d.Ax, MDx);
    }
    if (!conv) {
      hipLaunchKernelGGL(k_bb_prepare, dim3(1), dim3(kT), 0, ctx.stream, st.outer.d, tau0);
      PqnScal s = read_scal(ctx, st.outer.d.sc);
      conv = s.conv;
      kkt = s.e;
    }
    iters = k;
  } else {
    const bool rec = solver == PQN_BI_REC;
    BiSolver bs{ctx, st, o, cnt, n, M, rec ? 3 : 2, MDx, x0, {&ctx.hi, &ctx.lo, rec ? &ctx.lo2 : nullptr},
                {&st.outer, rec ? &st.mid : &st.inner, rec ? &st.inner : nullptr}, {&st.bi, &st.bi2}};
    double sigma = bs.sigma0();  // metric scale of the Mono-PQN solves (0 = set by their first step)
    BiSolver::Result r = bs.bi_level(0, o.kkt_tol_abs, o.k_max, sigma);
    conv = r.conv;
    kkt = r.kkt;
    iters = r.iters;
    ssn = bs.ssn;
    rejected = bs.rejected;
  }
  const PqnScal fin = read_scal(ctx, st.outer.d.sc);
  if (stats) {
    const double mx = std::max(fin.e, fin.e_prev);
    stats->kkt_rel = fin.have_prev && mx > 0.0 ? std::fabs(fin.e - fin.e_prev) / mx : 0.0;
    stats->iters = iters;
    stats->mvp_hi = cnt.mvp[0];
    stats->mvp_lo = cnt.mvp[1];
    stats->mvp_lo2 = cnt.mvp[2];
    auto ratio = [&](int f) {
      return (cnt.mvp[f] > 0 && cnt.mvp[0] > 0) ? (cnt.t[f] / cnt.mvp[f]) / (cnt.t[0] / cnt.mvp[0]) : 0.0;
    };
    stats->lo_hi_cost_ratio = ratio(1);
    stats->lo2_hi_cost_ratio = ratio(2);
    stats->emvp = cnt.mvp[0] + cnt.mvp[1] * ratio(1) + cnt.mvp[2] * ratio(2);
    stats->kkt_abs = kkt;
    stats->converged = conv ? 1 : 0;
    stats->ssn_steps = ssn;
    stats->gmres_iters = cnt.gmres;
    stats->model_rejected = rejected ? 1 : 0;
    stats->nonpos_curvature = fin.nonpos;
  }
  return conv;
}

pqn_status lcp_solve_host(pqn_ctx_impl& ctx, int n, const int32_t* pairs, const double* b, double* x, int solver,
                          const pqn_lcp_opts* opts, pqn_lcp_stats* stats) {
  Timer tm;
  pqn_lcp_stats st_local{};
  if (n == 0) {
    if (stats) *stats = st_local;
    return PQN_OK;
  }
  for (int l = 0; l < n; ++l)
    if (!std::isfinite(b[l])) throw Error(PQN_ERR_NUMERIC, "non-finite b");
  LcpState& st = state(ctx);
  st.ensure(n, ctx.M);
  st.set_n(n);
  const pqn_lcp_opts o = opts_or_default(opts);
  // x^(-1): the caller's x projected on x >= 0
  std::vector<double> xg(x, x + n);
  bool x0 = false;
  for (double& v : xg) {
    if (!std::isfinite(v)) throw Error(PQN_ERR_NUMERIC, "non-finite initial guess x");
    v = std::max(v, 0.0);
    x0 = x0 || v > 0.0;
  }
  HIPCHK(hipMemcpyAsync(st.pairs.p, pairs, 2 * (size_t)n * sizeof(int), hipMemcpyHostToDevice, ctx.stream));
  HIPCHK(hipMemcpyAsync(st.outer.d.b, b, (size_t)n * sizeof(double), hipMemcpyHostToDevice, ctx.stream));
  if (x0) HIPCHK(hipMemcpyAsync(st.outer.d.x, xg.data(), (size_t)n * sizeof(double), hipMemcpyHostToDevice, ctx.stream));
  HIPCHK(hipStreamSynchronize(ctx.stream));  // xg leaves scope only after the copy
  const bool conv = solve_device(ctx, n, solver, o, nullptr, &st_local, x0);
  HIPCHK(hipMemcpyAsync(x, st.outer.d.x, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  HIPCHK(hipStreamSynchronize(ctx.stream));
  ctx.end_far_timing();
  st_local.t_total_ms = tm.ms();
  if (stats) *stats = st_local;
  return conv ? PQN_OK : PQN_WARN_NOT_CONVERGED;
}

pqn_status lcp_solve_dev(pqn_ctx_impl& ctx, int n, const int32_t* pairs, const double* b, double* x, int solver,
                         const pqn_lcp_opts* opts, pqn_lcp_stats* stats) {
  Timer tm;
  pqn_lcp_stats st_local{};
  if (n == 0) {
    if (stats) *stats = st_local;
    return PQN_OK;
  }
  LcpState& st = state(ctx);
  st.ensure(n, ctx.M);
  st.set_n(n);
  const pqn_lcp_opts o = opts_or_default(opts);
  HIPCHK(hipMemcpyAsync(st.pairs.p, pairs, 2 * (size_t)n * sizeof(int), hipMemcpyDeviceToDevice, ctx.stream));
  HIPCHK(hipMemcpyAsync(st.outer.d.b, b, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, ctx.stream));
  HIPCHK(hipMemcpyAsync(st.outer.d.x, x, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, ctx.stream));
  hipLaunchKernelGGL(k_check_lcp_inputs, dim3(1), dim3(kT), 0, ctx.stream, st.pairs.p, st.outer.d.b, st.outer.d.x, n,
                     ctx.M, st.outer.d.sc);
  const PqnScal chk = read_scal(ctx, st.outer.d.sc);
  if (chk.bad) throw Error(PQN_ERR_INVALID, "invalid contact pair or non-finite b / x");
  const bool conv = solve_device(ctx, n, solver, o, nullptr, &st_local, chk.nonzero != 0);
  HIPCHK(hipMemcpyAsync(x, st.outer.d.x, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, ctx.stream));
  HIPCHK(hipStreamSynchronize(ctx.stream));
  ctx.end_far_timing();
  st_local.t_total_ms = tm.ms();
  if (stats) *stats = st_local;
  return conv ? PQN_OK : PQN_WARN_NOT_CONVERGED;
}

// b = Phi/dt + D^T U_nc (eq. (defAandb))
__global__ void k_make_b(const double* __restrict__ gaps, const double* __restrict__ dtu, double dt, int n,
                         double* __restrict__ b) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < n) b[l] = gaps[l] / dt + dtu[l];
}

pqn_status lcp_step(pqn_ctx_impl& ctx, double dt, double delta, int solver, const pqn_lcp_opts* opts,
                    pqn_step_stats* stats) {
  Timer tm;
  pqn_step_stats ss{};
  LcpState& st = state(ctx);
  const int M = ctx.M;
  Timer t_stage;
  const int n = lcp_find_contacts(ctx, delta);  // (reads the count back: the stream is synchronised)
  ss.t_contacts_ms = t_stage.ms();
  st.ensure(n, M);
  st.set_n(std::max(n, 1));
  // U_nc from the slip-driven solve (F = T = 0)
  t_stage = Timer();
  pqn_mvp_stats ms{};
  if (ctx.has_axes) {
    ctx.mobility(ctx.hi, nullptr, ctx.dax.p, st.Unc.p, &ms);
  } else {
    HIPCHK(hipMemsetAsync(st.Unc.p, 0, 6 * (size_t)M * sizeof(double), ctx.stream));
  }
  HIPCHK(hipStreamSynchronize(ctx.stream));
  ss.t_nc_ms = t_stage.ms();
  t_stage = Timer();
  ss.gmres_iters_nc = ms.gmres_iters;
  ss.n_contacts = n;
  bool conv = true;
  double* MDx = nullptr;
  if (n > 0) {
    HIPCHK(hipMemcpyAsync(st.pairs.p, st.cpairs.p, 2 * (size_t)n * sizeof(int), hipMemcpyDeviceToDevice,
                          ctx.stream));
    hipLaunchKernelGGL(k_DT_gather, dim3((n + kT - 1) / kT), dim3(kT), 0, ctx.stream, ctx.ctr.p, st.pairs.p,
                       st.Unc.p, n, st.outer.d.t1);
    hipLaunchKernelGGL(k_make_b, dim3((n + 255) / 256), dim3(256), 0, ctx.stream, st.cgaps.p, st.outer.d.t1, dt, n,
                       st.outer.d.b);
    const pqn_lcp_opts o = opts_or_default(opts);
    conv = solve_device(ctx, n, solver, o, st.MDx.p, &ss.lcp, false);
    if (!conv && ss.lcp.nonpos_curvature > 0) {
      // the iterate of a solve that met p.Ap <= 0 on A and did not converge can be
      // arbitrarily large: moving the spheres with it would scatter them
      throw Error(PQN_ERR_INDEFINITE,
                  "pqn_step: the contact LCP matrix A = D^T M D is not positive definite (p.Ap <= 0 along a "
                  "search direction; typically a near-contact pair the surface grid does not resolve) and the "
                  "solve did not converge; configuration unchanged");
    }
    MDx = st.MDx.p;
    std::vector<double> hx(n);
    HIPCHK(hipMemcpyAsync(hx.data(), st.outer.d.x, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
    HIPCHK(hipStreamSynchronize(ctx.stream));
    for (double v : hx) ss.n_active += v > 0.0;
  }
  ss.t_lcp_ms = t_stage.ms();
  t_stage = Timer();
  hipLaunchKernelGGL(k_euler, dim3((M + 255) / 256), dim3(256), 0, ctx.stream, ctx.ctr.p, ctx.dax.p, st.Unc.p, MDx,
                     M, dt, ctx.has_axes ? 1 : 0);
  HIPCHK(hipGetLastError());
  std::vector<double> c(3 * (size_t)M), ax(3 * (size_t)M);
  HIPCHK(hipMemcpyAsync(c.data(), ctx.ctr.p, c.size() * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  HIPCHK(hipMemcpyAsync(ax.data(), ctx.dax.p, ax.size() * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  HIPCHK(hipStreamSynchronize(ctx.stream));
  ctx.end_far_timing();
  try {
    ctx.set_configuration(c.data(), ctx.has_axes ? ax.data() : nullptr);
  } catch (...) {
    // the new configuration was rejected (e.g. a sphere with more near partners than
    // the near tables hold): the context keeps the old one, device copies included
    HIPCHK(hipMemcpyAsync(ctx.ctr.p, ctx.centers.data(), ctx.centers.size() * sizeof(double),
                          hipMemcpyHostToDevice, ctx.stream));
    HIPCHK(hipMemcpyAsync(ctx.dax.p, ctx.axes.data(), ctx.axes.size() * sizeof(double), hipMemcpyHostToDevice,
                          ctx.stream));
    HIPCHK(hipStreamSynchronize(ctx.stream));
    throw;
  }
  ss.t_update_ms = t_stage.ms();
  ss.t_total_ms = tm.ms();
  if (stats) *stats = ss;
  return conv ? PQN_OK : PQN_WARN_NOT_CONVERGED;
}

}  // namespace bipqn
