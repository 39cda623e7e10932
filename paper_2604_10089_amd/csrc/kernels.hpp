// Launch wrappers of the device kernels (kernels.hip).
#pragma once
#include "common.hpp"

namespace bipqn {

constexpr int kMaxRhs = 6;   // densities sharing one geometry pass

struct QPtrs {
  const double* p[kMaxRhs];
};
struct OPtrs {
  double* p[kMaxRhs];
};

__host__ __device__ constexpr int src32_stride(int K) { return ((3 + 3 * K + 3) / 4) * 4; }
__host__ __device__ constexpr int src64_stride(int K) { return ((3 + 3 * K + 1) / 2) * 2; }

// One suspension's far pair sum inside a multi-suspension launch (single density).
struct FarDesc {
  const void* src;
  const double* off;
  const double* ctr;
  const unsigned char* cls;
  double* part;
  int n, M, N, spc, ntb, item0;
  double scale;
  const int* live;  // null, or a flag: 0 = the segment's system is done (its blocks exit)
};

// Segment descriptors of the multi-suspension kernels; `start` is the first
// block (GEMM, near, moments), element (pack, combine, combo) or vector (dots)
// of the segment in the launch.
struct GemmDesc {
  const double* A;
  const double* B;
  double* C;
  long rbs;
  int R, Cn, K, lda, ldb, rb, ldc, tr, start;
  int rs, cb;  // C(r, col) at C[(r / rb) rbs + (r % rb) rs + (col / cb) cbs + (col % cb) ldc]
  long cbs;
  const int* live;  // null, or a flag: 0 = the segment's system is done (its blocks exit)
  int at;           // bit 0: A(r, k) = A[k * lda + r] (A stored by columns), else A[r * lda + k];
                    // bit 1 (64x64-tile launches only): C += A B
};
struct PackDesc {
  const double* q;
  const double* off;
  const double* w;
  void* src;
  int n, N, start;
  const int* live;  // null, or a flag: 0 = the segment's system is done (its blocks exit)
};
struct NearDesc {
  const double* ctr;
  const double* off;
  const double4* offup;
  const double* shab;
  const double* qup;
  const double* coef;  // harmonic coefficients [M][3][L]
  const int* pairs;
  double* part;
  double scale;
  int n, M, N, nup, p, L, nch, start;
  const int* live;  // null, or a flag: 0 = the segment's system is done (its blocks exit)
};
struct MomDesc {
  const double* q;
  const double* off;
  const double* w;
  double* mom;
  int n, N, start;
  const int* live;  // null, or a flag: 0 = the segment's system is done (its blocks exit)
};
struct CombDesc {
  const double* q;
  const double* selfo;
  const double* far;
  const double* near;
  const int* npart;
  const double* mom;
  const double* off;
  double* y;
  double a;
  int nchunks, n, N, start;
  const int* live;  // null, or a flag: 0 = the segment's system is done (its blocks exit)
};
struct DotDesc {
  const double* V;
  const double* w;
  double* partial;
  double* out;
  long ldv, len;
  int start;
  const int* live;  // null, or a flag: 0 = the segment's system is done (its blocks exit)
};
struct ComboDesc {
  double* w;
  const double* V;
  const double* h;
  double alpha, beta;
  long ldv, len;
  int nvec, start;
  const int* live;  // null, or a flag: 0 = the segment's system is done (its blocks exit)
};

// Device state of one system of the graph-captured batched GMRES (see k_gmres_step).
struct GmSys {
  int active;   // 1 while the cycle runs; cleared when it converges or fills
  int k;        // current Arnoldi index
  int its;      // iterations of this solve
  int conv;     // 1 if the last residual estimate met the tolerance
  int err;      // 1 = non-finite value or breakdown
  int max_iter;
  double bnorm, tol, hn, inv_hn, relres;
};
// Per system: Hessenberg (m+1) x m row-major, then cs [m], sn [m], g [m+1] (stride gm_stride(m)).
__host__ __device__ constexpr long gm_stride(int m) { return (long)(m + 1) * m + 3L * m + 1; }
struct ScaleDesc {
  double* w;
  const double* s;   // device scale factor
  const int* live;
  long len;
  int start;
};

void launch_gemm64_multi(hipStream_t s, const GemmDesc* d, int nd, int nblocks);
// One Givens step of GMRES for every active system of a batch at Arnoldi index j: the
// Hessenberg column from the CGS2 dot products in hbuf (system i at hbuf + i hs: pass 1
// [m+1], pass 2 [m+1], |w|^2), the rotations, the residual estimate and the end test.
void launch_gmres_step(hipStream_t s, GmSys* sys, double* hess, const double* hbuf, int hs, int m, int ns);
void launch_scale_multi(hipStream_t s, const ScaleDesc* d, int nd, int total);
void launch_pack_multi(hipStream_t s, const PackDesc* d, int nd, int total, int fp32);
void launch_near_multi(hipStream_t s, const NearDesc* d, int nd, int nblocks);
void launch_moments_multi(hipStream_t s, const MomDesc* d, int nd, int nblocks);
void launch_combine_multi(hipStream_t s, const CombDesc* d, int nd, int total);
void launch_dots_multi(hipStream_t s, const DotDesc* d, int nd, int nvec_total, int nb);
void launch_combo_multi(hipStream_t s, const ComboDesc* d, int nd, int total);

// prec: 0 = FP64 pair sums, 1 = FP32 pair sums (mixed)
void launch_pack(hipStream_t s, int prec, int K, const QPtrs& q, const double* off, const double* w, int n, int N,
                 void* src);
// n target nodes per sphere, ns source nodes per sphere in src (n, or the coarse far-source grid's count)
void launch_far(hipStream_t s, int prec, int K, int tpt, const void* src, const double* off, const double* ctr,
                const unsigned char* cls, int n, int ns, int M, int N, int spc, int nchunks, double scale,
                const OPtrs& part);
// The far pair sum of the preconditioner's coarse level (kernels k_far32c / k_far64c, one
// target per thread; otherwise as launch_far): ns records per source sphere, the first ns1
// (one coarse grid) summed for the pairs with cls 0, the rest (the other grid) for those
// with cls2 0.
void launch_far_coarse(hipStream_t s, int prec, int K, const void* src, const double* off, const double* ctr,
                       const unsigned char* cls, const unsigned char* cls2, int n, int ns, int ns1, int M, int N,
                       int spc, int nchunks, double scale, const OPtrs& part);
// far sources from the coarse densities qc [M][nc][3K] at the coarse grid (offsets off, weights w)
void launch_pack_coarse(hipStream_t s, int prec, int K, const double* qc, const double* off, const double* w, int nc,
                        int Nc, void* src);
void launch_far_multi(hipStream_t s, int prec, int tpt, const FarDesc* desc, int ndesc, int nitems);
// coef: harmonic coefficients of the K densities, [M][3K][L] (row 3r + c: density r, component c)
void launch_near(hipStream_t s, int K, int npairs_count, const double* ctr, const double* off, const double4* offup,
                 const double* shab, const double* qup, const double* coef, const int* npairs, int n, int M, int N,
                 int nup, int p, int L, double scale, const OPtrs& near_part);
// C(r, col) = sum_k A[r * lda + k] B[col * ldb + k], stored at C[(r / rb) * rbs + col * ldc + r % rb];
// grid z = batch with strides Az, Bz, Cz.
void launch_gemm64(hipStream_t s, int R, int Cn, int K, const double* A, int lda, long Az, const double* B, long Bz,
                   int ldb, double* C, long Cz, int rb, long rbs, int ldc, int batch, int at = 0);
// The same with 64x64 tiles (large products); the segmented form takes descriptors whose
// tr and start count 64x64 tiles. With 64x64 tiles, at = 2 | (A by columns) accumulates
// into C (C += A B).
void launch_gemm64_big(hipStream_t s, int R, int Cn, int K, const double* A, int lda, long Az, const double* B,
                       long Bz, int ldb, double* C, long Cz, int rb, long rbs, int ldc, int batch, int at = 0);
void launch_gemm64_multi_big(hipStream_t s, const GemmDesc* d, int nd, int nblocks);

void launch_rhs(hipStream_t s, const double* ctr, const double* FT, const double* axes, const double* off, int n,
                int M, int N, double a, double mu, double slip, double* rhs);
void launch_moments(hipStream_t s, const double* q, const double* off, const double* w, int n, int M, int N,
                    double* mom);
void launch_rigid_velocity(hipStream_t s, const double* mom, int M, double a, double* UO);
void launch_combine(hipStream_t s, const double* q, const double* selfo, int nself, const double* far_part,
                    int nchunks, const double* near_part, const int* npart, const double* mom, const double* off,
                    int n, int N, double a, double* y);
void launch_dots(hipStream_t s, const double* V, long ldv, int nvec, const double* w, long len, int nb,
                 double* partial, double* out);
void launch_combo(hipStream_t s, double* w, double beta, const double* V, long ldv, int nvec, const double* h,
                  double alpha, long len);
void launch_scale_copy(hipStream_t s, double* y, const double* x, double a, long len);
void launch_axpby(hipStream_t s, double* y, const double* x, double a, double b, long len);

}  // namespace bipqn
