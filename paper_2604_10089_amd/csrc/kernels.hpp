// Launch wrappers of the device kernels (kernels.hip).
#pragma once
#include "common.hpp"

namespace bipqn {

void launch_pack32(hipStream_t s, const double* q, const double* off, const double* w, int n, int N, float4* src);
void launch_pack64(hipStream_t s, const double* q, const double* off, const double* w, int n, int N, double2* src);
void launch_far32(hipStream_t s, int tpt, const float4* src, const double* off, const double* ctr,
                  const unsigned char* cls, int n, int M, int N, int spc, int nchunks, double scale, double* part);
void launch_far64(hipStream_t s, const double2* src, const double* off, const double* ctr, const unsigned char* cls,
                  int n, int M, int N, int spc, int nchunks, double scale, double* part);
void launch_near64(hipStream_t s, int max_slots, const double* ctr, const double* off, const double4* offup,
                   const double* qup, const double* coef, const int* partners, const int* npart, int n, int M, int N,
                   int nup, int p, int L, double scale, double* near_part);
void launch_gemm64(hipStream_t s, int R, int Cn, int K, const double* A, int lda, long Az, const double* B, long Bz,
                   int kb, long kbs, int ldb, double* C, long Cz, int rb, long rbs, int ldc, int batch);
void launch_near64p(hipStream_t s, int npairs_count, const double* ctr, const double* off, const double4* offup,
                    const double* qup, const double* coef, const int* npairs, int n, int M, int N, int nup, int p,
                    int L, double scale, double* near_part);
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
