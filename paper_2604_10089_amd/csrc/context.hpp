// Library context: device tables and buffers of both fidelity levels, the BIE
// operator, GMRES and the mobility product.
#pragma once
#include <chrono>
#include <memory>
#include <stdexcept>
#include <utility>

#include "../../include/bipqn.h"
#include "kernels.hpp"

namespace bipqn {

struct Error : std::runtime_error {
  pqn_status code;
  Error(pqn_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(x)                                                                                   \
  do {                                                                                              \
    hipError_t e_ = (x);                                                                            \
    if (e_ != hipSuccess)                                                                           \
      throw ::bipqn::Error(e_ == hipErrorOutOfMemory ? PQN_ERR_OOM : PQN_ERR_DEVICE,                \
                           std::string(#x) + ": " + hipGetErrorString(e_));                          \
  } while (0)

template <class T>
struct DevArray {
  T* p = nullptr;
  size_t count = 0;
  DevArray() = default;
  DevArray(const DevArray&) = delete;
  DevArray& operator=(const DevArray&) = delete;
  ~DevArray() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    count = 0;
  }
  void alloc(size_t n) {
    if (n <= count && p) return;
    release();
    if (n == 0) return;
    HIPCHK(hipMalloc((void**)&p, n * sizeof(T)));
    count = n;
  }
  void upload(const T* h, size_t n, hipStream_t s) {
    alloc(n);
    if (n) HIPCHK(hipMemcpyAsync(p, h, n * sizeof(T), hipMemcpyHostToDevice, s));
  }
};

struct Timer {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
};

struct Level {
  SphereTables tab;
  int M = 0, n = 0, N = 0, L = 0, nup = 0, p = 0;
  DevArray<double> off, w, G, T, Yup;
  DevArray<double4> offup;
  // per-matvec work buffers
  DevArray<float4> src32;
  DevArray<double2> src64;
  DevArray<double> far_part, near_part, coef, qup, selfo, mom;
  int nchunks = 1, spc = 1, tpt = 2;
  // GMRES
  int restart = 50, max_iter = 500;
  double tol = 1e-8;
  DevArray<double> V, x, r, rhs, tmp, d, partial, h, ycoef;
  int nb_dots = 128;
};

struct LcpState;
void lcp_release(LcpState* st);

struct pqn_ctx_impl {
  pqn_config_desc cfg{};
  int M = 0;
  double a = 1.0, mu = 1.0;
  std::vector<double> centers, axes;
  bool has_axes = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  Level hi, lo;
  bool has_lo = false;
  // configuration-dependent tables shared by both levels
  DevArray<double> ctr, dax;
  DevArray<unsigned char> cls;
  DevArray<int> partners, npart, near_list;
  int max_slots = 0, n_near = 0;
  std::vector<int> h_partners, h_npart;
  DevArray<double> FT, UO;
  // profiling of far launches
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
  size_t ev_used = 0;
  // counters of the current call
  int n_matvec = 0, n_far = 0;
  // LCP workspaces (lcp.hip)
  struct LcpState* lcp = nullptr;
  ~pqn_ctx_impl();

  Level& level(int fidelity) {
    if (fidelity == PQN_LOFI) {
      if (!has_lo) throw Error(PQN_ERR_STATE, "no low-fidelity grid in this context");
      return lo;
    }
    if (fidelity != PQN_HIFI) throw Error(PQN_ERR_INVALID, "fidelity must be PQN_HIFI or PQN_LOFI");
    return hi;
  }
  void setup_level(Level& lv, int nt, int np, double tol);
  void set_configuration(const double* c, const double* ax);
  void apply_operator(Level& lv, int precision, const double* q, double* y);
  // GMRES on (1/2 + D + P) x = rhs (device arrays of length 3N); returns iterations
  int gmres(Level& lv, int precision, const double* rhs, double* x, double tol, double* relres, bool* conv);
  void solve(Level& lv, const double* rhs, double* x, pqn_mvp_stats* st);
  void mobility(Level& lv, const double* FT_dev, const double* axes_dev, double* UO_dev, pqn_mvp_stats* st);
  double dot_host(const double* x, const double* y, long len, Level& lv);
  void begin_far_timing();
  double end_far_timing();
};

}  // namespace bipqn

struct pqn_ctx : bipqn::pqn_ctx_impl {};
