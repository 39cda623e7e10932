// Shared definitions of the bipqn HIP library (host and device).
#pragma once
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

namespace bipqn {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr int kMaxNear = 16;          // near partners per sphere (gap < near_gap)
constexpr int kMaxDegree = 40;        // largest spherical-harmonic degree p supported

// Index of the real harmonic (l, m, kind) in the degree-ordered basis:
// l outer; within l: m = 0, then (cos m phi, sin m phi) for m = 1..l.
__host__ __device__ inline int sh_index(int l, int m, int sinpart) {
  return l * l + (m == 0 ? 0 : 2 * m - 1 + sinpart);
}

// Orthonormal real spherical harmonics of degree <= p at the unit direction
// with cos/sin of the polar angle (ct, st) and of the azimuth (cp, sp).
// Fully normalised associated Legendre functions by the standard three-term
// recurrence in l at fixed m; azimuthal factors by the angle-addition
// recurrence. The callback receives (index, value) for every basis function,
// so device code can contract on the fly without storing (p+1)^2 values.
template <class F>
__host__ __device__ inline void real_sh_visit(int p, double ct, double st, double cp, double sp, F&& f) {
  const double inv4pi = 1.0 / (4.0 * kPi);
  double pmm = sqrt(inv4pi);             // P_0^0 normalised
  double cm = 1.0, sm = 0.0;             // cos(m phi), sin(m phi)
  for (int m = 0; m <= p; ++m) {
    if (m > 0) {
      pmm *= -sqrt((2.0 * m + 1.0) / (2.0 * m)) * st;
      double c2 = cm * cp - sm * sp;
      double s2 = sm * cp + cm * sp;
      cm = c2;
      sm = s2;
    }
    const double fac = (m == 0) ? 1.0 : sqrt(2.0);
    // l = m
    double plm2 = 0.0, plm1 = pmm;
    if (m == 0) {
      f(sh_index(m, 0, 0), plm1);
    } else {
      f(sh_index(m, m, 0), fac * plm1 * cm);
      f(sh_index(m, m, 1), fac * plm1 * sm);
    }
    for (int l = m + 1; l <= p; ++l) {
      double a = sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
      double b = (l - 1 > m) ? sqrt(((double)(l - 1) * (l - 1) - (double)m * m) / (4.0 * (l - 1) * (l - 1) - 1.0)) : 0.0;
      double pl = a * (ct * plm1 - b * plm2);
      plm2 = plm1;
      plm1 = pl;
      if (m == 0) {
        f(sh_index(l, 0, 0), pl);
      } else {
        f(sh_index(l, m, 0), fac * pl * cm);
        f(sh_index(l, m, 1), fac * pl * sm);
      }
    }
  }
}

// Host-side tables of one sphere grid (one fidelity level).
struct SphereTables {
  int n_theta = 0, n_phi = 0, n = 0, p = 0, L = 0;
  double radius = 1.0;
  std::vector<double> off;      // [n][3] node offsets from the centre
  std::vector<double> w;        // [n] quadrature weights (sum 4 pi a^2)
  std::vector<double> S;        // [3n][3n] self block, SoA rows (c*n+i), cols (d*n+k)
  std::vector<double> T;        // [L][n] analysis: coefficients = T q
  std::vector<double> G;        // [3n][3L] self block on coefficients: S = G (I3 x T)
  int up = 2, nt_up = 0, np_up = 0, n_up = 0;
  std::vector<double> off_up;   // [n_up][3] upsampled grid offsets
  std::vector<double> w_up;     // [n_up]
  std::vector<double> Y_up;     // [n_up][L] synthesis on the upsampled grid
  // finer grid of the close near pairs (gap < near_close_gap); n_up2 = 0 when unused
  int up2 = 0, n_up2 = 0;
  std::vector<double> off_up2, w_up2, Y_up2;
  // coarse far-source grid (far_theta x 2 far_theta nodes, nc of them; nc = 0 when unused):
  // the density truncated to degree Lc = far_theta^2 harmonics, synthesised there
  int nc = 0, Lc = 0;
  std::vector<double> off_c, w_c;  // [nc][3], [nc]
  std::vector<double> Y_c;         // [nc][Lc]
  std::vector<double> shab;     // [L][2] Legendre recurrence factors (sh_recurrence_table)
};

// Factors of the normalised Legendre recurrence used by real_sh_visit, one
// pair per (l, m) at slot sh_index(l, m, 0): for l > m the three-term
// coefficients (a_lm, b_lm) of P_l^m = a_lm (cos(theta) P_{l-1}^m - b_lm P_{l-2}^m);
// for l = m > 0 the order step -sqrt((2m+1)/(2m)) (P_m^m = step sin(theta) P_{m-1}^{m-1}).
std::vector<double> sh_recurrence_table(int p);

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
// Gauss-Legendre x trapezoid grid of ntc x npc nodes on a sphere of radius a: offsets [nc][3],
// weights [nc] and the real harmonics of degree <= p at the nodes [nc][(p + 1)^2].
void coarse_sh_grid(int ntc, int npc, double a, int p, std::vector<double>& off, std::vector<double>& w,
                    std::vector<double>& Y);
// close_up > 0: also the close-pair grid, close_up times finer per direction
void build_sphere_tables(int n_theta, int n_phi, double radius, int near_up, SphereTables& t, int close_up = 0,
                         int far_theta = 0);

}  // namespace bipqn
