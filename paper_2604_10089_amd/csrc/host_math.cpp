// Host-side FP64 set-up: Gauss-Legendre rules, sphere grids, spherical-harmonic
// analysis/synthesis tables and the singular self block of one sphere.
#include "common.hpp"

#include <algorithm>
#include <stdexcept>

namespace bipqn {

// Gauss-Legendre nodes/weights on [-1, 1], nodes ascending. Newton's method on
// the three-term Legendre recurrence from the Tricomi-type initial guess
// cos(pi (i - 1/4)/(n + 1/2)).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = 0.0;
      for (int k = 1; k <= n; ++k) {
        double p2 = p1;
        p1 = p0;
        p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
      }
      dp = n * (z * p0 - p1) / (z * z - 1.0);
      double dz = p0 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) {
        // one more evaluation of the derivative at the converged node
        p0 = 1.0;
        p1 = 0.0;
        for (int k = 1; k <= n; ++k) {
          double p2 = p1;
          p1 = p0;
          p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
        }
        dp = n * (z * p0 - p1) / (z * z - 1.0);
        break;
      }
    }
    double wi = 2.0 / ((1.0 - z * z) * dp * dp);
    x[n - 1 - i] = z;       // z > 0 for the largest nodes
    x[i] = -z;
    w[i] = wi;
    w[n - 1 - i] = wi;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
}

static void sh_row(int p, double ct, double st, double cp, double sp, double* out) {
  real_sh_visit(p, ct, st, cp, sp, [&](int idx, double v) { out[idx] = v; });
}

// Gauss-Legendre in cos(theta) x trapezoid in phi; node (k, l) = k*n_phi + l.
static void sphere_grid(int nt, int np, double a, std::vector<double>& off, std::vector<double>& w,
                        std::vector<double>* ct_out = nullptr, std::vector<double>* phi_out = nullptr) {
  std::vector<double> t, wt;
  gauss_legendre(nt, t, wt);
  off.resize(3 * nt * np);
  w.resize(nt * np);
  if (ct_out) ct_out->resize(nt * np);
  if (phi_out) phi_out->resize(nt * np);
  for (int k = 0; k < nt; ++k) {
    double st = std::sqrt(1.0 - t[k] * t[k]);
    for (int l = 0; l < np; ++l) {
      double ph = 2.0 * kPi * l / np;
      int i = k * np + l;
      off[3 * i + 0] = a * st * std::cos(ph);
      off[3 * i + 1] = a * st * std::sin(ph);
      off[3 * i + 2] = a * t[k];
      w[i] = a * a * wt[k] * (2.0 * kPi / np);
      if (ct_out) (*ct_out)[i] = t[k];
      if (phi_out) (*phi_out)[i] = ph;
    }
  }
}

// Self block by the rotated-pole rule. For target node x0 = (theta0, phi0) the
// sphere is re-gridded with x0 at the pole by R = Rz(phi0) Ry(theta0):
// Gauss-Legendre in theta' on [0, pi] with 3 n_theta points, trapezoid in phi'
// with 2 n_phi points from 0, weight a^2 sin(theta') w'. The density reaches
// the rotated nodes through its degree-p harmonic expansion (analysis T).
// Rows of the targets with phi index 0 are computed; every other row follows
// from the grid's rotation symmetry about z: S(R x, R y) = R S(x, y) R^T.
static void build_self_block(SphereTables& t) {
  const int n = t.n, nt = t.n_theta, np = t.n_phi, L = t.L, p = t.p;
  const double a = t.radius;
  std::vector<double> xi, wx;
  const int ntr = 3 * nt, npr = 2 * np;
  gauss_legendre(ntr, xi, wx);
  std::vector<double> loc(3 * ntr * npr), Wz(ntr * npr);
  for (int k = 0; k < ntr; ++k) {
    double th = 0.5 * kPi * (xi[k] + 1.0), wth = 0.5 * kPi * wx[k];
    for (int l = 0; l < npr; ++l) {
      double ph = 2.0 * kPi * l / npr;
      int z = k * npr + l;
      loc[3 * z + 0] = std::sin(th) * std::cos(ph);
      loc[3 * z + 1] = std::sin(th) * std::sin(ph);
      loc[3 * z + 2] = std::cos(th);
      Wz[z] = a * a * std::sin(th) * wth * (2.0 * kPi / npr);
    }
  }
  const int nz = ntr * npr;
  std::vector<double> t_gl, w_gl;
  gauss_legendre(nt, t_gl, w_gl);
  t.S.assign((size_t)9 * n * n, 0.0);
  std::vector<double> G((size_t)9 * L), Yz(L);
  // rows for phi index 0 of each theta row: Srow[k][c][d][col]
  std::vector<double> Srow((size_t)nt * 9 * n);
  for (int k = 0; k < nt; ++k) {
    const double ct0 = t_gl[k], st0 = std::sqrt(1.0 - ct0 * ct0);
    // R = Ry(theta0) (phi0 = 0): columns map local axes to global
    const double R[3][3] = {{ct0, 0.0, st0}, {0.0, 1.0, 0.0}, {-st0, 0.0, ct0}};
    const double x0[3] = {a * st0, 0.0, a * ct0};
    std::fill(G.begin(), G.end(), 0.0);
    for (int z = 0; z < nz; ++z) {
      double u[3];
      for (int c = 0; c < 3; ++c)
        u[c] = R[c][0] * loc[3 * z] + R[c][1] * loc[3 * z + 1] + R[c][2] * loc[3 * z + 2];
      double rho = std::sqrt(u[0] * u[0] + u[1] * u[1]);
      double cp = rho > 0 ? u[0] / rho : 1.0, sp = rho > 0 ? u[1] / rho : 0.0;
      double ctz = std::max(-1.0, std::min(1.0, u[2]));
      sh_row(p, ctz, rho, cp, sp, Yz.data());
      double r[3] = {x0[0] - a * u[0], x0[1] - a * u[1], x0[2] - a * u[2]};
      double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
      double rn = r[0] * u[0] + r[1] * u[1] + r[2] * u[2];
      double coef = Wz[z] * (3.0 / (4.0 * kPi)) * rn / (r2 * r2 * std::sqrt(r2));
      for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) {
          double kcd = coef * r[c] * r[d];
          double* g = &G[(size_t)(c * 3 + d) * L];
          for (int q = 0; q < L; ++q) g[q] += kcd * Yz[q];
        }
    }
    // G (9 x L) times analysis T (L x n)
    for (int cd = 0; cd < 9; ++cd) {
      double* row = &Srow[((size_t)k * 9 + cd) * n];
      for (int col = 0; col < n; ++col) row[col] = 0.0;
      for (int q = 0; q < L; ++q) {
        double g = G[(size_t)cd * L + q];
        const double* Tq = &t.T[(size_t)q * n];
        for (int col = 0; col < n; ++col) row[col] += g * Tq[col];
      }
    }
  }
  // fill all targets by rotation: target (k, s) = Rz(phi_s) applied to (k, 0)
  for (int k = 0; k < nt; ++k) {
    for (int s = 0; s < np; ++s) {
      const double ph = 2.0 * kPi * s / np, cs = std::cos(ph), sn = std::sin(ph);
      const double Rz[3][3] = {{cs, -sn, 0.0}, {sn, cs, 0.0}, {0.0, 0.0, 1.0}};
      const int i = k * np + s;
      for (int kk = 0; kk < nt; ++kk)
        for (int ll = 0; ll < np; ++ll) {
          const int col = kk * np + ll;
          const int col0 = kk * np + ((ll - s) % np + np) % np;
          double B[3][3];
          for (int c = 0; c < 3; ++c)
            for (int d = 0; d < 3; ++d) B[c][d] = Srow[((size_t)k * 9 + c * 3 + d) * n + col0];
          for (int c = 0; c < 3; ++c)
            for (int d = 0; d < 3; ++d) {
              double v = 0.0;
              for (int e = 0; e < 3; ++e)
                for (int f = 0; f < 3; ++f) v += Rz[c][e] * B[e][f] * Rz[d][f];
              t.S[((size_t)c * n + i) * 3 * n + (size_t)d * n + col] = v;
            }
        }
    }
  }
}

void coarse_sh_grid(int ntc, int npc, double a, int p, std::vector<double>& off, std::vector<double>& w,
                    std::vector<double>& Y) {
  std::vector<double> ct, ph;
  sphere_grid(ntc, npc, a, off, w, &ct, &ph);
  const int nc = ntc * npc, L = (p + 1) * (p + 1);
  Y.assign((size_t)nc * L, 0.0);
  for (int f = 0; f < nc; ++f) {
    const double st = std::sqrt(1.0 - ct[f] * ct[f]);
    sh_row(p, ct[f], st, std::cos(ph[f]), std::sin(ph[f]), &Y[(size_t)f * L]);
  }
}

std::vector<double> sh_recurrence_table(int p) {
  const int L = (p + 1) * (p + 1);
  std::vector<double> t(2 * (size_t)L, 0.0);
  for (int m = 0; m <= p; ++m) {
    if (m > 0) t[2 * sh_index(m, m, 0)] = -std::sqrt((2.0 * m + 1.0) / (2.0 * m));
    for (int l = m + 1; l <= p; ++l) {
      const int s = sh_index(l, m, 0);
      t[2 * s] = std::sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
      t[2 * s + 1] =
          (l - 1 > m) ? std::sqrt(((double)(l - 1) * (l - 1) - (double)m * m) / (4.0 * (l - 1) * (l - 1) - 1.0)) : 0.0;
    }
  }
  return t;
}

// Grid up times finer per direction and the degree-p synthesis on it.
static void upsampled_grid(const SphereTables& t, int up, std::vector<double>& off, std::vector<double>& w,
                           std::vector<double>& Y, int& n_up) {
  const int nt = up * t.n_theta, np = up * t.n_phi;
  n_up = nt * np;
  std::vector<double> ctu, phu;
  sphere_grid(nt, np, t.radius, off, w, &ctu, &phu);
  Y.assign((size_t)n_up * t.L, 0.0);
  for (int f = 0; f < n_up; ++f) {
    double st = std::sqrt(1.0 - ctu[f] * ctu[f]);
    sh_row(t.p, ctu[f], st, std::cos(phu[f]), std::sin(phu[f]), &Y[(size_t)f * t.L]);
  }
}

void build_sphere_tables(int n_theta, int n_phi, double radius, int near_up, SphereTables& t, int close_up,
                         int far_theta) {
  if (n_theta < 2 || n_phi < 2 * n_theta - 1 || n_theta - 1 > kMaxDegree)
    throw std::runtime_error("grid must have n_theta >= 2, n_phi >= 2 n_theta - 1, degree <= 40");
  t.n_theta = n_theta;
  t.n_phi = n_phi;
  t.n = n_theta * n_phi;
  t.p = n_theta - 1;
  t.L = n_theta * n_theta;
  t.radius = radius;
  std::vector<double> ct, ph;
  sphere_grid(n_theta, n_phi, radius, t.off, t.w, &ct, &ph);
  // analysis T[q][k] = Y_q(node k) * w_unit(k)
  t.T.assign((size_t)t.L * t.n, 0.0);
  std::vector<double> Y(t.L);
  for (int k = 0; k < t.n; ++k) {
    double st = std::sqrt(1.0 - ct[k] * ct[k]);
    sh_row(t.p, ct[k], st, std::cos(ph[k]), std::sin(ph[k]), Y.data());
    double wu = t.w[k] / (radius * radius);
    for (int q = 0; q < t.L; ++q) t.T[(size_t)q * t.n + k] = Y[q] * wu;
  }
  build_self_block(t);
  // G = S (I3 x Ygrid): since T Ygrid = I (exact quadrature of orthonormal harmonics),
  // S = G (I3 x T) and the self term can act on the harmonic coefficients.
  {
    std::vector<double> Yg((size_t)t.n * t.L);
    for (int k = 0; k < t.n; ++k) {
      double st = std::sqrt(1.0 - ct[k] * ct[k]);
      sh_row(t.p, ct[k], st, std::cos(ph[k]), std::sin(ph[k]), &Yg[(size_t)k * t.L]);
    }
    const int n = t.n, L = t.L;
    t.G.assign((size_t)9 * n * L, 0.0);
    for (int r = 0; r < 3 * n; ++r)
      for (int d = 0; d < 3; ++d) {
        const double* srow = &t.S[(size_t)r * 3 * n + (size_t)d * n];
        double* grow = &t.G[(size_t)r * 3 * L + (size_t)d * L];
        for (int k = 0; k < n; ++k) {
          const double sv = srow[k];
          const double* yk = &Yg[(size_t)k * L];
          for (int l = 0; l < L; ++l) grow[l] += sv * yk[l];
        }
      }
  }
  // upsampled grid for near pairs and the synthesis matrix on it
  t.up = near_up;
  t.nt_up = near_up * n_theta;
  t.np_up = near_up * n_phi;
  upsampled_grid(t, near_up, t.off_up, t.w_up, t.Y_up, t.n_up);
  t.up2 = close_up > 0 ? close_up : 0;
  t.n_up2 = 0;
  if (t.up2 > 0) upsampled_grid(t, t.up2, t.off_up2, t.w_up2, t.Y_up2, t.n_up2);
  // coarse far-source grid: degree far_theta - 1 synthesis at its Gauss-Legendre x trapezoid nodes
  t.nc = t.Lc = 0;
  if (far_theta > 0) {
    if (far_theta > n_theta) throw std::runtime_error("the coarse far-source grid must not be finer than the grid");
    const int ntc = far_theta, npc = 2 * far_theta, pc = far_theta - 1;
    t.nc = ntc * npc;
    t.Lc = ntc * ntc;
    std::vector<double> ctc, phc;
    sphere_grid(ntc, npc, radius, t.off_c, t.w_c, &ctc, &phc);
    t.Y_c.assign((size_t)t.nc * t.Lc, 0.0);
    for (int f = 0; f < t.nc; ++f) {
      const double st = std::sqrt(1.0 - ctc[f] * ctc[f]);
      sh_row(pc, ctc[f], st, std::cos(phc[f]), std::sin(phc[f]), &t.Y_c[(size_t)f * t.Lc]);
    }
  }
  t.shab = sh_recurrence_table(t.p);
}

}  // namespace bipqn
