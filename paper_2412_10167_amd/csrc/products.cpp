// Host tables of the product-arrangement analysis (Sec. "Analysis of final
// states", reactant-coordinate-based method) for J = 0 units.
//
// A point (r'_i, R'_inf, cos gamma'_n) of the product line of XY + Z is placed
// as atoms (XY centre of mass at the origin, R' along z, r' in the x-z plane),
// and the reactant Jacobi coordinates (r = B -> C, R from the BC centre of mass
// to A, their angle) are read off the positions.  The packet's function there
// is  Phi(r, R, x) = sum u[n][m][i] t_i(r) t_m(R) L_n(x)  with the sine-DVR
// functions t_i(q) = sum_k S_ki sqrt(2/L) sin(k pi (q - wall)/L) (zero outside
// the box) and the Legendre DVR functions L_n(x) = sum_j P[j][n] P~_j(x) of the
// plan's grids; for J = 0 the product-frame function is (r'R'/(rR)) Phi (the
// angular functions of both frames are the same constant, and the change of
// Jacobi vectors has unit Jacobian).  The line is stored DVR-weighted,
// sqrt(dr' w'_n) Phi'(r'_i, R'_inf, x'_n), so a channel projection is a plain sum.
#include <algorithm>
#include <cmath>
#include <vector>

#include "host_tables.h"
#include "plan.h"
#include "products.h"

namespace tdwp {

namespace {

constexpr double kPi = 3.14159265358979323846;

struct Vec3 {
  double x, y, z;
};
Vec3 operator-(Vec3 a, Vec3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
Vec3 operator*(double s, Vec3 a) { return {s * a.x, s * a.y, s * a.z}; }
Vec3 operator+(Vec3 a, Vec3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
double dot(Vec3 a, Vec3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// Sine-DVR functions t_i(q), i = 0..n-1, of a grid with wall `wall` and box length L.
void sine_functions(int n, double wall, double L, double q, double* out) {
  for (int i = 0; i < n; ++i) out[i] = 0.0;
  if (!(q > wall && q < wall + L)) return;
  const double s = std::sqrt(2.0 / (n + 1)), a = std::sqrt(2.0 / L);
  for (int k = 1; k <= n; ++k) {
    const double phi = a * std::sin(k * kPi * (q - wall) / L);
    for (int i = 0; i < n; ++i) out[i] += s * std::sin(k * kPi * (i + 1) / (n + 1)) * phi;
  }
}

}  // namespace

int build_product_tables(Plan* P) {
  const tdwp_config& c = P->cfg;
  if (c.prod_arrangement == 0) return TDWP_OK;
  if (c.prod_arrangement != 1 && c.prod_arrangement != 2) return TDWP_EINVAL;
  if (c.prod_n_r < 2 || c.prod_n_gamma < 2 || c.prod_n_r > 1024 || c.prod_n_gamma > 256)
    return TDWP_EINVAL;
  if (!(c.prod_r_min > 0) || !(c.prod_r_max > c.prod_r_min) || !(c.prod_R_inf > 0))
    return TDWP_EINVAL;
  const double mA = c.mass_A, mB = c.mass_B, mC = c.mass_C, M = mA + mB + mC;
  const bool ab = c.prod_arrangement == 1;   // AB + C, else AC + B
  const double mX = mA, mY = ab ? mB : mC, mZ = ab ? mC : mB;
  P->prod_mu = mZ * (mX + mY) / M;
  P->prod_m = mX * mY / (mX + mY);
  const int npr = c.prod_n_r, npg = c.prod_n_gamma;
  P->prod_np = npr * npg;
  P->prod_dr = (c.prod_r_max - c.prod_r_min) / (npr - 1);
  P->prod_L = (npr + 1) * P->prod_dr;
  P->prod_wall = c.prod_r_min - P->prod_dr;
  P->prod_r.resize(npr);
  for (int i = 0; i < npr; ++i) P->prod_r[i] = c.prod_r_min + i * P->prod_dr;
  gauss_legendre(npg, P->prod_x, P->prod_w);
  std::vector<double> eig;
  sine_kinetic(npr, P->prod_L, P->prod_m, c.rad_cut, P->prod_T, eig);
  P->prod_Br.resize(npr);
  for (int i = 0; i < npr; ++i) P->prod_Br[i] = 1.0 / (2.0 * P->prod_m * P->prod_r[i] * P->prod_r[i]);
  legendre_fbr_rows(npg - 1, 0, P->prod_x, P->prod_w, P->prod_P);   // rows sqrt(w') P~_j(x')
  // interpolation tables over the points p = n' * prod_n_r + i'
  const int nr = P->nr, nR = P->nR, ng = P->ng;
  P->prod_kr = (nr + 3) / 4 * 4;
  P->prod_kR = (nR + 3) / 4 * 4;
  const int np = P->prod_np;
  P->prod_wr.assign((size_t)np * P->prod_kr, 0.0);
  P->prod_wR.assign((size_t)np * P->prod_kR, 0.0);
  P->prod_wL.assign((size_t)np * ng, 0.0);
  P->prod_factor.assign(np, 0.0);
  std::vector<double> Pg;   // rows sqrt(w_n) P~_j(x_n) of the plan's gamma grid (Omega = 0)
  legendre_fbr_rows(ng - 1, 0, P->x, P->w, Pg);
  std::vector<double> one(1, 1.0), pt(1), lrow;
  for (int n = 0; n < npg; ++n) {
    const double xp = P->prod_x[n], sp = std::sqrt(std::max(1.0 - xp * xp, 0.0));
    for (int i = 0; i < npr; ++i) {
      const int p = n * npr + i;
      const double rp = P->prod_r[i], Rp = c.prod_R_inf;
      const Vec3 rhat{sp, 0.0, xp};
      const Vec3 X = -(mY / (mX + mY) * rp) * rhat;
      const Vec3 Y = (mX / (mX + mY) * rp) * rhat;
      const Vec3 Z{0.0, 0.0, Rp};
      const Vec3 A = X, B = ab ? Y : Z, C = ab ? Z : Y;
      const Vec3 rv = C - B;
      const Vec3 Rv = A - (1.0 / (mB + mC)) * (mB * B + mC * C);
      const double r = std::sqrt(dot(rv, rv)), R = std::sqrt(dot(Rv, Rv));
      double x = dot(rv, Rv) / (r * R);
      x = std::min(1.0, std::max(-1.0, x));
      sine_functions(nr, P->r_wall, P->Lr, r, P->prod_wr.data() + (size_t)p * P->prod_kr);
      sine_functions(nR, P->R_wall, P->LR, R, P->prod_wR.data() + (size_t)p * P->prod_kR);
      pt[0] = x;
      legendre_fbr_rows(ng - 1, 0, pt, one, lrow);   // P~_j(x), j = 0..ng-1
      for (int q = 0; q < ng; ++q) {
        double s = 0.0;
        for (int j = 0; j < ng; ++j) s += Pg[(size_t)j * ng + q] * lrow[j];
        P->prod_wL[(size_t)p * ng + q] = s;
      }
      P->prod_factor[p] = rp * Rp / (r * R) * std::sqrt(P->prod_dr * P->prod_w[n]);
    }
  }
  return TDWP_OK;
}

int product_channels(const Plan* P, const double* v_asym, int j, int n_states, double* energies,
                     double* chi) {
  const int n = (int)P->prod_r.size();
  if (n == 0 || !v_asym || j < 0 || n_states < 1 || n_states > n) return TDWP_EINVAL;
  std::vector<double> A(P->prod_T);
  for (int i = 0; i < n; ++i) {
    double rot = P->prod_Br[i] * (double)j * (j + 1);
    if (P->cfg.rot_cut > 0) rot = std::min(rot, P->cfg.rot_cut);
    A[(size_t)i * n + i] += v_asym[i] + rot;
  }
  std::vector<double> ev, vec;
  jacobi_eigh(n, A, ev, vec);
  for (int s = 0; s < n_states; ++s) {
    if (energies) energies[s] = ev[s];
    if (!chi) continue;
    double mx = 0.0, nrm = 0.0;
    for (int i = 0; i < n; ++i) {
      mx = std::max(mx, std::fabs(vec[(size_t)i * n + s]));
      nrm += vec[(size_t)i * n + s] * vec[(size_t)i * n + s];
    }
    double sign = 1.0;
    for (int i = 0; i < n; ++i)
      if (std::fabs(vec[(size_t)i * n + s]) > 1e-3 * mx) {
        sign = vec[(size_t)i * n + s] < 0 ? -1.0 : 1.0;
        break;
      }
    for (int i = 0; i < n; ++i) chi[(size_t)s * n + i] = vec[(size_t)i * n + s] * sign / std::sqrt(nrm);
  }
  return TDWP_OK;
}

}  // namespace tdwp
