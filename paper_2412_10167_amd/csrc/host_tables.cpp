// Plan tables built on the host once per plan (see host_tables.h).
#include "host_tables.h"

#include <algorithm>
#include <cmath>

namespace tdwp {

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const double pi = std::acos(-1.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    // Newton iteration on P_n from the asymptotic guess of the i-th largest root.
    double z = std::cos(pi * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
    }
    double wt = 2.0 / ((1.0 - z * z) * dp * dp);
    // descending roots z -> ascending order
    x[n - 1 - i] = z;
    x[i] = -z;
    w[n - 1 - i] = wt;
    w[i] = wt;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
}

void legendre_fbr_rows(int jmax, int omega, const std::vector<double>& x,
                       const std::vector<double>& w, std::vector<double>& out) {
  const int n = (int)x.size();
  const int nj = jmax - omega + 1;
  out.assign((size_t)nj * n, 0.0);
  for (int q = 0; q < n; ++q) {
    const double z = x[q];
    const double s2 = 1.0 - z * z;
    // Normalised sectoral start: Pt_{0,0} = 1/sqrt(2),
    // Pt_{m,m} = Pt_{m-1,m-1} * sqrt((2m+1)/(2m)) * sqrt(1 - z^2).
    double pmm = std::sqrt(0.5);
    for (int m = 1; m <= omega; ++m) pmm *= std::sqrt((2.0 * m + 1.0) / (2.0 * m) * s2);
    double pm2 = 0.0, pm1 = pmm;
    out[(size_t)0 * n + q] = pmm;
    for (int j = omega + 1; j <= jmax; ++j) {
      // Pt_j = a_j (z Pt_{j-1} - Pt_{j-2} / a_{j-1}),  a_j = sqrt((4j^2 - 1)/(j^2 - m^2))
      double aj = std::sqrt((4.0 * j * j - 1.0) / ((double)j * j - (double)omega * omega));
      double pj;
      if (j == omega + 1) {
        pj = aj * z * pm1;
      } else {
        double ajm1 = std::sqrt((4.0 * (j - 1) * (j - 1) - 1.0) /
                                ((double)(j - 1) * (j - 1) - (double)omega * omega));
        pj = aj * (z * pm1 - pm2 / ajm1);
      }
      out[(size_t)(j - omega) * n + q] = pj;
      pm2 = pm1;
      pm1 = pj;
    }
  }
  for (int r = 0; r < nj; ++r)
    for (int q = 0; q < n; ++q) out[(size_t)r * n + q] *= std::sqrt(w[q]);
}

void sine_kinetic(int n, double length, double mass, double cap, std::vector<double>& T,
                  std::vector<double>& eig) {
  const double pi = std::acos(-1.0);
  std::vector<double> S((size_t)n * n);
  const double c = std::sqrt(2.0 / (n + 1));
  for (int a = 1; a <= n; ++a)
    for (int i = 1; i <= n; ++i) {
      long prod = (long)a * i % (2L * (n + 1));  // exact argument reduction of a i pi / (n+1)
      S[(size_t)(a - 1) * n + (i - 1)] = c * std::sin(pi * (double)prod / (n + 1));
    }
  eig.resize(n);
  for (int a = 1; a <= n; ++a) {
    double k = pi * a / length;
    double e = k * k / (2.0 * mass);
    if (cap > 0.0) e = std::min(e, cap);
    eig[a - 1] = e;
  }
  T.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) {
      double s = 0.0;
      for (int a = 0; a < n; ++a) s += S[(size_t)a * n + i] * eig[a] * S[(size_t)a * n + j];
      T[(size_t)i * n + j] = s;
      T[(size_t)j * n + i] = s;
    }
}

void jacobi_eigh(int n, std::vector<double>& a, std::vector<double>& evals,
                 std::vector<double>& evecs) {
  evecs.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) evecs[(size_t)i * n + i] = 1.0;
  auto A = [&](int i, int j) -> double& { return a[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double v = A(i, j) * A(i, j);
        tot += v;
        if (i != j) off += v;
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A(p, q);
        if (apq == 0.0) continue;
        double app = A(p, p), aqq = A(q, q);
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) {  // columns p, q
          double akp = A(k, p), akq = A(k, q);
          A(k, p) = cs * akp - sn * akq;
          A(k, q) = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          double apk = A(p, k), aqk = A(q, k);
          A(p, k) = cs * apk - sn * aqk;
          A(q, k) = sn * apk + cs * aqk;
        }
        A(p, q) = A(q, p) = 0.0;
        for (int k = 0; k < n; ++k) {
          double vkp = evecs[(size_t)k * n + p], vkq = evecs[(size_t)k * n + q];
          evecs[(size_t)k * n + p] = cs * vkp - sn * vkq;
          evecs[(size_t)k * n + q] = sn * vkp + cs * vkq;
        }
      }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return A(x, x) < A(y, y); });
  evals.resize(n);
  std::vector<double> v2((size_t)n * n);
  for (int k = 0; k < n; ++k) {
    evals[k] = A(idx[k], idx[k]);
    for (int i = 0; i < n; ++i) v2[(size_t)i * n + k] = evecs[(size_t)i * n + idx[k]];
  }
  evecs.swap(v2);
}

void ell2_block(int J, int j, int om_lo, int om_hi, std::vector<double>& L) {
  const int n = om_hi - om_lo + 1;
  L.assign((size_t)n * n, 0.0);
  auto lam = [](int a, int o) {
    double v = (double)a * (a + 1) - (double)o * (o + 1);
    return v > 0 ? std::sqrt(v) : 0.0;
  };
  for (int k = 0; k < n; ++k) {
    int o = om_lo + k;
    L[(size_t)k * n + k] = (double)J * (J + 1) + (double)j * (j + 1) - 2.0 * o * o;
    if (k + 1 < n) {
      double c = -lam(J, o) * lam(j, o) * (o == 0 ? std::sqrt(2.0) : 1.0);
      L[(size_t)k * n + k + 1] = c;
      L[(size_t)(k + 1) * n + k] = c;
    }
  }
}

}  // namespace tdwp
