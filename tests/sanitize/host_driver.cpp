// Exercises the library's host-only C++ (the table builders and the host C-ABI
// calls of partial-wave sums and photodissociation spectra) in a program built
// with AddressSanitizer and UndefinedBehaviorSanitizer: every call with valid
// arguments at workload-like sizes, and the argument checks with invalid ones.
// Exit status 0 when every check holds; a sanitizer report aborts the run.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../include/tdwp.h"
#include "../../paper_2412_10167_amd/csrc/host_tables.h"

static int failures = 0;
static void check(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "check failed: %s\n", what);
    ++failures;
  }
}

int main() {
  using namespace tdwp;
  // Gauss-Legendre rule: weights sum to 2, nodes ascending and symmetric
  for (int n : {1, 2, 9, 48, 96}) {
    std::vector<double> x, w;
    gauss_legendre(n, x, w);
    double s = 0.0;
    for (double v : w) s += v;
    check(std::fabs(s - 2.0) < 1e-12, "Gauss-Legendre weights sum to 2");
    for (int i = 0; i < n; ++i) check(std::fabs(x[i] + x[n - 1 - i]) < 1e-13, "symmetric nodes");
    // FBR rows of every helicity: orthonormal
    for (int om : {0, 1, n > 3 ? 3 : 0}) {
      if (om > n - 1) continue;
      std::vector<double> P;
      legendre_fbr_rows(n - 1, om, x, w, P);
      const int rows = n - om;
      for (int a = 0; a < rows; ++a)
        for (int b = 0; b < rows; ++b) {
          double d = 0.0;
          for (int q = 0; q < n; ++q) d += P[(size_t)a * n + q] * P[(size_t)b * n + q];
          check(std::fabs(d - (a == b ? 1.0 : 0.0)) < 1e-10, "orthonormal FBR rows");
        }
    }
  }
  // sine-DVR kinetic matrix, capped and uncapped; its eigen-decomposition
  for (int n : {4, 33, 128}) {
    for (double cap : {0.0, 0.05}) {
      std::vector<double> T, eig;
      sine_kinetic(n, 8.0, 1800.0, cap, T, eig);
      std::vector<double> a(T), ev, vec;
      jacobi_eigh(n, a, ev, vec);
      for (int k = 0; k < n; ++k) {
        double r = 0.0;   // residual of T v_k = ev_k v_k
        for (int i = 0; i < n; ++i) {
          double s = 0.0;
          for (int j = 0; j < n; ++j) s += T[(size_t)i * n + j] * vec[(size_t)j * n + k];
          r = std::fmax(r, std::fabs(s - ev[k] * vec[(size_t)i * n + k]));
        }
        check(r < 1e-10, "Jacobi eigenpairs");
      }
    }
  }
  // l^2 blocks over helicity ranges
  for (int J : {0, 4, 40})
    for (int j : {0, 3, 47})
      for (int lo = 0; lo <= 1; ++lo) {
        const int hi = std::min(J, j);
        if (hi < lo) continue;
        std::vector<double> L;
        ell2_block(J, j, lo, hi, L);
        check(L.size() == (size_t)(hi - lo + 1) * (hi - lo + 1), "l^2 block size");
      }
  // partial-wave sums
  const int ne = 200;
  std::vector<double> e(ne), p1(ne), p2(ne), out(ne);
  for (int i = 0; i < ne; ++i) {
    e[i] = 0.01 + 0.0002 * i;
    p1[i] = 0.5 * (1.0 + std::tanh((e[i] - 0.03) / 0.004));
    p2[i] = 0.5 * (1.0 + std::tanh((e[i] - 0.032) / 0.004));
  }
  check(tdwp_jshift(p1.data(), e.data(), ne, 0, 1e-4, 6, out.data()) == TDWP_OK, "jshift");
  check(tdwp_jshift_interpolate(p1.data(), p2.data(), e.data(), ne, 0, 10, 1e-4, 4, out.data()) == TDWP_OK,
        "jshift interpolate");
  double b = 0.0;
  check(tdwp_fit_jshift_b(p1.data(), p2.data(), e.data(), ne, 0, 10, 1e-3, &b) == TDWP_OK, "fit B");
  const int Jc[3] = {0, 10, 20};
  const double Bc[3] = {1e-4, 1e-4, 1e-4};
  const int nfam = 2, nf = 3;
  std::vector<double> p((size_t)3 * nfam * nf * ne);
  for (size_t q = 0; q < p.size(); ++q) p[q] = p1[q % ne] * (1.0 + 0.1 * (double)(q / ne % 5));
  const int fam_jmin[2] = {0, 1};
  std::vector<double> c((size_t)nf * ne), sigma((size_t)nf * ne);
  check(tdwp_cumulative_probability(Jc, Bc, 3, p.data(), nfam, fam_jmin, nf, e.data(), ne, 30, c.data()) ==
            TDWP_OK, "cumulative probability");
  check(tdwp_cross_section(c.data(), nf, e.data(), ne, 1200.0, 0, sigma.data()) == TDWP_OK, "cross section");
  // photodissociation spectra from an autocorrelation series
  const long nk = 3000;
  std::vector<double> C(2 * nk), a0(ne), hnu(ne), sg(ne);
  for (long k = 0; k < nk; ++k) {
    C[2 * k] = std::cos(0.1 * k) * std::exp(-1e-3 * k);
    C[2 * k + 1] = std::sin(0.1 * k) * std::exp(-1e-3 * k);
  }
  for (int i = 0; i < ne; ++i) hnu[i] = 0.05 + 0.001 * i;
  check(tdwp_energy_content(C.data(), nk, -0.2, 0.8, e.data(), ne, a0.data()) == TDWP_OK, "energy content");
  check(tdwp_photo_cross_section(C.data(), nk, -0.2, 0.8, -0.1, hnu.data(), ne, sg.data()) == TDWP_OK,
        "photo cross section");
  // argument checks
  check(tdwp_jshift(nullptr, e.data(), ne, 0, 1e-4, 6, out.data()) == TDWP_EINVAL, "jshift NULL");
  check(tdwp_jshift(p1.data(), e.data(), 0, 0, 1e-4, 6, out.data()) == TDWP_EINVAL, "jshift n_e");
  check(tdwp_jshift_interpolate(p1.data(), p2.data(), e.data(), ne, 10, 0, 1e-4, 4, out.data()) == TDWP_EINVAL,
        "interpolate J order");
  const int Jbad[3] = {0, 20, 10};
  check(tdwp_cumulative_probability(Jbad, Bc, 3, p.data(), nfam, fam_jmin, nf, e.data(), ne, 30, c.data()) ==
            TDWP_EINVAL, "cumulative probability J order");
  check(tdwp_cross_section(c.data(), nf, e.data(), ne, -1.0, 0, sigma.data()) == TDWP_EINVAL, "cross section mu");
  check(tdwp_energy_content(C.data(), nk, 0.8, -0.2, e.data(), ne, a0.data()) == TDWP_EINVAL, "bounds order");
  check(tdwp_photo_cross_section(C.data(), 0, -0.2, 0.8, -0.1, hnu.data(), ne, sg.data()) == TDWP_EINVAL,
        "photo n_k");
  if (failures) return 1;
  std::printf("host driver: all checks passed\n");
  return 0;
}
