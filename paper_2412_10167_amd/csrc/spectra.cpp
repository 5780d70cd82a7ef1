// Energy content and photodissociation cross section from the autocorrelation
// of a photodissociation packet (Eqs. fourier-transform, chebyshev-transform,
// spectrum; c_k of Eq. chebyshev-expansion-constants, hbar = 1).  Host code on
// host arrays; the contracts are in tdwp.h.
//
// With theta = arccos E_s, Re c_k(H_s, E) = (2 - delta_k0) cos(k theta) / (dE sin theta).
// cos(k theta) follows the rotation (cos, sin)(k+1) = (cos, sin)(k) rotated by
// theta, restarted from the library cos and sin every kAnchor terms so that its
// rounding stays below kAnchor ulps.  Ranges of energies run on host threads.
#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "../../include/tdwp.h"

namespace {

constexpr long kAnchor = 256;
constexpr double kCau = 137.035999084;   // speed of light, atomic units (CODATA 2018)

// sum_k Re c_k(H_s, E) C_k at one energy; false outside the open spectral range
bool transform_at(const double* C, long n_k, double e_min, double e_max, double E, double* out) {
  const double E0 = 0.5 * (e_max + e_min), dE = 0.5 * (e_max - e_min);
  const double x = (E - E0) / dE;
  if (!(x > -1.0 && x < 1.0)) return false;
  const double th = std::acos(x), ct = std::cos(th), st = std::sin(th);
  double sum = 0.0, c = 1.0, s = 0.0;
  for (long k = 0; k < n_k; ++k) {
    if (k % kAnchor == 0) {
      c = std::cos((double)k * th);
      s = std::sin((double)k * th);
    }
    sum += (k ? 2.0 : 1.0) * c * C[k];
    const double cn = c * ct - s * st;
    s = s * ct + c * st;
    c = cn;
  }
  *out = sum / (dE * st);
  return true;
}

bool range_ok(long n_k, double e_min, double e_max, int n_e) {
  return n_k >= 1 && n_e >= 1 && std::isfinite(e_min) && std::isfinite(e_max) && e_max > e_min;
}

// f(i) for i in [0, n): ranges of energies on host threads (one per 64 energies at
// least, at most 16); every energy's sum is independent, so the results do not
// depend on the split.
template <class F>
void for_energies(int n, F&& f) {
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const int n_thr = (int)std::min<long>((long)hw, std::max<long>(1, (long)n / 64));
  if (n_thr == 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  std::vector<std::thread> pool;
  for (int t = 0; t < n_thr; ++t) {
    const int i0 = (int)((long)n * t / n_thr), i1 = (int)((long)n * (t + 1) / n_thr);
    pool.emplace_back([&f, i0, i1] {
      for (int i = i0; i < i1; ++i) f(i);
    });
  }
  for (auto& th : pool) th.join();
}

bool inside(double e_min, double e_max, double E) {
  const double x = (E - 0.5 * (e_max + e_min)) / (0.5 * (e_max - e_min));
  return x > -1.0 && x < 1.0;
}

}  // namespace

extern "C" {

int tdwp_energy_content(const double* C, long n_k, double e_min, double e_max, const double* E,
                        int n_e, double* a0) {
  if (!C || !E || !a0 || !range_ok(n_k, e_min, e_max, n_e)) return TDWP_EINVAL;
  for (int i = 0; i < n_e; ++i)
    if (!inside(e_min, e_max, E[i])) return TDWP_EINVAL;
  const double pi = std::acos(-1.0);
  for_energies(n_e, [&](int i) {
    double v = 0.0;
    transform_at(C, n_k, e_min, e_max, E[i], &v);   // inside the range: checked above
    a0[i] = v / pi;
  });
  return TDWP_OK;
}

int tdwp_photo_cross_section(const double* C, long n_k, double e_min, double e_max, double E_i,
                             const double* hnu, int n_e, double* sigma) {
  if (!C || !hnu || !sigma || !range_ok(n_k, e_min, e_max, n_e) || !std::isfinite(E_i))
    return TDWP_EINVAL;
  for (int i = 0; i < n_e; ++i)
    if (!(hnu[i] > 0.0) || !inside(e_min, e_max, E_i + hnu[i])) return TDWP_EINVAL;
  const double pi = std::acos(-1.0);
  const double A = 4.0 * pi / kCau;   // 1/(hbar^2 eps0 c), hbar = 1, eps0 = 1/(4 pi)
  for_energies(n_e, [&](int i) {
    double v = 0.0;
    transform_at(C, n_k, e_min, e_max, E_i + hnu[i], &v);   // inside the range: checked above
    sigma[i] = A * hnu[i] / (2.0 * pi) * 2.0 * v;
  });
  return TDWP_OK;
}

}  // extern "C"
