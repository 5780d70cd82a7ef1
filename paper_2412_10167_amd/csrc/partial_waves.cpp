// Partial-wave sums of state-resolved probabilities (Sec. "Cross sections"):
// J-shifting of a computed probability curve to another total angular momentum,
// J-shifting interpolation between two computed ones (Eq.
// J-shifting-interpolation), the cumulative probability (Eq.
// cumulative-probability) and the integral cross section (Eq.
// collisional-xsection).  Host code on host arrays; the contracts are in tdwp.h.
//
// Every J-shifted curve is the computed curve read at energies moved by one
// constant, so its linear-interpolation stencil (left index and weight at each
// grid energy) depends on J and the grid only.  The cumulative sum builds the
// stencils of a J once and applies them to every final state, after summing the
// families present at that J (the shifted curve is linear in the computed one);
// ranges of final states run on host threads.
#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "../../include/tdwp.h"

namespace {

double jj1(int J) { return (double)J * (J + 1); }

bool ascending(const double* e, int n) {
  for (int i = 1; i < n; ++i)
    if (!(e[i] > e[i - 1])) return false;
  return true;
}

// Stencil of p(e_i - s) on the ascending grid e: value = p[lo] + t (p[lo+1] - p[lo]),
// with lo = n - 1, t = 0 past the top end and lo = 0, t = 0 below the bottom end
// (a curve keeps its end values outside the grid).  The read points e_i - s
// ascend with i, so one forward walk finds every cell.
struct Stencil {
  std::vector<int> lo;
  std::vector<double> t;
  void build(const double* e, int n, double s) {
    lo.resize(n);
    t.resize(n);
    int c = 0;
    for (int i = 0; i < n; ++i) {
      const double x = e[i] - s;
      if (x <= e[0]) {
        lo[i] = 0;
        t[i] = 0.0;
        continue;
      }
      if (x >= e[n - 1]) {
        lo[i] = n - 1;
        t[i] = 0.0;
        continue;
      }
      while (e[c + 1] <= x) ++c;
      lo[i] = c;
      t[i] = (x - e[c]) / (e[c + 1] - e[c]);
    }
  }
  double at(const double* p, int i) const {
    const int l = lo[i];
    return t[i] == 0.0 ? p[l] : p[l] + t[i] * (p[l + 1] - p[l]);
  }
};

// Where the curve of a total angular momentum J comes from: the computed index
// c1 with weight w1 read shifted by s1, plus c2 with weight w2 read shifted by
// -s2 (w2 = 0 for plain J-shifting from one computed J).
struct Source {
  int c1, c2;
  double w1, w2, s1, s2;
};

Source source_of(int J, const int* Jc, int n_calc, const double* B) {
  Source src{0, 0, 1.0, 0.0, 0.0, 0.0};
  if (J <= Jc[0]) {   // below (or at) the first computed J: shift the first one down
    src.s1 = B[0] * (jj1(J) - jj1(Jc[0]));
    return src;
  }
  if (J >= Jc[n_calc - 1]) {   // at or beyond the last computed J
    src.c1 = src.c2 = n_calc - 1;
    src.s1 = B[n_calc - 1] * (jj1(J) - jj1(Jc[n_calc - 1]));
    return src;
  }
  int c = 0;
  while (Jc[c + 1] < J) ++c;
  const int J1 = Jc[c], J2 = Jc[c + 1];
  src.c1 = c;
  src.c2 = c + 1;
  if (J == J2) {
    src.c1 = c + 1;
    return src;
  }
  src.w2 = (double)(J - J1) / (J2 - J1);
  src.w1 = 1.0 - src.w2;
  src.s1 = B[c] * (jj1(J) - jj1(J1));
  src.s2 = B[c] * (jj1(J2) - jj1(J));
  return src;
}

}  // namespace

extern "C" {

int tdwp_jshift(const double* p_ref, const double* e, int n_e, int J_ref, double B, int J,
                double* out) {
  if (!p_ref || !e || !out || n_e < 1 || J_ref < 0 || J < 0 || !(B >= 0.0) || !ascending(e, n_e))
    return TDWP_EINVAL;
  Stencil st;
  st.build(e, n_e, B * (jj1(J) - jj1(J_ref)));
  for (int i = 0; i < n_e; ++i) out[i] = st.at(p_ref, i);
  return TDWP_OK;
}

int tdwp_jshift_interpolate(const double* p1, const double* p2, const double* e, int n_e, int J1,
                            int J2, double B, int J, double* out) {
  if (!p1 || !p2 || !e || !out || n_e < 1 || J1 < 0 || J2 <= J1 || J < J1 || J > J2 ||
      !(B >= 0.0) || !ascending(e, n_e))
    return TDWP_EINVAL;
  const int Jc[2] = {J1, J2};
  const double Bc[2] = {B, B};
  const Source s = source_of(J, Jc, 2, Bc);
  Stencil a, b;
  a.build(e, n_e, s.s1);
  b.build(e, n_e, -s.s2);
  const double* pc[2] = {p1, p2};
  for (int i = 0; i < n_e; ++i) {
    double v = s.w1 * a.at(pc[s.c1], i);
    if (s.w2 != 0.0) v += s.w2 * b.at(pc[s.c2], i);
    out[i] = v;
  }
  return TDWP_OK;
}

int tdwp_cumulative_probability(const int* J_calc, const double* B, int n_calc, const double* p,
                                int n_fam, const int* fam_jmin, int n_f, const double* e, int n_e,
                                int J_max, double* c_out) {
  if (!J_calc || !B || !p || !e || !c_out || n_calc < 1 || n_fam < 1 || n_f < 1 || n_e < 1 ||
      J_max < 0 || !ascending(e, n_e))
    return TDWP_EINVAL;
  for (int c = 0; c < n_calc; ++c)
    if (J_calc[c] < 0 || (c && J_calc[c] <= J_calc[c - 1]) || !(B[c] >= 0.0)) return TDWP_EINVAL;
  if (fam_jmin)
    for (int f = 0; f < n_fam; ++f)
      if (fam_jmin[f] < 0) return TDWP_EINVAL;
  // The J-shifted curve is linear in the computed one, so the families present
  // at a J are summed before shifting.  Present at J is every family whose
  // smallest J is <= J: level q sums the families of the q+1 lowest distinct
  // smallest-J values.  The levels of a computed J are built in one of two
  // slots when an interval first needs them; the computed index needed rises
  // with J, so each computed J is summed once and p is read once.
  std::vector<int> jmin(n_fam, 0), order(n_fam);
  if (fam_jmin) jmin.assign(fam_jmin, fam_jmin + n_fam);
  for (int k = 0; k < n_fam; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return jmin[x] < jmin[y]; });
  std::vector<int> level_j, level_end;   // smallest J of level q; its families order[0, end)
  for (int k = 0; k < n_fam; ++k) {
    if (!level_j.empty() && jmin[order[k]] == level_j.back()) {
      level_end.back() = k + 1;
    } else {
      level_j.push_back(jmin[order[k]]);
      level_end.push_back(k + 1);
    }
  }
  const int n_lev = (int)level_j.size();
  const size_t row = (size_t)n_e, per_fam = (size_t)n_f * row, per_c = (size_t)n_fam * per_fam;
  // Final states [f0, f1) of the sum: independent of every other final state,
  // so ranges of them run on host threads with results identical to one thread.
  auto run = [&](int f0, int f1) {
    const size_t nfr = (size_t)(f1 - f0) * row;   // values of one level for the range
    std::vector<double> slot_buf[2];
    int slot_c[2] = {-1, -1};
    for (auto& v : slot_buf) v.resize((size_t)n_lev * nfr);
    auto levels_of = [&](int c, int keep) -> const double* {
      for (int k = 0; k < 2; ++k)
        if (slot_c[k] == c) return slot_buf[k].data();
      const int k = (slot_c[0] == keep) ? 1 : 0;
      double* dst = slot_buf[k].data();
      int fam = 0;
      for (int q = 0; q < n_lev; ++q) {
        double* lv = dst + (size_t)q * nfr;
        if (q) std::copy(lv - nfr, lv, lv);
        else std::fill(lv, lv + nfr, 0.0);
        for (; fam < level_end[q]; ++fam) {
          const double* src = p + (size_t)c * per_c + (size_t)order[fam] * per_fam + (size_t)f0 * row;
          for (size_t x = 0; x < nfr; ++x) lv[x] += src[x];
        }
      }
      slot_c[k] = c;
      return dst;
    };
    std::fill(c_out + (size_t)f0 * row, c_out + (size_t)f1 * row, 0.0);
    Stencil a, b;
    int lev = -1;
    for (int J = 0; J <= J_max; ++J) {
      while (lev + 1 < n_lev && level_j[lev + 1] <= J) ++lev;
      if (lev < 0) continue;   // no family has a state at this J
      const Source s = source_of(J, J_calc, n_calc, B);
      const double* S1 = levels_of(s.c1, s.c2) + (size_t)lev * nfr;
      const double* S2 = levels_of(s.c2, s.c1) + (size_t)lev * nfr;
      a.build(e, n_e, s.s1);
      if (s.w2 != 0.0) b.build(e, n_e, -s.s2);
      const double g = 2.0 * J + 1.0;
      const double g1 = g * s.w1, g2 = g * s.w2;
      for (int f = f0; f < f1; ++f) {
        const double* p1 = S1 + (size_t)(f - f0) * row;
        const double* p2 = S2 + (size_t)(f - f0) * row;
        double* out = c_out + (size_t)f * row;
        if (s.w2 == 0.0) {
          for (int i = 0; i < n_e; ++i) out[i] += g1 * a.at(p1, i);
        } else {
          for (int i = 0; i < n_e; ++i) out[i] += g1 * a.at(p1, i) + g2 * b.at(p2, i);
        }
      }
    }
  };
  // one thread per 16 final states at least, up to the host's cores (at most 16)
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const int n_thr = (int)std::min<long>((long)hw, std::max<long>(1, (long)n_f / 16));
  if (n_thr == 1) {
    run(0, n_f);
  } else {
    std::vector<std::thread> pool;
    for (int t = 0; t < n_thr; ++t) {
      const int f0 = (int)((long)n_f * t / n_thr), f1 = (int)((long)n_f * (t + 1) / n_thr);
      pool.emplace_back(run, f0, f1);
    }
    for (auto& th : pool) th.join();
  }
  return TDWP_OK;
}

int tdwp_cross_section(const double* c, int n_f, const double* e_col, int n_e, double mu, int j0,
                       double* sigma) {
  if (!c || !e_col || !sigma || n_f < 1 || n_e < 1 || !(mu > 0.0) || j0 < 0) return TDWP_EINVAL;
  for (int i = 0; i < n_e; ++i)
    if (!(e_col[i] > 0.0)) return TDWP_EINVAL;
  const double pi = std::acos(-1.0);
  for (int i = 0; i < n_e; ++i) {
    const double k2 = 2.0 * mu * e_col[i];   // K0^2 at this collision energy, hbar = 1
    const double scale = pi / (k2 * (2.0 * j0 + 1.0));
    for (int f = 0; f < n_f; ++f) sigma[(size_t)f * n_e + i] = scale * c[(size_t)f * n_e + i];
  }
  return TDWP_OK;
}

int tdwp_fit_jshift_b(const double* p1, const double* p2, const double* e, int n_e, int J1, int J2,
                      double B_max, double* B_out) {
  if (!p1 || !p2 || !e || !B_out || n_e < 2 || J1 < 0 || J2 <= J1 || !(B_max > 0.0) ||
      !ascending(e, n_e))
    return TDWP_EINVAL;
  const double d = jj1(J2) - jj1(J1);
  Stencil st;
  // squared misfit between the J1 curve shifted to J2 and the computed J2 curve
  auto cost = [&](double Bv) {
    st.build(e, n_e, Bv * d);
    double sum = 0.0;
    for (int i = 0; i < n_e; ++i) {
      const double r = st.at(p1, i) - p2[i];
      sum += r * r;
    }
    return sum;
  };
  const int n_scan = 512;
  int best = 0;
  double best_c = cost(0.0);
  for (int k = 1; k <= n_scan; ++k) {
    const double ck = cost(B_max * k / n_scan);
    if (ck < best_c) {
      best_c = ck;
      best = k;
    }
  }
  // golden-section search over the two scan cells around the best scan point
  double lo = B_max * (best > 0 ? best - 1 : 0) / n_scan;
  double hi = B_max * (best < n_scan ? best + 1 : n_scan) / n_scan;
  const double g = 0.5 * (std::sqrt(5.0) - 1.0);
  double x1 = hi - g * (hi - lo), x2 = lo + g * (hi - lo);
  double f1 = cost(x1), f2 = cost(x2);
  while (hi - lo > 1e-13 * B_max) {
    if (f1 <= f2) {
      hi = x2;
      x2 = x1;
      f2 = f1;
      x1 = hi - g * (hi - lo);
      f1 = cost(x1);
    } else {
      lo = x1;
      x1 = x2;
      f1 = f2;
      x2 = lo + g * (hi - lo);
      f2 = cost(x2);
    }
  }
  double Bf = 0.5 * (lo + hi);
  if (cost(Bf) > best_c) Bf = B_max * best / n_scan;
  *B_out = Bf;
  return TDWP_OK;
}

}  // extern "C"
