// Initial photodissociation packet (Eq. initial-photo-wvp): the transition
// dipole times the initial bound state, projected on the helicity functions
// W^{JMp}_Omega of a unit's final J (Eq. angular-functions, Lambda = 0 states
// with sigma = +1).  The transition operator is
//   d.e = sum_pq (-1)^p (e)_{-p} D^{1*}_{pq}(Euler angles) d_q(r, R, gamma),
// and the Euler-angle integral <W_Omega| D^{1*}_{pq} |W_Omega_i> reduces, for
// each signed helicity of the two functions, to
//   8 pi^2 / (2J + 1) <1 p J_i M_i | J M> <1 q J_i Omega_i' | J Omega'>.
// The projection is local in (r, R, gamma): every helicity block of the packet
// is a sum of dipole components times bound-state blocks, point by point.
// Built once per packet on the host and installed as a photodissociation
// packet (its autocorrelation is formed along the propagation).
#include <cmath>
#include <vector>

#include "plan.h"

namespace {

// <1 m1 j m2 | J M> for rank one coupled to integer j, from the closed-form
// j x 1 tables <j m2 1 m1 | J M> and the exchange phase (-1)^(1 + j - J).
double cg_rank1(int m1, int j, int m2, int J, int M) {
  if (m1 < -1 || m1 > 1 || m1 + m2 != M || std::abs(m2) > j || std::abs(M) > J) return 0.0;
  const double jj = j, MM = M;
  double v = 0.0;
  if (J == j + 1) {
    if (m1 == 1) v = std::sqrt((jj + MM) * (jj + MM + 1) / ((2 * jj + 1) * (2 * jj + 2)));
    else if (m1 == 0) v = std::sqrt((jj - MM + 1) * (jj + MM + 1) / ((2 * jj + 1) * (jj + 1)));
    else v = std::sqrt((jj - MM) * (jj - MM + 1) / ((2 * jj + 1) * (2 * jj + 2)));
  } else if (J == j && j > 0) {
    if (m1 == 1) v = -std::sqrt((jj + MM) * (jj - MM + 1) / (2 * jj * (jj + 1)));
    else if (m1 == 0) v = MM / std::sqrt(jj * (jj + 1));
    else v = std::sqrt((jj - MM) * (jj + MM + 1) / (2 * jj * (jj + 1)));
  } else if (J == j - 1 && j > 0) {
    if (m1 == 1) v = std::sqrt((jj - MM) * (jj - MM + 1) / (2 * jj * (2 * jj + 1)));
    else if (m1 == 0) v = -std::sqrt((jj - MM) * (jj + MM) / (jj * (2 * jj + 1)));
    else v = std::sqrt((jj + MM + 1) * (jj + MM) / (2 * jj * (2 * jj + 1)));
  } else {
    return 0.0;
  }
  return ((1 + j - J) % 2 == 0) ? v : -v;
}

double w_norm(int J, int om) {
  const double pi = 3.14159265358979323846;
  return std::sqrt((2.0 * J + 1.0) / (16.0 * pi * pi * (om == 0 ? 2.0 : 1.0)));
}

// <W^{J M par}_om | D^{1*}_{pol q} | W^{Ji Mi pari}_omi> over the Euler angles.
double coupling(int J, int M, int par, int Ji, int Mi, int pari, int om, int omi, int q, int pol) {
  const double pi = 3.14159265358979323846;
  const double cm = cg_rank1(pol, Ji, Mi, J, M);
  if (cm == 0.0) return 0.0;
  double sum = 0.0;
  for (int s : {1, -1}) {
    const double fs = s > 0 ? 1.0 : par * (((J + om) % 2) ? -1.0 : 1.0);
    for (int si : {1, -1}) {
      const double fi = si > 0 ? 1.0 : pari * (((Ji + omi) % 2) ? -1.0 : 1.0);
      sum += fs * fi * cg_rank1(q, Ji, si * omi, J, s * om);
    }
  }
  return w_norm(J, om) * w_norm(Ji, omi) * 8.0 * pi * pi / (2.0 * J + 1.0) * cm * sum;
}

}  // namespace

extern "C" int tdwp_photo_packet(tdwp_plan_t p, int unit, int slot, int elec, int J_i, int M_i,
                                 int p_i, int om_lo_i, int n_om_i, const double* bound,
                                 const double* dip, int pol) {
  if (!p || !bound || !dip) return TDWP_EINVAL;
  if (unit < 0 || unit >= (int)p->units.size()) return TDWP_EINVAL;
  if (elec < 0 || elec >= p->ne || J_i < 0 || std::abs(M_i) > J_i || (p_i != 1 && p_i != -1))
    return TDWP_EINVAL;
  if (pol < -1 || pol > 1 || n_om_i < 1 || om_lo_i < 0 || om_lo_i + n_om_i - 1 > J_i)
    return TDWP_EINVAL;
  // an Omega_i = 0 component exists only for p_i (-1)^J_i = +1 (Eq. angular-functions)
  if (om_lo_i == 0 && p_i * ((J_i % 2) ? -1 : 1) != 1) return TDWP_EINVAL;
  const tdwp::UnitInfo& U = p->units[unit];
  const int M = M_i + pol;
  if (std::abs(M) > U.J) return TDWP_EINVAL;
  const size_t pts = (size_t)p->ng * p->nR * p->nr;
  std::vector<double> u((size_t)U.n_om * p->ne * pts, 0.0);
  for (int a = 0; a < U.n_om; ++a) {
    const int om = U.om_lo + a;
    double* dst = u.data() + ((size_t)a * p->ne + elec) * pts;
    for (int b = 0; b < n_om_i; ++b) {
      const int omi = om_lo_i + b;
      const double* src = bound + (size_t)b * pts;
      for (int q = -1; q <= 1; ++q) {
        const double c = ((pol % 2) ? -1.0 : 1.0) *
                         coupling(U.J, M, U.parity, J_i, M_i, p_i, om, omi, q, pol);
        if (c == 0.0) continue;
        const double* d = dip + (size_t)(q + 1) * pts;
        for (size_t x = 0; x < pts; ++x) dst[x] += c * d[x] * src[x];
      }
    }
  }
  return tdwp_set_packet_values(p, unit, slot, u.data());
}
