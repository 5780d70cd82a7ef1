"""FP64 CPU oracle for the photodissociation analysis of arXiv 2412.10167
(MADWAVE3): autocorrelation of the propagated packet, its Chebyshev transform
to the energy content a_0(E) (Eqs. fourier-transform, chebyshev-transform)
and the total photodissociation cross section (Eq. spectrum).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the library and imports nothing from it; the recursion is the one of
oracle/tdwp_oracle.py (Sec. 2.2, Eq. wvp-k).

  autocorrelation  C_k = <u_0|u_k>, k = 0..K, along the damped recursion.
  energy_content   a_0(E) = (1/pi) sum_k Re c_k(H_s, E) C_k with c_k of Eq.
                   chebyshev-expansion-constants (hbar = 1), i.e. Eq.
                   chebyshev-transform.
  cross_section    sigma(h nu) = A h nu / (2 pi) sum_k 2 Re[c_k(H_s, E) C_k],
                   E = E_i + h nu (Eq. spectrum).
  lowest_state     the lowest eigenpair of the dense H (the initial bound state's
                   definition; the paper finds it with a Lanczos method).
  photo_packet     the initial packet of Eq. initial-photo-wvp: d.e times the
                   bound state projected on the helicity functions of the final
                   J (Eq. angular-functions), with the transition operator
                   sum_pq (-1)^p e_{-p} D^{1*}_{pq} d_q of the same section.

Readings (each also listed in the design notes):
  * The components C_k of a real packet under the real recursion are real, so
    Re[c_k C_k] = C_k Re c_k = C_k (2 - delta_k0) cos(k theta) / (dE sin theta),
    theta = arccos E_s, E_s = (E - E0)/dE; energies must lie strictly inside
    (E_min, E_max).
  * A = 1/(hbar^2 eps0 c) as printed; in atomic units (hbar = 1, 4 pi eps0 = 1)
    A = 4 pi / c with c = 137.035999084 (CODATA 2018).  The textbook
    golden-rule prefactor of the absorption cross section is pi times this; the
    printed one is kept.
  * h nu is the photon energy and E_i the energy of the initial bound state on
    the energy scale of H, so the final energy is E = E_i + h nu.

  * Initial packet: Lambda = 0 electronic states with sigma = +1 on both sides
    (so |-Lambda, sigma> = |Lambda, sigma> in Eq. angular-functions); Wigner
    functions in the convention D^j_{m'm}(phi, theta, chi) = e^{-i m' phi}
    d^j_{m'm}(theta) e^{-i m chi}; Clebsch-Gordan coefficients with the Condon-
    Shortley phase; the polarisation component (e)_{-p} has unit amplitude and
    the final M is M_i + p; the body-frame spherical components d_q are real
    inputs (a dipole in the x-z plane has d_{+-1} = -+ d_x / sqrt(2), d_0 = d_z).
    The Euler-angle integral of W* D^{1*} W then reduces to
    8 pi^2/(2J+1) <1 p J_i M_i|J M> <1 q J_i Omega_i'|J Omega'> summed over the
    two signed helicities of each W.

Pinned by tests/test_photo_oracle.py: the undamped autocorrelation against an
eigendecomposition of the dense H (and, with a uniform damping d, against
d^k times it), the normalisation sum rule (the integral of
a_0 over the spectral range is C_0) and the first moment (<u_0|H|u_0>) by exact
quadrature, the Dirichlet-kernel closed form of a_0 for an eigenstate packet,
and the integrated cross section sum rule.  photo_packet: Clebsch-Gordan
closed forms and orthonormality, the Euler-angle integral of W* D^{1*} W by
direct quadrature with Wigner's d-function sum, and the closed form of a
J_i = 0 -> J = 1 packet under linear polarisation.  lowest_state is a library
eigensolver on the dense H, whose construction the tdwp_oracle pins fix
(symmetry, spectrum, closed-form special cases).
"""
import math

import numpy as np

from oracle import tdwp_oracle as O

C_AU = 137.035999084          # speed of light in atomic units (CODATA 2018)
A_AU = 4.0 * math.pi / C_AU   # A = 1/(hbar^2 eps0 c) with hbar = 1, eps0 = 1/(4 pi)


def autocorrelation(op, unit_index, u0, K, undamped=False, damping=None):
    """C_k = <u_0|u_k> for k = 0..K: u_1 = D H_s u_0, u_{k+1} = D (2 H_s u_k - D u_{k-1}).
    `damping` replaces D by any array broadcastable to u (tests); `undamped` sets D = 1."""
    if damping is not None:
        D = damping
    else:
        D = np.ones_like(op.D) if undamped else op.D
    C = np.empty(K + 1)
    C[0] = float(np.sum(u0 * u0))
    if K == 0:
        return C
    u_prev = u0
    u = D * O.apply_Hs(op, unit_index, u0)
    C[1] = float(np.sum(u0 * u))
    for k in range(1, K):
        u_next = D * (2.0 * O.apply_Hs(op, unit_index, u) - D * u_prev)
        u_prev, u = u, u_next
        C[k + 1] = float(np.sum(u0 * u))
    return C


def lowest_state(op, unit_index):
    """Lowest eigenpair of the dense H of one unit (the bound state the preparatory
    stage finds iteratively), by a library symmetric eigensolver: (E, psi) with psi
    DVR-normalised and its largest component positive."""
    lam, V = np.linalg.eigh(O.dense_H(op, unit_index))
    psi = V[:, 0]
    psi = psi * np.sign(psi[np.argmax(np.abs(psi))])
    return float(lam[0]), psi.reshape(op.unit_shape(unit_index))


def _re_ck(E, e_min, e_max, K):
    """Re c_k(H_s, E), k = 0..K-1, for each E: shape [n_E][K]."""
    E0, dE = 0.5 * (e_max + e_min), 0.5 * (e_max - e_min)
    Es = (np.asarray(E, dtype=np.float64) - E0) / dE
    assert np.all(np.abs(Es) < 1.0), "energies must lie inside the spectral range"
    theta = np.arccos(Es)
    out = np.empty((Es.size, K))
    for k in range(K):
        out[:, k] = (1.0 if k == 0 else 2.0) * np.cos(k * theta) / (dE * np.sin(theta))
    return out


def energy_content(C, e_min, e_max, E):
    """a_0(E) of Eq. chebyshev-transform from C_0..C_{K-1}."""
    C = np.asarray(C, dtype=np.float64)
    return _re_ck(E, e_min, e_max, C.size) @ C / math.pi


def cross_section(C, e_min, e_max, E_i, hnu):
    """sigma(h nu) of Eq. spectrum (bohr^2) at photon energies hnu."""
    C = np.asarray(C, dtype=np.float64)
    hnu = np.asarray(hnu, dtype=np.float64)
    s = _re_ck(E_i + hnu, e_min, e_max, C.size) @ C
    return A_AU * hnu / (2.0 * math.pi) * 2.0 * s


# ---------------------------------------------------------------------------
# Initial packet of Eq. initial-photo-wvp
# ---------------------------------------------------------------------------

def clebsch_gordan(j1, m1, j2, m2, J, M):
    """<j1 m1 j2 m2 | J M> for integer angular momenta, Condon-Shortley phase,
    by Racah's closed formula."""
    if m1 + m2 != M or not abs(j1 - j2) <= J <= j1 + j2:
        return 0.0
    if abs(m1) > j1 or abs(m2) > j2 or abs(M) > J:
        return 0.0
    f = math.factorial
    pre = math.sqrt((2 * J + 1) * f(J + j1 - j2) * f(J - j1 + j2) * f(j1 + j2 - J)
                    / f(j1 + j2 + J + 1))
    pre *= math.sqrt(f(J + M) * f(J - M) * f(j1 - m1) * f(j1 + m1) * f(j2 - m2) * f(j2 + m2))
    total = 0.0
    for k in range(j1 + j2 - J + 1):
        den = (k, j1 + j2 - J - k, j1 - m1 - k, j2 + m2 - k, J - j2 + m1 + k, J - j1 - m2 + k)
        if min(den) < 0:
            continue
        term = 1.0
        for x in den:
            term *= f(x)
        total += (-1) ** k / term
    return pre * total


def helicity_norm(J, omega):
    """Normalisation of W^{JMp}_{Omega Lambda} (Eq. angular-functions)."""
    return math.sqrt((2 * J + 1) / (16.0 * math.pi ** 2 * (1 + (omega == 0))))


def dipole_coupling(J, M, par, Ji, Mi, pari, omega, omega_i, q, pol):
    """Euler-angle integral <W^{J M par}_{omega} | D^{1*}_{pol q} | W^{Ji Mi pari}_{omega_i}>
    for Lambda = 0, sigma = +1 states: each W is N [D^{J*}_{M, omega} + par (-1)^(J+omega)
    D^{J*}_{M, -omega}], and the integral of D^J_{M a} D^{1*}_{pol q} D^{Ji*}_{Mi b} over
    the Euler angles is 8 pi^2/(2J+1) <1 pol Ji Mi|J M> <1 q Ji b|J a>."""
    if M != Mi + pol:
        return 0.0
    cg_m = clebsch_gordan(1, pol, Ji, Mi, J, M)
    total = 0.0
    for s, fs in ((1, 1.0), (-1, par * (-1) ** (J + omega))):
        for si, fi in ((1, 1.0), (-1, pari * (-1) ** (Ji + omega_i))):
            total += fs * fi * clebsch_gordan(1, q, Ji, si * omega_i, J, s * omega)
    return (helicity_norm(J, omega) * helicity_norm(Ji, omega_i) * 8.0 * math.pi ** 2
            / (2 * J + 1) * cg_m * total)


def photo_packet(spec, unit_index, elec, Ji, Mi, pari, omega_i_list, bound, dip, pol):
    """Packet u[n_Omega][n_elec][n_gamma][n_R][n_r] of unit `unit_index` (its J and
    parity, helicities of omega_range) in diabatic state `elec` (Eq. initial-photo-wvp):
        Phi_Omega = sum_{Omega_i, q} (-1)^pol <W_Omega|D^{1*}_{pol q}|W_{Omega_i}> d_q Phi_i,Omega_i
    bound[b] is the bound state's component Omega_i = omega_i_list[b], dip[q + 1]
    the body-frame component d_q, both DVR-weighted arrays [n_gamma][n_R][n_r]
    (the dipole is local, so it multiplies the coefficients point by point)."""
    from oracle import tdwp_oracle as Ot
    unit = spec["units"][unit_index]
    oms = Ot.omega_range(unit)
    J, par = unit["J"], unit["parity"]
    M = Mi + pol
    bound = np.asarray(bound, dtype=np.float64)
    dip = np.asarray(dip, dtype=np.float64)
    u = np.zeros((len(oms), spec["n_elec"]) + bound.shape[1:])
    for a, om in enumerate(oms):
        for b, omi in enumerate(omega_i_list):
            for q in (-1, 0, 1):
                c = (-1) ** pol * dipole_coupling(J, M, par, Ji, Mi, pari, om, omi, q, pol)
                if c != 0.0:
                    u[a, elec] += c * dip[q + 1] * bound[b]
    return u
