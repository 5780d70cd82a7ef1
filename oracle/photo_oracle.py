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

Pinned by tests/test_photo_oracle.py: the undamped autocorrelation against an
eigendecomposition of the dense H (and, with a uniform damping d, against
d^k times it), the normalisation sum rule (the integral of
a_0 over the spectral range is C_0) and the first moment (<u_0|H|u_0>) by exact
quadrature, the Dirichlet-kernel closed form of a_0 for an eigenstate packet,
and the integrated cross section sum rule.  lowest_state is a library
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
