"""FP64 CPU oracle for the partial-wave sums of arXiv 2412.10167 (MADWAVE3),
Sec. "Cross sections" and Sec. "Higher partial wave, J>0, and cross sections".

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the library and imports nothing from it.

Plain on purpose: one Python loop per sum of the equations, every curve read
between grid points with numpy's linear interpolation (np.interp, which keeps
the end values outside the grid).  Energies and rotational constants in
hartree, masses in electron masses, hbar = 1.

  jshift                 J-shifting approach (the reference the section cites,
                         and the caption of the J-shifting figure): the curve of
                         J_ref moved up in energy by B [J(J+1) - J_ref(J_ref+1)].
  jshift_interpolate     Eq. J-shifting-interpolation.
  probability_at_J       which computed curves make the curve of a given J.
  cumulative_probability Eq. cumulative-probability.
  cross_section          Eq. collisional-xsection.
  fit_jshift_b           the fitted B of an interval (the section states that B
                         is fitted per interval, not how).

Readings where the paper is garbled or silent (each also listed in the design
notes):
  * The weights printed in Eq. J-shifting-interpolation are exchanged: as
    printed, J = J1 would return the J2 curve shifted down to J1.  The weight
    of the J1 term here is (J2 - J)/(J2 - J1) and that of the J2 term
    (J - J1)/(J2 - J1), so the computed curves are reproduced at J1 and J2.
  * The figure caption's J-shifting formula lost its B and its sign; the text
    says the curves move up with J, so P^J(E) = P^{J_ref}(E - B [J(J+1) -
    J_ref(J_ref+1)]).
  * One B per computed J, as in the per-J table of the cross-section program
    (a J and the constant for the interval that starts at it); the last one
    J-shifts above the last computed J, the first one below the first.
  * A family (Omega0, p) with Omega0 > J has no state at that J: it adds
    nothing there, and its curve at a computed J below Omega0 is zero.
  * The fitted B minimises the summed squared difference between the J1 curve
    J-shifted to J2 and the computed J2 curve, over B in [0, B_max].

Pinned by tests/test_xsection_oracle.py: exact reproduction at computed J,
curves that are exactly J-shifted linear functions (closed forms for the
interpolation and the cumulative sum), the (2J+1) degeneracy sum in closed
form, brute-force sums when every J is computed, the classical geometric
limit pi b^2 of the cross section (with the (2 j0 + 1) families), and the
recovery of a known B from exactly shifted analytic curves.
"""
import math

import numpy as np


def _rot(J):
    return J * (J + 1)


def jshift(p_ref, energies, J_ref, B, J):
    """P^J(E) = P^{J_ref}(E - B [J(J+1) - J_ref(J_ref+1)]) on the grid."""
    e = np.asarray(energies, dtype=np.float64)
    shift = B * (_rot(J) - _rot(J_ref))
    return np.interp(e - shift, e, np.asarray(p_ref, dtype=np.float64))


def jshift_interpolate(p1, p2, energies, J1, J2, B, J):
    """Eq. J-shifting-interpolation for J1 <= J <= J2 (weights as read above)."""
    assert J1 < J2 and J1 <= J <= J2
    e = np.asarray(energies, dtype=np.float64)
    up = np.interp(e - B * (_rot(J) - _rot(J1)), e, np.asarray(p1, dtype=np.float64))
    down = np.interp(e + B * (_rot(J2) - _rot(J)), e, np.asarray(p2, dtype=np.float64))
    return (J2 - J) / (J2 - J1) * up + (J - J1) / (J2 - J1) * down


def probability_at_J(J, J_calc, B, curves, energies):
    """|S^J|^2 of one family and final state: curves[c] is the computed curve at
    J_calc[c]; B[c] is the constant of the interval starting at J_calc[c]."""
    J_calc = list(J_calc)
    if J in J_calc:
        return np.asarray(curves[J_calc.index(J)], dtype=np.float64)
    if J < J_calc[0]:
        return jshift(curves[0], energies, J_calc[0], B[0], J)
    if J > J_calc[-1]:
        return jshift(curves[-1], energies, J_calc[-1], B[-1], J)
    c = max(i for i in range(len(J_calc)) if J_calc[i] < J)
    return jshift_interpolate(curves[c], curves[c + 1], energies, J_calc[c], J_calc[c + 1],
                              B[c], J)


def cumulative_probability(J_calc, B, p, energies, J_max, fam_jmin=None):
    """Eq. cumulative-probability: C[f](E) = sum_J sum_fam (2J+1) |S^J_{fam,f}(E)|^2.

    p[c][fam][f][i]: computed probabilities at J_calc[c]; fam runs over the
    (Omega0, p) families, f over the final states; fam_jmin[fam] the smallest J
    of each family (default 0).  Returns C[f][i]."""
    p = np.asarray(p, dtype=np.float64)
    n_calc, n_fam, n_f, n_e = p.shape
    assert len(J_calc) == n_calc and len(B) == n_calc
    if fam_jmin is None:
        fam_jmin = [0] * n_fam
    C = np.zeros((n_f, n_e))
    for J in range(J_max + 1):
        for fam in range(n_fam):
            if J < fam_jmin[fam]:
                continue
            for f in range(n_f):
                C[f] += (2 * J + 1) * probability_at_J(J, J_calc, B, p[:, fam, f, :], energies)
    return C


def cross_section(C, e_col, mu, j0):
    """Eq. collisional-xsection: sigma = pi / (K0^2 (2 j0 + 1)) C, K0^2 = 2 mu E (bohr^2)."""
    C = np.asarray(C, dtype=np.float64)
    out = np.empty_like(C)
    for i, E in enumerate(np.asarray(e_col, dtype=np.float64)):
        K0_sq = 2.0 * mu * E
        out[..., i] = math.pi / (K0_sq * (2 * j0 + 1)) * C[..., i]
    return out


def jshift_misfit(p1, p2, energies, J1, J2, B):
    """Summed squared difference between p1 J-shifted from J1 to J2 and p2."""
    r = jshift(p1, energies, J1, B, J2) - np.asarray(p2, dtype=np.float64)
    return float(np.sum(r * r))


def fit_jshift_b(p1, p2, energies, J1, J2, B_max, n_scan=4096):
    """argmin over B in [0, B_max] of jshift_misfit: a dense scan, then scipy's
    bounded scalar minimiser inside the two cells around the best scan point."""
    from scipy.optimize import minimize_scalar

    grid = np.linspace(0.0, B_max, n_scan + 1)
    cost = [jshift_misfit(p1, p2, energies, J1, J2, b) for b in grid]
    k = int(np.argmin(cost))
    lo, hi = grid[max(k - 1, 0)], grid[min(k + 1, n_scan)]
    res = minimize_scalar(lambda b: jshift_misfit(p1, p2, energies, J1, J2, b),
                          bounds=(lo, hi), method="bounded",
                          options={"xatol": 1e-14 * B_max, "maxiter": 500})
    return float(res.x) if res.fun <= cost[k] else float(grid[k])
