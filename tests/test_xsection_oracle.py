"""Pins of the partial-wave-sum oracle (Sec. "Cross sections": Eqs.
collisional-xsection, cumulative-probability, J-shifting-interpolation) against
closed forms, brute-force sums and a classical limit (no GPU needed).

A plausible slip in the oracle breaks at least one of them:
  - the printed weights (exchanged), or a weight on the wrong curve:
    reproduction at computed J and linear blending of constant curves;
  - a wrong sign or a J^2 for J(J+1) in either shift: exactly J-shifted
    linear curves;
  - a wrong degeneracy factor or a family counted below its smallest J: the
    closed-form (2J+1) sums and the brute-force sum over every computed J;
  - a wrong K0^2 or a missing (2 j0 + 1): the classical limit pi b^2;
  - a fit that is not a minimum, or on the wrong curve: recovery of a known B.
"""
import math

import numpy as np
import pytest

from oracle import xsection_oracle as X
from workloads import amu, ev
from workloads.partial_waves import energy_grid, families, probability_curves

# Effective rotational constant of the J-shifting figure (H + H2), 1.7 meV.
B_FIG = ev(1.7e-3)


def test_interpolation_reproduces_the_computed_curves():
    rng = np.random.default_rng(1)
    e = energy_grid(57, 0.0, 0.1, seed=2)
    p1, p2 = rng.uniform(size=57), rng.uniform(size=57)
    np.testing.assert_array_equal(X.jshift_interpolate(p1, p2, e, 4, 9, B_FIG, 4), p1)
    np.testing.assert_array_equal(X.jshift_interpolate(p1, p2, e, 4, 9, B_FIG, 9), p2)
    np.testing.assert_array_equal(X.jshift(p1, e, 7, B_FIG, 7), p1)
    curves = [p1, p2, rng.uniform(size=57)]
    for c, J in enumerate((0, 3, 8)):
        np.testing.assert_array_equal(X.probability_at_J(J, (0, 3, 8), [B_FIG] * 3, curves, e),
                                      curves[c])


def test_interpolation_of_constant_curves_is_linear_in_J():
    # a constant curve is unchanged by any shift, so only the weights act
    e = np.linspace(0.0, 0.1, 40)
    a, b = 0.2, 0.9
    for J in range(3, 12):
        got = X.jshift_interpolate(np.full(40, a), np.full(40, b), e, 3, 11, B_FIG, J)
        np.testing.assert_allclose(got, a + (b - a) * (J - 3) / 8, rtol=0, atol=1e-15)


def _linear_family(alpha, beta, B):
    # P^J(E) = alpha (E - B J(J+1)) + beta: exactly J-shifted linear curves
    return lambda J, e: alpha * (e - B * J * (J + 1)) + beta


def test_jshift_of_exactly_shifted_linear_curves():
    B = 10 * B_FIG
    fam = _linear_family(0.3, 0.05, B)
    e = energy_grid(301, 0.0, 2.0, seed=5)
    inner = (e > 0.6) & (e < 1.4)          # all read points stay inside the grid
    for J_ref, J in ((0, 5), (7, 3), (2, 11)):
        got = X.jshift(fam(J_ref, e), e, J_ref, B, J)
        np.testing.assert_allclose(got[inner], fam(J, e)[inner], rtol=0, atol=1e-13)
    for J in range(4, 13):
        got = X.jshift_interpolate(fam(4, e), fam(12, e), e, 4, 12, B, J)
        np.testing.assert_allclose(got[inner], fam(J, e)[inner], rtol=0, atol=1e-13)


def test_jshift_moves_a_threshold_up_by_the_rotational_energy():
    # a ramp from 0 to 1 between e_a and e_b, grid points on both kinks
    e = np.linspace(0.0, 1.0, 1001)
    ramp = lambda x, a, b: np.clip((x - a) / (b - a), 0.0, 1.0)
    B = 0.25e-3
    got = X.jshift(ramp(e, 0.2, 0.3), e, 0, B, 10)          # shift 110 B = 0.0275
    np.testing.assert_allclose(got, ramp(e, 0.2275, 0.3275), rtol=0, atol=1e-12)


def test_cumulative_degeneracy_sum_closed_form():
    # J-independent constant curves: sum_{J=jmin}^{N} (2J+1) = (N+1)^2 - jmin^2
    e = np.linspace(0.01, 0.05, 9)
    fams, jmin = families(3)
    J_calc, N, q = [0, 5, 12, 20], 23, 0.37
    p = np.full((4, len(fams), 2, 9), q)
    for c, J in enumerate(J_calc):
        for k, jm in enumerate(jmin):
            if J < jm:
                p[c, k] = 0.0
    # families with Omega0 = 1..3 start inside [0, 5]: their J < 5 terms blend the
    # zero row at J = 0 with q at J = 5 (weight J / 5 when B = 0)
    C = X.cumulative_probability(J_calc, [0.0] * 4, p, e, N, fam_jmin=jmin)
    expect = 0.0
    for jm in jmin:
        for J in range(jm, N + 1):
            w = 1.0 if (J >= 5 or jm == 0) else J / 5.0
            expect += (2 * J + 1) * q * w
    np.testing.assert_allclose(C, expect, rtol=1e-14)
    # with every family starting at J = 0 the plain closed form holds
    p0 = np.full((4, len(fams), 2, 9), q)
    C0 = X.cumulative_probability(J_calc, [B_FIG] * 4, p0, e, N)
    np.testing.assert_allclose(C0, q * len(fams) * (N + 1) ** 2, rtol=1e-14)


def test_cumulative_with_every_J_computed_is_the_direct_sum():
    rng = np.random.default_rng(11)
    e = energy_grid(33, ev(0.2), ev(1.5), seed=12)
    N = 9
    fams, jmin = families(2)
    p = probability_curves(N + 1, len(fams), 3, e, seed=13, fam_jmin=jmin, J_calc=range(N + 1))
    B = rng.uniform(0.0, 5 * B_FIG, N + 1)             # irrelevant when every J is computed
    C = X.cumulative_probability(range(N + 1), B, p, e, N, fam_jmin=jmin)
    direct = np.zeros((3, 33))
    for J in range(N + 1):
        for k, jm in enumerate(jmin):
            if J >= jm:
                direct += (2 * J + 1) * p[J, k]
    np.testing.assert_allclose(C, direct, rtol=1e-14, atol=0)


def test_cumulative_of_exactly_shifted_linear_curves_closed_form():
    # sum_{J=0}^{N} (2J+1) [alpha (E - B J(J+1)) + beta]
    #   = (alpha E + beta) (N+1)^2 - alpha B N (N+1)^2 (N+2) / 2
    B, alpha, beta, N = B_FIG, 0.4, 0.02, 40
    fam = _linear_family(alpha, beta, B)
    e = energy_grid(401, 0.0, 1.0, seed=21)
    J_calc = [3, 6, 10, 17, 25, 31, 36]           # first above 0, last below N
    p = np.stack([fam(J, e) for J in J_calc])[:, None, None, :]
    C = X.cumulative_probability(J_calc, [B] * len(J_calc), p, e, N)[0]
    inner = (e > 0.15) & (e < 0.85)               # largest shift B N(N+1) = 0.1 hartree
    closed = (alpha * e + beta) * (N + 1) ** 2 - alpha * B * N * (N + 1) ** 2 * (N + 2) / 2
    np.testing.assert_allclose(C[inner], closed[inner], rtol=1e-12)


@pytest.mark.parametrize("j0", [0, 1, 3])
def test_cross_section_classical_limit(j0):
    # every partial wave up to J_max reacts with probability 1; the impact
    # parameter of the last one is b = (J_max + 1) / K0, and the cross section
    # tends to the disk area pi b^2 (exactly for j0 = 0; the families with
    # Omega0 > 0 miss J < Omega0, a relative 2 sum Omega0^2 / ((2 j0 + 1)(J_max+1)^2))
    mu = amu(1.008) * amu(3.022) / amu(4.030)
    b, N = 3.0, 400
    K0 = (N + 1) / b
    E = K0 ** 2 / (2 * mu)
    e = np.array([0.5 * E, E, 1.5 * E])
    fams, jmin = families(j0)
    p = np.ones((N + 1, len(fams), 1, 3))
    for J in range(N + 1):
        for k, jm in enumerate(jmin):
            if J < jm:
                p[J, k] = 0.0
    C = X.cumulative_probability(range(N + 1), [0.0] * (N + 1), p, e, N, fam_jmin=jmin)
    sigma = X.cross_section(C, e, mu, j0)[0]
    missing = 2 * sum(om * om for om in range(1, j0 + 1)) / ((2 * j0 + 1) * (N + 1) ** 2)
    assert sigma[1] == pytest.approx(math.pi * b * b * (1 - missing), rel=1e-12)
    # at other energies K0 changes: sigma scales as 1/E at fixed J_max
    assert sigma[0] == pytest.approx(2 * sigma[1], rel=1e-12)
    assert sigma[2] == pytest.approx(sigma[1] / 1.5, rel=1e-12)


def test_fit_recovers_a_grid_aligned_shift_exactly():
    # piecewise-linear curve with kinks on the grid, J2 curve shifted by exactly
    # 7 grid steps: the misfit vanishes at the true B and nowhere else nearby
    e = np.linspace(0.0, 1.0, 501)
    h = e[1] - e[0]
    ramp = lambda x: np.clip((x - 0.3) / 0.2, 0.0, 1.0) * (1 - 0.3 * np.clip((x - 0.6) / 0.2, 0, 1))
    J1, J2 = 4, 6
    B_true = 7 * h / (J2 * (J2 + 1) - J1 * (J1 + 1))
    got = X.fit_jshift_b(ramp(e), ramp(e - 7 * h), e, J1, J2, 5 * B_true)
    assert got == pytest.approx(B_true, rel=1e-9)
    assert X.jshift_misfit(ramp(e), ramp(e - 7 * h), e, J1, J2, got) < 1e-20


def test_fit_recovers_the_constant_of_smooth_shifted_curves():
    e = np.linspace(ev(0.2), ev(1.5), 2000)
    f = lambda x: 0.8 / (1.0 + np.exp(-(x - ev(0.5)) / ev(0.04)))
    J1, J2 = 10, 12
    shift = B_FIG * (J2 * (J2 + 1) - J1 * (J1 + 1))
    got = X.fit_jshift_b(f(e), f(e - shift), e, J1, J2, 4 * B_FIG)
    assert got == pytest.approx(B_FIG, rel=1e-4)
    # identical curves: B = 0
    assert X.fit_jshift_b(f(e), f(e), e, J1, J2, 4 * B_FIG) == pytest.approx(0.0, abs=1e-12)


def test_fit_is_a_minimum_of_the_misfit_by_brute_force():
    e = energy_grid(25, 0.0, 0.2, seed=31)
    p = probability_curves(2, 1, 1, e, seed=32)
    p1, p2 = p[0, 0, 0], p[1, 0, 0]
    B_max = 0.2 / 30
    got = X.fit_jshift_b(p1, p2, e, 2, 4, B_max)
    best = min(X.jshift_misfit(p1, p2, e, 2, 4, b) for b in np.linspace(0, B_max, 20001))
    assert 0.0 <= got <= B_max
    assert X.jshift_misfit(p1, p2, e, 2, 4, got) <= best + 1e-15


def test_each_interval_uses_its_own_constant():
    # thresholds E_J that rise by B_c [J(J+1) - J_c(J_c+1)] inside interval c, with
    # a different B_c per interval: P^J(E) = alpha (E - E_J) + beta exactly
    alpha, beta = 0.5, 0.1
    J_calc = [0, 4, 9, 15]
    B = [B_FIG, 3 * B_FIG, 0.5 * B_FIG, 2 * B_FIG]
    E_J, Ec = {}, 0.0
    for c, Jc in enumerate(J_calc):
        J_end = J_calc[c + 1] if c + 1 < len(J_calc) else 20
        for J in range(Jc, J_end + 1):
            E_J[J] = Ec + B[c] * (J * (J + 1) - Jc * (Jc + 1))
        Ec = E_J[J_end]
    e = energy_grid(301, 0.0, 0.3, seed=41)
    inner = (e > 0.1) & (e < 0.2)
    curves = [alpha * (e - E_J[J]) + beta for J in J_calc]
    for J in range(0, 21):
        got = X.probability_at_J(J, J_calc, B, curves, e)
        np.testing.assert_allclose(got[inner], (alpha * (e - E_J[J]) + beta)[inner],
                                   rtol=0, atol=1e-13)
    C = X.cumulative_probability(J_calc, B, np.stack(curves)[:, None, None, :], e, 20)[0]
    direct = sum((2 * J + 1) * (alpha * (e - E_J[J]) + beta) for J in range(21))
    np.testing.assert_allclose(C[inner], direct[inner], rtol=1e-13)
