"""Pins of the photodissociation oracle (Eqs. fourier-transform,
chebyshev-transform, spectrum, with c_k of Eq. chebyshev-expansion-constants)
against an eigendecomposition, exact quadrature sum rules and a closed form
(no GPU needed).

A plausible slip breaks at least one of them:
  - a wrong overlap index or recursion step: eigendecomposition of the dense H;
  - a wrong (2 - delta_k0), 1/pi, 1/(dE sin theta) or sign of the phase: the
    normalisation sum rule, the first moment, the eigenstate closed form;
  - a wrong prefactor of sigma or a wrong energy E_i + h nu: the integrated
    cross-section sum rule and the position of an eigenstate's peak.
"""
import math

import numpy as np
import pytest

from oracle import photo_oracle as PH
from oracle import tdwp_oracle as O
from workloads import config, ev
from workloads.photo import photo_packet


def tiny_spec(J=0, omega_max=0, n_elec=1, n_R=7, n_r=6, n_gamma=5):
    s = config(1)
    s.update(n_R=n_R, n_r=n_r, n_gamma=n_gamma, n_elec=n_elec)
    s["units"] = [dict(J=J, parity=(-1) ** J, omega_max=omega_max, n_packets=1)]
    if n_elec > 1:
        s["pes"]["shifts"] = [0.0, ev(0.5)][:n_elec]
        s["pes"]["couplings"] = {(0, 1): ev(0.1)}
    return s


def _eigen(op):
    H = O.dense_H(op, 0)
    lam, V = np.linalg.eigh(H)
    return H, lam, V


def test_undamped_autocorrelation_is_spectral_sum():
    # C_k = sum_n |<n|u_0>|^2 T_k(E_s,n) when D = 1
    op = O.Operator(tiny_spec(J=1, omega_max=1, n_elec=2))
    H, lam, V = _eigen(op)
    u0 = photo_packet(op.spec, 0, op.r, op.R, op.x, op.w)
    wts = (V.T @ u0.ravel()) ** 2
    theta = np.arccos((lam - op.E0) / op.dE)
    C = PH.autocorrelation(op, 0, u0, 50, undamped=True)
    for k in (0, 1, 2, 9, 50):
        assert C[k] == pytest.approx(float(np.sum(wts * np.cos(k * theta))), abs=1e-13 * C[0])


def test_uniformly_damped_autocorrelation_is_scaled_spectral_sum():
    # D = d everywhere: u_k = d^k T_k(H_s) u_0, so C_k = d^k sum_n |<n|u_0>|^2 T_k(E_s,n)
    op = O.Operator(tiny_spec(J=1, omega_max=1))
    H, lam, V = _eigen(op)
    u0 = photo_packet(op.spec, 0, op.r, op.R, op.x, op.w)
    wts = (V.T @ u0.ravel()) ** 2
    theta = np.arccos((lam - op.E0) / op.dE)
    d = 0.97
    C = PH.autocorrelation(op, 0, u0, 40, damping=d)
    for k in (1, 2, 5, 40):
        ref = d ** k * float(np.sum(wts * np.cos(k * theta)))
        assert C[k] == pytest.approx(ref, abs=1e-13 * C[0])


def test_damped_autocorrelation_starts_at_the_norm():
    op = O.Operator(tiny_spec())
    u0 = photo_packet(op.spec, 0, op.r, op.R, op.x, op.w)
    C = PH.autocorrelation(op, 0, u0, 40)
    assert C[0] == pytest.approx(float(np.sum(u0 * u0)), rel=1e-15)
    # the first component is the overlap with u_1 = D H_s u_0
    u1 = op.D * O.apply_Hs(op, 0, u0)
    assert C[1] == pytest.approx(float(np.sum(u0 * u1)), rel=1e-14)


def _theta_quadrature(M):
    th = (np.arange(M) + 0.5) * math.pi / M            # midpoint rule, exact for cos(k th), k < 2M
    return th, math.pi / M


@pytest.mark.parametrize("K", [1, 2, 17, 200])
def test_energy_content_normalisation_and_first_moment(K):
    # E = E0 + dE cos th:  int a_0 dE = C_0  and  int E a_0 dE = E0 C_0 + dE C_1
    rng = np.random.default_rng(K)
    C = rng.standard_normal(K)
    e_min, e_max = -0.3, 1.7
    E0, dE = 1.0 * (e_max + e_min) / 2, (e_max - e_min) / 2
    th, h = _theta_quadrature(4 * K + 8)
    E = E0 + dE * np.cos(th)
    a0 = PH.energy_content(C, e_min, e_max, E)
    jac = dE * np.sin(th) * h
    tol = 1e-13 * (K + 10) * np.max(np.abs(C))      # rounding of sums of about 4K terms
    assert float(np.sum(a0 * jac)) == pytest.approx(C[0], abs=tol)
    first = E0 * C[0] + (dE * C[1] if K > 1 else 0.0)
    assert float(np.sum(E * a0 * jac)) == pytest.approx(first, abs=tol)


def test_first_moment_is_the_packet_energy():
    # undamped: int E a_0(E) dE = <u_0|H|u_0>, from the oracle's own C_0, C_1
    op = O.Operator(tiny_spec(J=1, omega_max=1))
    H, _, _ = _eigen(op)
    u0 = photo_packet(op.spec, 0, op.r, op.R, op.x, op.w).ravel()
    C = PH.autocorrelation(op, 0, u0.reshape(op.unit_shape(0)), 3, undamped=True)
    th, h = _theta_quadrature(64)
    E = op.E0 + op.dE * np.cos(th)
    a0 = PH.energy_content(C, op.Emin, op.Emax, E)
    mean = float(np.sum(E * a0 * op.dE * np.sin(th) * h))
    assert mean == pytest.approx(float(u0 @ H @ u0), rel=1e-12)


def test_eigenstate_energy_content_is_a_dirichlet_kernel():
    # C_k = cos(k th_n):  sum_{k<K} (2 - d_k0) cos(k th) cos(k th_n)
    #   = [D_K(th - th_n) + D_K(th + th_n)] / 2,  D_K(x) = sin((K - 1/2) x) / sin(x / 2)
    e_min, e_max, K = 0.0, 2.0, 64
    th_n = 1.1
    C = np.cos(np.arange(K) * th_n)
    E = np.linspace(0.01, 1.99, 301)
    th = np.arccos(E - 1.0)
    Dk = lambda x: np.sin((K - 0.5) * x) / np.sin(0.5 * x)
    closed = 0.5 * (Dk(th - th_n) + Dk(th + th_n)) / (math.pi * 1.0 * np.sin(th))
    got = PH.energy_content(C, e_min, e_max, E)
    np.testing.assert_allclose(got, closed, rtol=0, atol=1e-11 * np.max(np.abs(closed)))
    # the peak sits at the eigenvalue E_n = E0 + dE cos th_n
    assert abs(E[np.argmax(got)] - (1.0 + math.cos(th_n))) < 0.01


def test_cross_section_sum_rule_and_energy_origin():
    # int sigma(h nu) / h nu d(h nu) = A int a_0 dE = A C_0 (over the whole range)
    rng = np.random.default_rng(3)
    C = rng.standard_normal(40)
    C[0] = 2.5
    e_min, e_max, E_i = -0.2, 0.8, -0.5
    E0, dE = 0.3, 0.5
    th, h = _theta_quadrature(200)
    E = E0 + dE * np.cos(th)
    hnu = E - E_i
    sig = PH.cross_section(C, e_min, e_max, E_i, hnu)
    total = float(np.sum(sig / hnu * dE * np.sin(th) * h))
    assert total == pytest.approx(4 * math.pi / 137.035999084 * C[0], rel=1e-12)
    # sigma is A h nu a_0 at the final energy E_i + h nu
    a0 = PH.energy_content(C, e_min, e_max, E_i + hnu)
    ref = 4 * math.pi / 137.035999084 * hnu * a0
    np.testing.assert_allclose(sig, ref, rtol=0, atol=1e-13 * np.max(np.abs(ref)))


# ---- initial packet of Eq. initial-photo-wvp -----------------------------------------------

@pytest.mark.parametrize("j", [0, 1, 2, 5, 9])
def test_clebsch_gordan_closed_forms_for_rank_one(j):
    """The standard j x 1 tables, <j m 1 0|j m> = m / sqrt(j(j+1)),
    <j m 1 0|j+1 m> = sqrt((j-m+1)(j+m+1)/((2j+1)(j+1))) and
    <j m-1 1 1|j+1 m> = sqrt((j+m)(j+m+1)/((2j+1)(2j+2))), read in the order 1 x j
    through <j1 m1 j2 m2|J M> = (-1)^(j1+j2-J) <j2 m2 j1 m1|J M>."""
    for m in range(-j, j + 1):
        if j > 0:
            assert abs(PH.clebsch_gordan(1, 0, j, m, j, m) + m / math.sqrt(j * (j + 1))) < 1e-14
        want = math.sqrt((j - m + 1) * (j + m + 1) / ((2 * j + 1) * (j + 1)))
        assert abs(PH.clebsch_gordan(1, 0, j, m, j + 1, m) - want) < 1e-14
    for m in range(-j, j + 2):
        want = math.sqrt((j + m) * (j + m + 1) / ((2 * j + 1) * (2 * j + 2)))
        assert abs(PH.clebsch_gordan(1, 1, j, m - 1, j + 1, m) - want) < 1e-14


@pytest.mark.parametrize("j2", [0, 1, 3, 4])
def test_clebsch_gordan_orthonormal(j2):
    """sum_{m1 m2} <1 m1 j2 m2|J M><1 m1 j2 m2|J' M'> = delta_JJ' delta_MM'."""
    Js = range(abs(j2 - 1), j2 + 2)
    for J in Js:
        for Jp in Js:
            for M in range(-J, J + 1):
                s = sum(PH.clebsch_gordan(1, m1, j2, M - m1, J, M) * PH.clebsch_gordan(1, m1, j2, M - m1, Jp, M)
                        for m1 in (-1, 0, 1))
                assert abs(s - (1.0 if J == Jp else 0.0)) < 1e-13


def _wigner_small_d(j, mp, m, beta):
    """d^j_{m' m}(beta) by Wigner's explicit sum (independent of the coupling route)."""
    f = math.factorial
    c, s = np.cos(beta / 2.0), np.sin(beta / 2.0)
    out = np.zeros_like(beta)
    for k in range(max(0, m - mp), min(j + m, j - mp) + 1):
        num = (-1) ** (mp - m + k) * math.sqrt(f(j + mp) * f(j - mp) * f(j + m) * f(j - m))
        den = f(j + m - k) * f(k) * f(j - k - mp) * f(k - m + mp)
        out = out + num / den * c ** (2 * j - 2 * k + m - mp) * s ** (2 * k - m + mp)
    return out


def _W(J, M, par, om, phi, th, chi):
    """W^{JMp}_{Omega, Lambda=0} of Eq. angular-functions (sigma = +1) on Euler-angle grids."""
    def Dstar(mp, m):
        return np.exp(1j * mp * phi) * _wigner_small_d(J, mp, m, th) * np.exp(1j * m * chi)
    norm = math.sqrt((2 * J + 1) / (16 * math.pi ** 2 * (1 + (om == 0))))
    return norm * (Dstar(M, om) + par * (-1) ** (J + om) * Dstar(M, -om))


@pytest.mark.parametrize("J,par,Ji,Mi,pari,pol", [(1, -1, 0, 0, 1, 0), (2, 1, 1, 0, -1, 0),
                                                  (3, -1, 2, 1, 1, 1), (2, -1, 2, -1, -1, -1),
                                                  (4, 1, 3, 2, 1, -1)])
def test_dipole_coupling_equals_euler_angle_quadrature(J, par, Ji, Mi, pari, pol):
    """<W_Omega|D^{1*}_{pol q}|W_Omega_i> by direct quadrature over (phi, theta, chi)
    with Wigner's d-function sum equals the oracle's Clebsch-Gordan reduction, for
    every Omega, Omega_i and q (zero where the selection rules forbid)."""
    n_ang, n_th = 16, 96
    phi = 2 * math.pi * np.arange(n_ang) / n_ang
    xg, wg = np.polynomial.legendre.leggauss(n_th)
    th = 0.5 * math.pi * (xg + 1.0)
    wt = 0.5 * math.pi * wg * np.sin(th)
    P, T, C = np.meshgrid(phi, th, phi, indexing="ij")
    wts = (2 * math.pi / n_ang) ** 2 * wt[None, :, None]
    M = Mi + pol
    if abs(M) > J:
        pytest.skip("M outside the final J")
    oms = [o for o in range(0, J + 1) if not (o == 0 and par * (-1) ** J != 1)]
    omis = [o for o in range(0, Ji + 1) if not (o == 0 and pari * (-1) ** Ji != 1)]
    checked = 0
    for om in oms:
        Wf = np.conj(_W(J, M, par, om, P, T, C))
        for omi in omis:
            Wi = _W(Ji, Mi, pari, omi, P, T, C)
            for q in (-1, 0, 1):
                D1s = np.exp(1j * pol * P) * _wigner_small_d(1, pol, q, T) * np.exp(1j * q * C)
                quad = np.sum(wts * Wf * D1s * Wi)
                want = PH.dipole_coupling(J, M, par, Ji, Mi, pari, om, omi, q, pol)
                assert abs(quad.imag) < 1e-13
                assert abs(quad.real - want) < 1e-12, (om, omi, q, quad, want)
                checked += abs(want) > 1e-6
    assert checked > 0


def test_photo_packet_j0_to_j1_linear_polarisation_closed_form():
    """J_i = 0 -> J = 1 (final parity -1, helicities 0 and 1), linear polarisation:
    Phi_0 = d_z Phi_i / sqrt(3) and Phi_1 = -d_x Phi_i / sqrt(3) for a dipole in the
    x-z plane (d_{+-1} = -+ d_x / sqrt(2), d_0 = d_z): the relative sign of the two
    helicity blocks is fixed, and |Phi_0|^2 + |Phi_1|^2 = |d|^2 |Phi_i|^2 / 3."""
    s = tiny_spec(J=1, omega_max=1)
    s["units"] = [dict(J=1, parity=-1, omega_max=1, n_packets=1)]
    rng = np.random.default_rng(7)
    shape = (s["n_gamma"], s["n_R"], s["n_r"])
    bound = rng.standard_normal((1,) + shape)
    dx, dz = rng.standard_normal(shape), rng.standard_normal(shape)
    dip = np.stack([dx / math.sqrt(2), dz, -dx / math.sqrt(2)])
    u = PH.photo_packet(s, 0, 0, 0, 0, 1, [0], bound, dip, 0)
    assert u.shape == (2, 1) + shape
    assert np.max(np.abs(u[0, 0] - dz * bound[0] / math.sqrt(3))) < 1e-14
    assert np.max(np.abs(u[1, 0] + dx * bound[0] / math.sqrt(3))) < 1e-14
    # the same J with parity +1 (helicity 1 only) is reached by no in-plane dipole
    s["units"] = [dict(J=1, parity=1, omega_max=1, n_packets=1)]
    assert np.max(np.abs(PH.photo_packet(s, 0, 0, 0, 0, 1, [0], bound, dip, 0))) < 1e-15
