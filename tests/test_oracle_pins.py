"""Pins of the FP64 oracle against closed forms, exact identities, brute force on
tiny grids and library special cases (no GPU needed).

Each test names the property of the method it fixes; a plausible slip in the
oracle (a dropped term, a wrong sign, a transposed operand, a wrong Coriolis
factor, a misplaced wall) breaks at least one of them.
"""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.special

from oracle import tdwp_oracle as O
from workloads import asymptotic_potential, config, ev
from workloads import pes as PES


def tiny_spec(J=0, omega_max=0, n_elec=1, n_R=7, n_r=6, n_gamma=5, rot_cut=None, rad_cut=None,
              couplings=None):
    s = config(1)
    s.update(n_R=n_R, n_r=n_r, n_gamma=n_gamma, n_elec=n_elec)
    s["units"] = [dict(J=J, parity=(-1) ** J, omega_max=omega_max, n_packets=1)]
    if n_elec > 1:
        s["pes"]["shifts"] = [0.0, ev(0.5), ev(1.0)][:n_elec]
        s["pes"]["couplings"] = couplings if couplings is not None else {(0, 1): ev(0.1)}
    if rot_cut is not None:
        s["rot_cut"] = rot_cut
    if rad_cut is not None:
        s["rad_cut"] = rad_cut
    return s


# P1 -- Gauss-Legendre quadrature ---------------------------------------------------------

@pytest.mark.parametrize("n", [5, 24, 80])
def test_gauss_legendre_exact_for_polynomials(n):
    x, w = O.gauss_legendre(n)
    assert np.all(np.diff(x) > 0)
    assert abs(w.sum() - 2.0) < 1e-13
    for p in range(0, 2 * n):
        exact = 0.0 if p % 2 else 2.0 / (p + 1)
        assert abs(np.sum(w * x ** p) - exact) < 1e-12 * max(1.0, n / 10)


# P2 -- normalised associated Legendre tables -----------------------------------------------

@pytest.mark.parametrize("n,omega", [(24, 0), (24, 1), (24, 2), (24, 5), (80, 0), (64, 8), (96, 4)])
def test_legendre_table_orthonormal(n, omega):
    x, w = O.gauss_legendre(n)
    P = O.legendre_table(n - 1, omega, x, w)
    assert P.shape == (n - omega, n)
    assert np.max(np.abs(P @ P.T - np.eye(n - omega))) < 2e-13


@pytest.mark.parametrize("omega", [0, 1, 2, 3])
def test_legendre_matches_scipy_without_condon_shortley(omega):
    x = np.linspace(-0.97, 0.98, 13)
    mine = O.assoc_legendre_normalised(12, omega, x)
    for idx, j in enumerate(range(omega, 13)):
        norm = math.sqrt((2 * j + 1) / 2.0 * math.factorial(j - omega) / math.factorial(j + omega))
        ref = (-1) ** omega * scipy.special.lpmv(omega, j, x) * norm
        assert np.max(np.abs(mine[idx] - ref)) < 1e-12


# P3 -- sine DVR ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [6, 48, 193])
def test_sine_dvr_orthogonal_involution(n):
    S = O.sine_dvr(n)
    assert np.max(np.abs(S @ S - np.eye(n))) < 1e-13


@pytest.mark.parametrize("n", [6, 48, 64])
def test_sine_kinetic_equals_colbert_miller_closed_form(n):
    """Uncapped S diag(k^2/2M) S equals the particle-in-a-box sine-DVR formula
    obtained by summing the finite trigonometric series (Colbert & Miller 1992)."""
    M, L = 1224.6, 8.3
    T, _ = O.sine_kinetic(n, L, M, cap=0.0)
    Np = n + 1
    pref = (1.0 / (2 * M)) * (math.pi ** 2 / L ** 2) / 2.0
    ref = np.empty((n, n))
    for i in range(1, n + 1):
        for k in range(1, n + 1):
            if i == k:
                ref[i - 1, k - 1] = pref * ((2 * Np * Np + 1) / 3.0 - 1.0 / math.sin(math.pi * i / Np) ** 2)
            else:
                ref[i - 1, k - 1] = pref * (-1) ** (i - k) * (
                    1.0 / math.sin(math.pi * (i - k) / (2 * Np)) ** 2
                    - 1.0 / math.sin(math.pi * (i + k) / (2 * Np)) ** 2)
    assert np.max(np.abs(T - ref)) < 1e-10 * np.max(np.abs(ref))


def test_sine_kinetic_cap_only_clips_eigenvalues():
    T, e = O.sine_kinetic(40, 7.0, 1000.0, cap=0.01)
    ev_ = np.linalg.eigvalsh(T)
    assert np.max(ev_) <= 0.01 + 1e-14
    assert np.allclose(np.sort(ev_), np.sort(e), atol=1e-13)


# P4 -- l^2 with the Coriolis coupling ------------------------------------------------------

@pytest.mark.parametrize("J,j", [(1, 1), (3, 2), (5, 5), (20, 7), (4, 9), (0, 3)])
def test_ell2_spectrum_is_l_l_plus_1(J, j):
    """With the full Omega range the parity-adapted block of l^2 has eigenvalues
    l(l+1), |J-j| <= l <= J+j; the block containing Omega = 0 takes (j + l - J) even."""
    om, L = O.ell2_matrix(J, j, list(range(0, J + 1)))
    got = np.sort(np.linalg.eigvalsh(L))
    ls = [l for l in range(abs(J - j), J + j + 1) if (j + l - J) % 2 == 0]
    assert len(ls) == len(om)
    assert np.allclose(got, np.sort([l * (l + 1) for l in ls]), atol=1e-9)
    if J >= 1 and j >= 1:
        om1, L1 = O.ell2_matrix(J, j, list(range(1, J + 1)))
        ls1 = [l for l in range(abs(J - j), J + j + 1) if (j + l - J) % 2 == 1]
        assert np.allclose(np.sort(np.linalg.eigvalsh(L1)), np.sort([l * (l + 1) for l in ls1]), atol=1e-9)


# P5 -- diatomic solve against analytic Morse levels ----------------------------------------

def test_morse_levels_on_propagation_grid():
    s = config(1)
    s["v_cut"] = 0.0
    s["rad_cut"] = 0.0
    op = O.Operator(s)
    pes = s["pes"]
    va = PES.morse_singlet(op.r, pes["De"], pes["a"], pes["re"]) + pes["De"]
    e, chi = O.diatomic_states(op, va, 0, 4)
    De, a = pes["De"], pes["a"]
    w = a * math.sqrt(2 * De / op.m)
    exact = np.array([w * (v + 0.5) - w * w * (v + 0.5) ** 2 / (4 * De) for v in range(4)])
    assert abs(w * 27.211386245988 - 0.47929) < 1e-4
    assert np.max(np.abs(e - exact)) * 27.211386245988 * 1000 < 0.05      # meV
    # eigen-equation residual and sign convention
    Hd = op.Tr + np.diag(va)
    for v in range(4):
        assert np.linalg.norm(Hd @ chi[v] - e[v] * chi[v]) < 1e-12
        first = np.nonzero(np.abs(chi[v]) > 1e-3 * np.abs(chi[v]).max())[0][0]
        assert chi[v][first] > 0


# P6, P7 -- assembled H on a tiny grid --------------------------------------------------------

@pytest.mark.parametrize("J,omega_max,n_elec,capped", [(0, 0, 1, True), (3, 2, 2, True), (3, 2, 2, False),
                                                       (2, 2, 3, True)])
def test_dense_H_symmetric_and_bounded(J, omega_max, n_elec, capped):
    s = tiny_spec(J=J, omega_max=omega_max, n_elec=n_elec,
                  rot_cut=None if capped else 0.0, rad_cut=None if capped else 0.0)
    op = O.Operator(s)
    H = O.dense_H(op, 0)
    assert np.max(np.abs(H - H.T)) < 1e-14 * np.max(np.abs(H))
    lam = np.linalg.eigvalsh(H)
    assert lam[0] >= op.Emin - 1e-12 and lam[-1] <= op.Emax + 1e-12


def test_uncapped_angular_block_equals_l2_operator():
    """Caps off: the DVR angular term equals P^T [j(j+1) B_r + B_R l^2] P built by hand."""
    s = tiny_spec(J=2, omega_max=1, rot_cut=0.0, rad_cut=0.0, n_gamma=4)
    s["v_cut"] = 0.0
    op = O.Operator(s)
    rng = np.random.default_rng(7)
    u = rng.standard_normal(op.unit_shape(0))
    h = O.apply_H(op, 0, u) - (u @ op.Tr) - np.matmul(op.TR, u) - op.V[0][None, None] * u
    oms = O.omega_range(s["units"][0])
    ref = np.zeros_like(u)
    i, m = 2, 3
    for j in range(op.jmax + 1):
        om, L = O.ell2_matrix(2, j, oms)
        for a, oa in enumerate(om):
            for b, ob in enumerate(om):
                coef = op.BR[m] * L[a, b] + (op.Br[i] * j * (j + 1) if a == b else 0.0)
                ref[oms.index(oa), 0, :, m, i] += coef * op.P[oa][j - oa] * (op.P[ob][j - ob] @ u[oms.index(ob), 0, :, m, i])
    assert np.max(np.abs(h[:, :, :, m, i] - ref[:, :, :, m, i])) < 1e-13 * np.max(np.abs(ref))


# P8 -- undamped recursion equals Chebyshev polynomials of H_s -------------------------------

def test_undamped_recursion_is_chebyshev_polynomial():
    s = tiny_spec(J=2, omega_max=1, n_elec=2)
    op = O.Operator(s)
    H = O.dense_H(op, 0)
    Hs = (H - op.E0 * np.eye(len(H))) / op.dE
    lam, V = np.linalg.eigh(Hs)
    rng = np.random.default_rng(7)
    u0 = rng.standard_normal(op.unit_shape(0))
    u0 /= np.linalg.norm(u0)
    K = 60
    run = O.propagate(op, 0, u0, K, keep_vectors="all", undamped=True)
    for k in (0, 1, 2, 7, 33, 60):
        ref = V @ (np.cos(k * np.arccos(lam)) * (V.T @ u0.ravel()))
        assert np.max(np.abs(run["vectors"][k].ravel() - ref)) < 1e-12


# P9 -- time reconstruction from Chebyshev components ---------------------------------------

def test_time_reconstruction_matches_exact_propagator():
    s = tiny_spec(J=1, omega_max=1)
    op = O.Operator(s)
    H = O.dense_H(op, 0)
    rng = np.random.default_rng(7)
    u0 = rng.standard_normal(op.unit_shape(0))
    u0 /= np.linalg.norm(u0)
    t = 40.0
    K = int(t * op.dE) + 60
    run = O.propagate(op, 0, u0, K, keep_vectors="all", undamped=True)
    vecs = np.array([run["vectors"][k] for k in range(K + 1)])
    psi = O.time_reconstruct(op, vecs, t).ravel()
    ref = scipy.linalg.expm(-1j * H * t) @ u0.ravel()
    assert np.max(np.abs(psi - ref)) < 1e-11
    assert abs(np.linalg.norm(psi) - 1.0) < 1e-11


# P10 -- damped energy accumulation: exact generating-function identity -----------------------

def test_damped_energy_sum_equals_resolvent():
    """sum_k c_k u_k = (1/(dE sin th)) (I - 2 z D H_s + z^2 D^2)^-1 (I - z^2 D^2) u_0, z = e^{-i th},
    derived from Eq. wvp-k; the damping here is strong everywhere so the series converges."""
    s = tiny_spec(J=2, omega_max=1, n_elec=2)
    op = O.Operator(s)
    shape = op.unit_shape(0)
    rng = np.random.default_rng(7)
    Dfull = rng.uniform(0.80, 0.95, size=shape)
    u0 = rng.standard_normal(shape)
    K = 900
    run = O.propagate(op, 0, u0, K, keep_vectors="all", damping=Dfull)
    vecs = np.array([run["vectors"][k].ravel() for k in range(K + 1)])
    H = O.dense_H(op, 0)
    n = len(H)
    Hs = (H - op.E0 * np.eye(n)) / op.dE
    Dd = np.diag(Dfull.ravel())
    for E in (op.E0 - 0.7 * op.dE, op.E0 + 0.1 * op.dE, op.E0 + 0.93 * op.dE):
        c = O.chebyshev_energy_coeffs(op, np.array([E]), K)[0]
        got = c @ vecs
        th = math.acos((E - op.E0) / op.dE)
        z = np.exp(-1j * th)
        M = np.eye(n) - 2 * z * Dd @ Hs + z * z * Dd @ Dd
        ref = np.linalg.solve(M, (np.eye(n) - z * z * Dd @ Dd) @ u0.ravel()) / (op.dE * math.sin(th))
        assert np.max(np.abs(got - ref)) < 1e-11 * np.max(np.abs(ref))


# Flux interpolation rows: exact on the sine basis ----------------------------------------------

@pytest.mark.parametrize("nb", [1, 5, 17])
def test_flux_rows_interpolate_sine_basis_exactly(nb):
    s = config(1)
    op = O.Operator(s)
    rs = 4.61
    a, d = O.flux_rows(op, rs)
    L, r0 = op.Lr, op.r_wall
    kn = nb * math.pi / L
    f = math.sqrt(2 / L) * np.sin(kn * (op.r - r0))
    u = math.sqrt(op.dr) * f
    assert abs(a @ u - math.sqrt(2 / L) * math.sin(kn * (rs - r0))) < 1e-13
    assert abs(d @ u - math.sqrt(2 / L) * kn * math.cos(kn * (rs - r0))) < 1e-12 * max(1, kn)


# P17 -- LEPS fixture -------------------------------------------------------------------------

def test_leps_limits_and_symmetry():
    s = config(1)
    p = s["pes"]
    r = np.linspace(0.9, 4.0, 7)
    far = PES.leps(np.full_like(r, 60.0), r, np.full_like(r, 60.5), p["De"], p["a"], p["re"], p["sato"])
    assert np.max(np.abs(far - PES.morse_singlet(r, p["De"], p["a"], p["re"]))) < 1e-14
    rng = np.random.default_rng(7)
    d = rng.uniform(1.0, 4.0, size=(3, 20))
    v = PES.leps(d[0], d[1], d[2], p["De"], p["a"], p["re"], p["sato"])
    for perm in ((1, 2, 0), (2, 0, 1), (0, 2, 1)):
        assert np.max(np.abs(v - PES.leps(d[perm[0]], d[perm[1]], d[perm[2]], p["De"], p["a"], p["re"], p["sato"]))) < 1e-15
    s["v_cut"] = 0.0
    va = asymptotic_potential(s, r, 0)
    tab = PES.diabatic_matrix(s, r, 80.0, 0.3)[0]
    assert np.max(np.abs(va - tab)) < 1e-12


# P19 -- J > 0 with a single helicity is J = 0 shifted by B_R J(J+1) ----------------------------

def test_single_helicity_is_centrifugal_shift():
    s0 = tiny_spec(J=0, omega_max=0, rot_cut=0.0)
    s3 = tiny_spec(J=3, omega_max=0, rot_cut=0.0)
    op0, op3 = O.Operator(s0, bounds=(0.0, 1.0)), O.Operator(s3, bounds=(0.0, 1.0))
    rng = np.random.default_rng(7)
    u = rng.standard_normal(op0.unit_shape(0))
    d = O.apply_H(op3, 0, u) - O.apply_H(op0, 0, u)
    assert np.max(np.abs(d - 12 * op0.BR[None, None, None, :, None] * u)) < 1e-13


# P20 -- decoupled diabatic states ------------------------------------------------------------

def test_uncoupled_second_state_stays_empty_and_first_matches_single_state():
    s2 = tiny_spec(J=2, omega_max=1, n_elec=2, couplings={})
    s1 = tiny_spec(J=2, omega_max=1, n_elec=1)
    op2 = O.Operator(s2, bounds=(0.0, 1.0))
    op1 = O.Operator(s1, bounds=(0.0, 1.0))
    rng = np.random.default_rng(7)
    u1 = rng.standard_normal(op1.unit_shape(0))
    u2 = np.zeros(op2.unit_shape(0))
    u2[:, 0] = u1[:, 0]
    r2 = O.propagate(op2, 0, u2, 30, keep_vectors=(30,))
    r1 = O.propagate(op1, 0, u1, 30, keep_vectors=(30,))
    assert np.max(np.abs(r2["vectors"][30][:, 1])) == 0.0
    assert np.max(np.abs(r2["vectors"][30][:, 0] - r1["vectors"][30][:, 0])) < 1e-13


# P4 continued -- the capped branch of the angular term (several helicities) ------------------

def _angular_part(op, u):
    """Angular + Coriolis part of H u (H u minus the radial kinetic and potential terms)."""
    h = O.apply_H(op, 0, u) - (u @ op.Tr) - np.matmul(op.TR, u)
    for p, (la, lb) in enumerate(op.pairs):
        h[:, la] -= op.V[p][None] * u[:, lb]
        if la != lb:
            h[:, lb] -= op.V[p][None] * u[:, la]
    return h


def _fbr_block(op, unit, j, m, i):
    """The matrix of the angular term on the FBR coefficients c[Omega][j] at the grid
    point (R_m, r_i), over the helicities Omega <= j of the unit: column b is the
    FBR image of the DVR vector whose only coefficient is (Omega_b, j)."""
    oms = O.omega_range(unit)
    om = [o for o in oms if o <= j]
    A = np.zeros((len(om), len(om)))
    for b, ob in enumerate(om):
        u = np.zeros(op.unit_shape(0))
        u[oms.index(ob), 0, :, m, i] = op.P[ob][j - ob]
        h = _angular_part(op, u)
        for a, oa in enumerate(om):
            A[a, b] = op.P[oa][j - oa] @ h[oms.index(oa), 0, :, m, i]
    return om, A


def test_capped_branch_with_cap_above_spectrum_equals_l2_operator():
    """rot_cut above every block eigenvalue: the capped branch (eigenvectors of the
    l^2 block) must reproduce B_r j(j+1) + B_R l^2 built by hand at every point and j;
    an eigenvector matrix applied transposed fails this."""
    s = tiny_spec(J=4, omega_max=3, rot_cut=50.0, rad_cut=0.0, n_gamma=6, n_R=5, n_r=4)
    s["v_cut"] = 0.0
    op = O.Operator(s)
    oms = O.omega_range(s["units"][0])
    assert oms == [0, 1, 2, 3]
    rng = np.random.default_rng(7)
    u = rng.standard_normal(op.unit_shape(0))
    h = _angular_part(op, u)
    ref = np.zeros_like(u)
    for m in range(s["n_R"]):
        for i in range(s["n_r"]):
            for j in range(op.jmax + 1):
                om, L = O.ell2_matrix(4, j, oms)
                for a, oa in enumerate(om):
                    for b, ob in enumerate(om):
                        coef = op.BR[m] * L[a, b] + (op.Br[i] * j * (j + 1) if a == b else 0.0)
                        ref[oms.index(oa), 0, :, m, i] += coef * op.P[oa][j - oa] * (
                            op.P[ob][j - ob] @ u[oms.index(ob), 0, :, m, i])
    assert np.max(np.abs(h - ref)) < 1e-13 * np.max(np.abs(ref))


def test_biting_cap_clips_closed_form_eigenvalues_of_each_block():
    """A cap inside the block spectra: each (R_m, r_i, j) block of the angular term has
    eigenvalues min(B_r j(j+1) + B_R l(l+1), rot_cut) with l(l+1) from the closed form
    (|J-j| <= l <= J+j, (j + l - J) even for the block holding Omega = 0), and it is a
    function of the l^2 block (it commutes with it)."""
    J = 3
    s = tiny_spec(J=J, omega_max=J, rad_cut=0.0, n_gamma=6, n_R=5, n_r=4)
    s["v_cut"] = 0.0
    probe = O.Operator(dict(s, rot_cut=0.0))
    m, i = 1, 2
    levels = sorted(probe.Br[i] * j * (j + 1) + probe.BR[m] * l * (l + 1)
                    for j in range(probe.jmax + 1) for l in range(abs(J - j), J + j + 1))
    cap = levels[len(levels) // 2]
    s["rot_cut"] = cap
    op = O.Operator(s)
    oms = O.omega_range(s["units"][0])
    bitten = kept = 0
    for j in range(op.jmax + 1):
        om, A = _fbr_block(op, s["units"][0], j, m, i)
        if not om:
            continue
        ls = [l for l in range(abs(J - j), J + j + 1) if (j + l - J) % 2 == 0]
        assert len(ls) == len(om)
        exact = np.sort([min(op.Br[i] * j * (j + 1) + op.BR[m] * l * (l + 1), cap) for l in ls])
        assert np.max(np.abs(np.sort(np.linalg.eigvalsh(0.5 * (A + A.T))) - exact)) < 1e-13 * cap
        assert np.max(np.abs(A - A.T)) < 1e-14 * cap
        _, L = O.ell2_matrix(J, j, oms)
        assert np.max(np.abs(A @ L - L @ A)) < 1e-12 * cap * np.max(np.abs(L))
        bitten += int(np.sum(exact >= cap))
        kept += int(np.sum(exact < cap))
    assert bitten > 0 and kept > 0


# P11 -- free spreading of a Gaussian (kinetic terms, time reconstruction) ---------------------

def test_free_gaussian_spreads_analytically():
    """V = 0, J = 0, caps and absorbers off: a Gaussian amplitude exp(-(x-x0)^2 / 2 G^2)
    in R and in r keeps its form and its width grows as G sqrt(1 + (t / (M G^2))^2),
    with M = mu along R and m along r, until it reaches the walls.  Psi(t) comes from
    the undamped Chebyshev components (Eq. chebyshev-expansion-constants)."""
    s = config(1)
    s.update(n_R=72, n_r=60, n_gamma=3, rad_cut=0.0, rot_cut=0.0, v_cut=0.0)
    s["units"] = [dict(J=0, parity=1, omega_max=0, n_packets=1)]
    shape = (1, 1, 3, 72, 60)
    op = O.Operator(s, vtable=np.zeros((1,) + shape[2:]))
    GR, Gr, R0, r0 = 0.6, 0.55, 6.25, 4.25
    pk = dict(unit=0, slot=0, v0=0, j0=0, omega0=0, elec0=0, R0=R0, width=GR, ecol_mean=0.0)
    chi = np.sqrt(op.dr) * np.exp(-((op.r - r0) ** 2) / (2 * Gr * Gr))
    u0 = O.initial_packet(op, 0, pk, chi)
    t_max = 700.0
    K = int(t_max * op.dE * 1.1) + 80
    run = O.propagate(op, 0, u0, K, keep_vectors="all", undamped=True)
    vecs = np.array([run["vectors"][k] for k in range(K + 1)])
    for t in (0.0, 150.0, 400.0, 700.0):
        psi = O.time_reconstruct(op, vecs, t)
        dens = np.abs(psi[0, 0]) ** 2                      # (gamma, R, r)
        assert abs(dens.sum() - 1.0) < 1e-10
        for axis, x, M, G, t_lim in ((1, op.R, op.mu, GR, 700.0), (2, op.r, op.m, Gr, 400.0)):
            if t > t_lim:
                continue
            p = dens.sum(axis=tuple(a for a in range(3) if a != axis))
            mean = float(p @ x)
            var = float(p @ (x - mean) ** 2)
            want = 0.5 * (G * math.sqrt(1.0 + (t / (M * G * G)) ** 2)) ** 2
            assert abs(var - want) < 1e-7 * want, (t, axis, var, want)
