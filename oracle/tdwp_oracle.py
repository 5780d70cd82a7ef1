"""FP64 CPU oracle for the damped real Chebyshev wave-packet method.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the GPU library and imports nothing from it.

Plain and slow on purpose: every operator is a dense per-axis matrix applied
with numpy matmul/einsum, every sum is written as its definition.  All
quantities are in atomic units (hbar = 1, bohr, hartree, electron masses).

Notation follows arXiv 2412.10167 (MADWAVE3):
  Jacobi coordinates (r, R, gamma), helicity Omega, diabatic state Lambda
  (Sec. 2.1, Eqs. total-function, angular-functions, hamiltonian);
  modified Chebyshev recursion with damping e^{-phi} (Sec. 2.2, Eq. wvp-k,
  Eq. imaginary-potential); energy-domain coefficients c_k (Eq.
  chebyshev-expansion-constants); collision packet (Sec. 2.3.1, Eqs.
  initial-collision-wvp, initial-gaussian, initial-flux-collisions); total
  flux (Eq. total-flux) and S-matrix from Chebyshev projections (Eqs.
  Chebyshev-products-overlaps, S-matrix-from-chebyshev).

Readings where the paper is silent or garbled (each also listed in the design
notes): DST-I sine DVR with walls one step outside the first and last points;
radial and rotational caps applied to FBR eigenvalues; rigorous Gershgorin
spectral bounds; FBR range j = Omega..n_gamma-1; normalised associated Legendre
functions without the Condon-Shortley phase; ascending Gauss-Legendre nodes;
and the Green's-function normalisation of the flux and S-matrix prefactors.

Parity is pinned for every function here by tests under tests/ (closed forms,
exact identities, brute force on tiny grids, physical invariants) except the
physical accuracy of P(E) on the synthetic surface, which nothing external
fixes ("parity unpinned" for that property alone; the invariants still bind).
"""
import math

import numpy as np


# ---------------------------------------------------------------------------
# Masses and grids (Sec. 2.1)
# ---------------------------------------------------------------------------

def reduced_masses(spec):
    """mu = m_A (m_B + m_C) / M and m = m_B m_C / (m_B + m_C) (Sec. 2.1, after Eq. hamiltonian)."""
    mA, mB, mC = spec["mass_A"], spec["mass_B"], spec["mass_C"]
    return mA * (mB + mC) / (mA + mB + mC), mB * mC / (mB + mC)


def radial_grid(xmin, xmax, n):
    """Equidistant points x_1..x_N from xmin to xmax; Dirichlet walls one step
    outside at x_0 and x_{N+1}; box length L = (N + 1) dx."""
    dx = (xmax - xmin) / (n - 1)
    x = xmin + dx * np.arange(n)
    wall = xmin - dx
    return x, dx, (n + 1) * dx, wall


def gauss_legendre(n):
    """Gauss-Legendre nodes cos(gamma_n) in ascending order and weights (Sec. 2.1)."""
    x, w = np.polynomial.legendre.leggauss(n)
    order = np.argsort(x)
    return x[order], w[order]


def assoc_legendre_normalised(jmax, omega, x):
    """Rows j = omega..jmax of the L2([-1,1])-normalised associated Legendre
    functions P~_{j omega}(x), without the Condon-Shortley phase.

    Unnormalised recurrence in j at fixed order, then the textbook norm
    sqrt((2j+1)/2 (j-omega)!/(j+omega)!)."""
    x = np.asarray(x, float)
    out = np.zeros((jmax - omega + 1, x.size))
    # P_omega^omega = (2 omega - 1)!! (1 - x^2)^{omega/2}
    dfact = 1.0
    for k in range(1, 2 * omega, 2):
        dfact *= k
    p_prev = dfact * (1.0 - x * x) ** (0.5 * omega)
    vals = [p_prev]
    if jmax > omega:
        p_cur = x * (2 * omega + 1) * p_prev
        vals.append(p_cur)
        for j in range(omega + 2, jmax + 1):
            p_next = (x * (2 * j - 1) * p_cur - (j + omega - 1) * p_prev) / (j - omega)
            p_prev, p_cur = p_cur, p_next
            vals.append(p_cur)
    for idx, j in enumerate(range(omega, jmax + 1)):
        lognorm = 0.5 * (math.log((2 * j + 1) / 2.0) + math.lgamma(j - omega + 1)
                         - math.lgamma(j + omega + 1))
        out[idx] = vals[idx] * math.exp(lognorm)
    return out


def legendre_table(jmax, omega, x, w):
    """P^Omega[j][n] = sqrt(w_n) P~_{j Omega}(x_n), j = Omega..jmax (DVR -> FBR, Sec. 2.1 item 3)."""
    return assoc_legendre_normalised(jmax, omega, x) * np.sqrt(w)[None, :]


def sine_dvr(n):
    """Orthogonal DST-I matrix S_{ni} = sqrt(2/(N+1)) sin(n pi i/(N+1)), n, i = 1..N."""
    k = np.arange(1, n + 1)
    return math.sqrt(2.0 / (n + 1)) * np.sin(np.pi * np.outer(k, k) / (n + 1))


def sine_kinetic(n, length, mass, cap):
    """-(1/2M) d^2/dx^2 in the sine DVR: S diag(min(k_n^2/2M, cap)) S, k_n = n pi / L
    (real sine transform of Sec. 2.1 item 2; radial cap radcutmaxeV of Table tab:parameters)."""
    S = sine_dvr(n)
    kn = np.pi * np.arange(1, n + 1) / length
    e = kn * kn / (2.0 * mass)
    if cap > 0:
        e = np.minimum(e, cap)
    return S @ np.diag(e) @ S, e


# ---------------------------------------------------------------------------
# Angular momentum in the body-fixed frame (Sec. 2.1: l^2 = J^2 + j^2 - 2 J.j)
# ---------------------------------------------------------------------------

def omega_range(unit):
    """Helicities in the expansion of Eq. total-function for Lambda = 0 states:
    Omega_min = 0 when p (-1)^J = +1 (else 1), up to omega_max."""
    lo = 0 if unit["parity"] * (-1) ** unit["J"] == 1 else 1
    return list(range(lo, unit["omega_max"] + 1))


def ell2_matrix(J, j, omegas):
    """<J Omega j| l^2 |J Omega' j> on the Omega list (with Omega <= j):
    diagonal J(J+1) + j(j+1) - 2 Omega^2, Coriolis coupling between Omega and
    Omega+1 equal to -lambda(J,Omega) lambda(j,Omega), times sqrt(2) between
    the parity-adapted Omega = 0 and 1 functions (1/sqrt(1+delta_{Omega 0})
    in Eq. angular-functions)."""
    om = [o for o in omegas if o <= j]
    n = len(om)
    L = np.zeros((n, n))

    def lam(a, o):
        return math.sqrt(max(a * (a + 1) - o * (o + 1), 0))
    for a, o in enumerate(om):
        L[a, a] = J * (J + 1) + j * (j + 1) - 2 * o * o
        if a + 1 < n:
            c = -lam(J, o) * lam(j, o) * (math.sqrt(2.0) if o == 0 else 1.0)
            L[a, a + 1] = L[a + 1, a] = c
    return om, L


# ---------------------------------------------------------------------------
# Operator set-up
# ---------------------------------------------------------------------------

class Operator:
    """Grids, per-axis matrices, angular blocks, damping and potential of one plan."""

    def __init__(self, spec, vtable=None, bounds=None):
        self.spec = spec
        self.mu, self.m = reduced_masses(spec)
        self.r, self.dr, self.Lr, self.r_wall = radial_grid(spec["r_min"], spec["r_max"], spec["n_r"])
        self.R, self.dR, self.LR, self.R_wall = radial_grid(spec["R_min"], spec["R_max"], spec["n_R"])
        self.x, self.w = gauss_legendre(spec["n_gamma"])
        self.jmax = spec["n_gamma"] - 1
        self.Tr, self.er = sine_kinetic(spec["n_r"], self.Lr, self.m, spec["rad_cut"])
        self.TR, self.eR = sine_kinetic(spec["n_R"], self.LR, self.mu, spec["rad_cut"])
        self.Br = 1.0 / (2.0 * self.m * self.r ** 2)
        self.BR = 1.0 / (2.0 * self.mu * self.R ** 2)
        om_all = sorted({o for u in spec["units"] for o in omega_range(u)})
        self.P = {o: legendre_table(self.jmax, o, self.x, self.w) for o in om_all}
        self.n_elec = spec["n_elec"]
        self.pairs = [(a, b) for a in range(self.n_elec) for b in range(a, self.n_elec)]
        if vtable is None:
            from workloads.pes import diabatic_matrix
            vtable = diabatic_matrix(spec, self.r[None, None, :], self.R[None, :, None],
                                     self.x[:, None, None])
        self.V = np.asarray(vtable, float).reshape(len(self.pairs), spec["n_gamma"],
                                                    spec["n_R"], spec["n_r"])
        self.D = np.exp(-absorber(self.r, spec["abs_r_start"], spec["abs_r_strength"], spec["abs_r_power"])[None, :]
                        - absorber(self.R, spec["abs_R_start"], spec["abs_R_strength"], spec["abs_R_power"])[:, None])
        if bounds is None:
            bounds = spectral_bounds(self)
        self.Emin, self.Emax = bounds
        self.E0 = 0.5 * (self.Emax + self.Emin)
        self.dE = 0.5 * (self.Emax - self.Emin)

    def unit_shape(self, u):
        unit = self.spec["units"][u]
        return (len(omega_range(unit)), self.n_elec, self.spec["n_gamma"], self.spec["n_R"], self.spec["n_r"])


def absorber(x, start, strength, power):
    """phi(x) = A (x - x_I)^n for x > x_I, zero before (Eq. imaginary-potential)."""
    d = np.maximum(x - start, 0.0)
    return np.where(x > start, strength * d ** power, 0.0)


def spectral_bounds(op):
    """(E_min, E_max) bracketing the spectrum of H on the grid (Sec. 2.2 text after Eq. wvp-k).

    Kinetic and angular terms are positive semi-definite, so E_min is the
    lowest Gershgorin bound of the per-point potential matrix; E_max adds the
    largest eigenvalue of every term."""
    s = op.spec
    n = op.n_elec
    diag = {}
    for p, (a, b) in enumerate(op.pairs):
        if a == b:
            diag[a] = op.V[p]
    offsum = [np.zeros_like(op.V[0]) for _ in range(n)]
    for p, (a, b) in enumerate(op.pairs):
        if a != b:
            offsum[a] = offsum[a] + np.abs(op.V[p])
            offsum[b] = offsum[b] + np.abs(op.V[p])
    vlo = min(float(np.min(diag[a] - offsum[a])) for a in range(n))
    vhi = max(float(np.max(diag[a] + offsum[a])) for a in range(n))
    ang = 0.0
    for unit in s["units"]:
        oms = omega_range(unit)
        for j in range(op.jmax + 1):
            om, L = ell2_matrix(unit["J"], j, oms)
            if not om:
                continue
            lmax = float(np.max(np.linalg.eigvalsh(L)))
            e = op.Br[0] * j * (j + 1) + op.BR[0] * lmax
            if s["rot_cut"] > 0:
                e = min(e, s["rot_cut"])
            ang = max(ang, e)
    return vlo, vhi + float(np.max(op.er)) + float(np.max(op.eR)) + ang


# ---------------------------------------------------------------------------
# H . u  (Eq. hamiltonian applied term by term, Sec. 2.1 items 1-5)
# ---------------------------------------------------------------------------

def apply_H(op, unit_index, u):
    """H u for one packet of unit `unit_index`; u has shape (n_Omega, n_Lambda, n_gamma, n_R, n_r)."""
    s = op.spec
    unit = s["units"][unit_index]
    oms = omega_range(unit)
    J = unit["J"]
    h = u @ op.Tr                              # -(1/2m) d^2/dr^2 along r (Tr symmetric)
    h = h + np.matmul(op.TR, u)                # -(1/2mu) d^2/dR^2 along R
    # Angular terms in the FBR: c[Omega][j] = sum_n P^Omega[j][n] u[Omega][n]
    c = {o: np.einsum("jn,lnmi->ljmi", op.P[o], u[a]) for a, o in enumerate(oms)}
    d = {o: np.zeros_like(c[o]) for o in oms}
    for j in range(op.jmax + 1):
        om, L = ell2_matrix(J, j, oms)
        if not om:
            continue
        cj = np.stack([c[o][:, j - o] for o in om])          # (n_om, n_Lambda, n_R, n_r)
        rot = op.Br[None, :] * j * (j + 1)                    # j^2/(2 m r^2) on (R, r)
        if s["rot_cut"] > 0:
            ell, U = np.linalg.eigh(L)
            e = rot[None, :, :] + op.BR[None, :, None] * ell[:, None, None]
            e = np.minimum(e, s["rot_cut"])                   # capped rotational energy
            t = np.einsum("oa,olmi->almi", U, cj)
            t = t * e[:, None, :, :]
            dj = np.einsum("oa,almi->olmi", U, t)
        else:
            dj = cj * rot[None, None] + np.einsum("op,plmi->olmi", L, cj) * op.BR[None, None, :, None]
        for a, o in enumerate(om):
            d[o][:, j - o] = dj[a]
    for a, o in enumerate(oms):
        h[a] = h[a] + np.einsum("jn,ljmi->lnmi", op.P[o], d[o])
    # Diabatic potential matrix, diagonal in the grid (Sec. 2.1 item 5)
    for p, (la, lb) in enumerate(op.pairs):
        h[:, la] = h[:, la] + op.V[p][None] * u[:, lb]
        if la != lb:
            h[:, lb] = h[:, lb] + op.V[p][None] * u[:, la]
    return h


def apply_Hs(op, unit_index, u):
    """Scaled Hamiltonian H_s = (H - E0)/dE (Sec. 2.2)."""
    return (apply_H(op, unit_index, u) - op.E0 * u) / op.dE


def dense_H(op, unit_index):
    """H assembled column by column by acting on unit vectors (tiny grids only)."""
    shape = op.unit_shape(unit_index)
    n = int(np.prod(shape))
    H = np.empty((n, n))
    e = np.zeros(n)
    for i in range(n):
        e[:] = 0.0
        e[i] = 1.0
        H[:, i] = apply_H(op, unit_index, e.reshape(shape)).ravel()
    return H


# ---------------------------------------------------------------------------
# Diatomic channel functions (preparatory stage, Sec. 4)
# ---------------------------------------------------------------------------

def diatomic_states(op, v_asym, j, n_states):
    """Lowest n_states eigenpairs of T_r + V_asym(r) + min(j(j+1)/(2 m r^2), rotcut)
    on the propagation r grid; vectors DVR-normalised (sum chi_i^2 = 1) with the
    first component above 1e-3 of the maximum made positive."""
    rot = op.Br * j * (j + 1)
    if op.spec["rot_cut"] > 0:
        rot = np.minimum(rot, op.spec["rot_cut"])
    Hd = op.Tr + np.diag(np.asarray(v_asym, float) + rot)
    e, vecs = np.linalg.eigh(Hd)
    chis = []
    for v in range(n_states):
        c = vecs[:, v].copy()
        first = np.nonzero(np.abs(c) > 1e-3 * np.max(np.abs(c)))[0][0]
        if c[first] < 0:
            c = -c
        chis.append(c / np.linalg.norm(c))
    return e[:n_states].copy(), np.array(chis)


# ---------------------------------------------------------------------------
# Initial collision packet (Sec. 2.3.1)
# ---------------------------------------------------------------------------

def gaussian_R(op, packet):
    """DVR-weighted, unit-normalised g_m = sqrt(dR) g(R_m) with
    g(R) ~ exp(-(R-R0)^2 / (2 Gamma^2)) [e^{-i k0 R} + e^{i k0 R}] (Eq. initial-gaussian),
    k0 = sqrt(2 mu E_mean)."""
    k0 = math.sqrt(2.0 * op.mu * packet["ecol_mean"])
    g = np.exp(-((op.R - packet["R0"]) ** 2) / (2.0 * packet["width"] ** 2)) * 2.0 * np.cos(k0 * op.R)
    g = math.sqrt(op.dR) * g
    return g / np.linalg.norm(g)


def initial_packet(op, unit_index, packet, chi0):
    """u_0 = W_{Omega0 Lambda0} chi_{v0 j0}(r) Y_{j0 Omega0}(gamma) g(R) (Eq. initial-collision-wvp)
    in the DVR: P^{Omega0}[j0][n] g_m chi_i in block (Omega0, Lambda0), unit norm."""
    shape = op.unit_shape(unit_index)
    oms = omega_range(op.spec["units"][unit_index])
    u = np.zeros(shape)
    o0, j0 = packet["omega0"], packet["j0"]
    pj = op.P[o0][j0 - o0]
    pj = pj / np.linalg.norm(pj)
    chi = np.asarray(chi0, float)
    chi = chi / np.linalg.norm(chi)
    g = gaussian_R(op, packet)
    u[oms.index(o0), packet["elec0"]] = pj[:, None, None] * g[None, :, None] * chi[None, None, :]
    return u


def ghat(op, g, K):
    """Continuous Fourier amplitude int dR e^{iKR} g(R) of the unit-normalised g (Eq. initial-flux-collisions)."""
    K = np.atleast_1d(K)
    return np.exp(1j * np.outer(K, op.R)) @ (math.sqrt(op.dR) * g)


# ---------------------------------------------------------------------------
# Slices for the flux and the channel projections
# ---------------------------------------------------------------------------

def flux_rows(op, r_star):
    """Rows a_i, d_i giving Phi(r*) and dPhi/dr(r*) from DVR coefficients via the
    sine basis sqrt(2/L) sin(n pi (r - r_wall)/L)."""
    n = op.spec["n_r"]
    S = sine_dvr(n)
    kn = np.pi * np.arange(1, n + 1) / op.Lr
    phi = math.sqrt(2.0 / op.Lr) * np.sin(kn * (r_star - op.r_wall))
    dphi = math.sqrt(2.0 / op.Lr) * kn * np.cos(kn * (r_star - op.r_wall))
    return S.T @ phi, S.T @ dphi


def r_inf_index(op):
    """Grid index of R nearest to R_inf."""
    return int(math.floor((op.spec["R_inf"] - op.spec["R_min"]) / op.dR + 0.5))


# ---------------------------------------------------------------------------
# Modified Chebyshev recursion (Eq. wvp-k)
# ---------------------------------------------------------------------------

def propagate(op, unit_index, u0, K, keep_vectors=(), undamped=False, damping=None,
              extra_r_flux=(), line_fn=None):
    """Chebyshev components u_0..u_K with norms and per-k slices.

    u_1 = D H_s u_0;  u_{k+1} = D (2 H_s u_k - D u_{k-1});  D = e^{-phi}.
    `damping` replaces D by any array broadcastable to u (tests); `undamped`
    sets D = 1.  Returns dict with norms[k], s_val[k], s_der[k] (flux line at
    r*; one more pair per entry of extra_r_flux in `extra`), w[k] (R_inf line
    / sqrt(dR)), lines[k] = line_fn(u_k) when line_fn is given (another
    analysis line, e.g. a product arrangement's), and the vectors u_k for k in
    keep_vectors ("all" keeps every one)."""
    if damping is not None:
        D = damping
    else:
        D = np.ones_like(op.D) if undamped else op.D
    a_row, d_row = flux_rows(op, op.spec["r_flux"])
    extra_rows = [flux_rows(op, rs) for rs in extra_r_flux]
    mi = r_inf_index(op)
    out = dict(norms=np.empty(K + 1), s_val=[], s_der=[], w=[], vectors={},
               extra=[([], []) for _ in extra_rows], lines=[])

    def record(k, u):
        out["norms"][k] = float(np.sum(u * u))
        out["s_val"].append(u @ a_row)
        out["s_der"].append(u @ d_row)
        for (lv, ld), (ar, dr) in zip(out["extra"], extra_rows):
            lv.append(u @ ar)
            ld.append(u @ dr)
        out["w"].append(u[:, :, :, mi, :] / math.sqrt(op.dR))
        if line_fn is not None:
            out["lines"].append(line_fn(u))
        if keep_vectors == "all" or k in keep_vectors:
            out["vectors"][k] = u.copy()

    record(0, u0)
    if K == 0:
        return _stack(out)
    u_prev = u0
    u = D * apply_Hs(op, unit_index, u0)
    record(1, u)
    for k in range(1, K):
        u_next = D * (2.0 * apply_Hs(op, unit_index, u) - D * u_prev)
        u_prev, u = u, u_next
        record(k + 1, u)
    return _stack(out)


def _stack(out):
    for key in ("s_val", "s_der", "w", "lines"):
        out[key] = np.array(out[key])
    out["extra"] = [(np.array(lv), np.array(ld)) for lv, ld in out["extra"]]
    return out


# ---------------------------------------------------------------------------
# Energy-domain analysis (Eqs. wvf-chebyshev, chebyshev-expansion-constants,
# total-flux, Chebyshev-products-overlaps, S-matrix-from-chebyshev)
# ---------------------------------------------------------------------------

def collision_energies(spec):
    n = spec["n_energy"]
    return spec["ecol_min"] + (spec["ecol_max"] - spec["ecol_min"]) * np.arange(n) / (n - 1)


def chebyshev_energy_coeffs(op, E_tot, K):
    """c_k(E) = (2 - delta_k0) e^{-i k theta} / (dE sin theta), theta = arccos E_s, k = 0..K."""
    Es = (np.asarray(E_tot) - op.E0) / op.dE
    theta = np.arccos(Es)
    k = np.arange(K + 1)
    ph = np.outer(theta, k)
    c = (np.cos(ph) - 1j * np.sin(ph)) / (op.dE * np.sin(theta))[:, None]
    c[:, 1:] *= 2.0
    return c


def analyse(op, unit_index, packet, run, E_v0j0, channels=(), flux_slices=None):
    """Reactive flux per Lambda and inelastic |S|^2 per channel on the collision-energy grid.

    channels: sequence of dicts (elec, v, j, omega, energy, chi[n_r]).
    Returns dict(p_reac [n_elec][n_E], p_inel [n_ch][n_E])."""
    s = op.spec
    ecol = collision_energies(s)
    E_tot = ecol + E_v0j0
    K = run["norms"].size - 1
    c = chebyshev_energy_coeffs(op, E_tot, K)                          # (n_E, K+1)
    nE = ecol.size
    # Phi(E) = sum_k c_k s_k (energy-resolved slices)
    s_val, s_der = (run["s_val"], run["s_der"]) if flux_slices is None else flux_slices
    phi_v = (c @ s_val.reshape(K + 1, -1)).reshape((nE,) + s_val.shape[1:])   # (E, Om, Lam, gam, R)
    phi_d = (c @ s_der.reshape(K + 1, -1)).reshape((nE,) + s_der.shape[1:])
    g = gaussian_R(op, packet)
    K0 = np.sqrt(2.0 * op.mu * ecol)
    gh = ghat(op, g, K0)
    flux = np.imag(np.conj(phi_v) * phi_d).sum(axis=(1, 3, 4)) / op.m  # (E, Lam)
    p_reac = (K0[:, None] * flux / (op.mu * np.abs(gh)[:, None] ** 2)).T
    oms = omega_range(s["units"][unit_index])
    mi = r_inf_index(op)
    R_inf = op.R[mi]
    p_inel = np.zeros((len(channels), nE))
    for f, ch in enumerate(channels):
        o = ch["omega"]
        if o not in oms or ch["j"] < o:
            continue
        pj = op.P[o][ch["j"] - o]
        Cf = np.einsum("kni,n,i->k", run["w"][:, oms.index(o), ch["elec"]], pj, np.asarray(ch["chi"]))
        initial = (ch["elec"] == packet["elec0"] and ch["v"] == packet["v0"] and ch["j"] == packet["j0"]
                   and o == packet["omega0"])
        kf = packet.get("k_min_elastic", 0) if initial else 0
        phi_f = c[:, kf:] @ Cf[kf:]
        Ef = E_tot - ch["energy"]
        open_ = Ef > 0
        Kf = np.sqrt(np.where(open_, 2.0 * op.mu * Ef, 0.0))
        S = -np.sqrt(K0 * Kf) * np.exp(-1j * Kf * R_inf) * phi_f / (op.mu * gh)
        p_inel[f] = np.where(open_, np.abs(S) ** 2, 0.0)
    return dict(p_reac=p_reac, p_inel=p_inel, energies=ecol)


def time_reconstruct(op, run_vectors, t):
    """Psi(t) = sum_k (2 - delta_k0) e^{-i E0 t} (-i)^k J_k(t dE) u_k (Eq. chebyshev-expansion-constants);
    run_vectors: array (K+1, ...) of undamped components."""
    from scipy.special import jv
    K = run_vectors.shape[0] - 1
    k = np.arange(K + 1)
    f = (2.0 - (k == 0)) * np.exp(-1j * op.E0 * t) * (-1j) ** k * jv(k, t * op.dE)
    return np.tensordot(f, run_vectors, axes=(0, 0))
