"""FP64 CPU oracle for state-to-state analysis in a product arrangement from a
packet propagated in reactant Jacobi coordinates (the reactant-coordinate-based
method of Sec. "Analysis of final states", Eqs. final-states,
Chebyshev-products-overlaps, S-matrix-from-chebyshev), for J = 0.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the library and imports nothing from it.

  * Geometry: the atoms are placed from Jacobi coordinates (Sec. 4 distance
    relations, A + BC labels as in oracle/tdwp_oracle.py: r = B -> C, R from the
    BC centre of mass to A, gamma their angle); a product arrangement XY + Z is
    AB + C ("C") or AC + B ("B"), with r' = X -> Y, R' from the XY centre of
    mass to Z and gamma' their angle.  Every coordinate change goes through the
    atom positions.
  * The packet's function: u[n][m][i] = sqrt(dr dR w_n) Phi(r_i, R_m, x_n) is the
    DVR form of Phi(r, R, x) = sum u[n][m][i] t_i(r) t_m(R) L_n(x), with the
    sine-DVR functions t_i = sum_k S_ki sqrt(2/L) sin(k pi (x - x_wall)/L) (zero
    outside the box) and the Legendre DVR functions L_n(x) = sum_j P[j][n]
    P~_j(x); at the grid points they reduce to the packet's values.
  * Product line (Eq. Chebyshev-products-overlaps at R' = R'_inf): on a product
    grid r'_i (equidistant) x gamma'_n (Gauss-Legendre), the product-frame
    function Phi'(r', R', x') = (r' R' / (r R)) Phi(r, R, x) (for J = 0 the
    angular functions of both frames are the same constant and the Jacobi
    change has unit Jacobian), stored DVR-weighted as
    sqrt(dr' w'_n) Phi'(r'_i, R'_inf, x'_n).
  * Product channels chi'_{v'j'} (Eq. final-states): eigenvectors of the
    diatomic XY Hamiltonian on the product r' grid (reduced mass m' of XY, the
    caller's asymptotic potential, the caps of the propagation), as for the
    reactant channels.
  * S-matrix (Eq. S-matrix-from-chebyshev, with the Green's-function
    normalisation of the reactant channels): |S'_f|^2 = K0 K'_f |Phi'_f|^2 /
    (mu mu' |g^(K0)|^2), Phi'_f = sum_k c_k C'_f(k), K'_f = sqrt(2 mu' (E - E'_f));
    the outgoing flux of channel f over the incoming flux, mu' the reduced mass
    of Z + XY.

Pinned by tests/test_products_oracle.py: interatomic distances preserved by the
coordinate changes and their round trip; the interpolation exact on the basis
functions; norms equal in both coordinate sets (the Jacobian and the r'R'/(rR)
factor); and, on a reactive run, the products' probabilities against the total
reactive flux.
"""
import math

import numpy as np

from oracle import tdwp_oracle as O

ARRANGEMENTS = ("C", "B")   # AB + C, AC + B


def _masses(spec):
    return spec["mass_A"], spec["mass_B"], spec["mass_C"]


def positions_from_reactant(spec, r, R, x):
    """Atom positions (A, B, C), each (..., 3), from reactant Jacobi (r, R, cos gamma):
    BC centre of mass at the origin, R along z, r in the x-z plane."""
    mA, mB, mC = _masses(spec)
    r, R, x = np.broadcast_arrays(np.asarray(r, float), np.asarray(R, float), np.asarray(x, float))
    s = np.sqrt(np.maximum(1.0 - x * x, 0.0))
    rhat = np.stack([s, np.zeros_like(s), x], axis=-1)
    zhat = np.stack([np.zeros_like(s), np.zeros_like(s), np.ones_like(s)], axis=-1)
    A = R[..., None] * zhat
    B = -(mC / (mB + mC)) * r[..., None] * rhat
    C = (mB / (mB + mC)) * r[..., None] * rhat
    return A, B, C


def _jacobi(X, Y, Z, mX, mY):
    """(r, R, cos gamma) with r = Y - X, R from the XY centre of mass to Z."""
    rv = Y - X
    Rv = Z - (mX * X + mY * Y) / (mX + mY)
    r = np.linalg.norm(rv, axis=-1)
    R = np.linalg.norm(Rv, axis=-1)
    x = np.sum(rv * Rv, axis=-1) / (r * R)
    return r, R, np.clip(x, -1.0, 1.0)


def product_from_reactant(spec, arrangement, r, R, x):
    """Product Jacobi (r', R', cos gamma') of XY + Z from reactant (r, R, cos gamma)."""
    mA, mB, mC = _masses(spec)
    A, B, C = positions_from_reactant(spec, r, R, x)
    if arrangement == "C":
        return _jacobi(A, B, C, mA, mB)
    return _jacobi(A, C, B, mA, mC)


def reactant_from_product(spec, arrangement, rp, Rp, xp):
    """Reactant Jacobi (r, R, cos gamma) from product (r', R', cos gamma'): the product
    atoms placed with the XY centre of mass at the origin and R' along z."""
    mA, mB, mC = _masses(spec)
    mX, mY = (mA, mB) if arrangement == "C" else (mA, mC)
    rp, Rp, xp = np.broadcast_arrays(np.asarray(rp, float), np.asarray(Rp, float), np.asarray(xp, float))
    s = np.sqrt(np.maximum(1.0 - xp * xp, 0.0))
    rhat = np.stack([s, np.zeros_like(s), xp], axis=-1)
    zhat = np.stack([np.zeros_like(s), np.zeros_like(s), np.ones_like(s)], axis=-1)
    X = -(mY / (mX + mY)) * rp[..., None] * rhat
    Y = (mX / (mX + mY)) * rp[..., None] * rhat
    Z = Rp[..., None] * zhat
    if arrangement == "C":
        A, B, C = X, Y, Z
    else:
        A, C, B = X, Y, Z
    return _jacobi(B, C, A, mB, mC)


def product_masses(spec, arrangement):
    """(mu', m'): reduced mass of Z + XY and of the diatom XY."""
    mA, mB, mC = _masses(spec)
    mX, mY, mZ = (mA, mB, mC) if arrangement == "C" else (mA, mC, mB)
    M = mA + mB + mC
    return mZ * (mX + mY) / M, mX * mY / (mX + mY)


class Products:
    """Product grid of one arrangement: r'_i (n_r points over [r_min, r_max], walls
    one step outside), Gauss-Legendre cos gamma'_n (n_gamma), the line R' = R_inf."""

    def __init__(self, op, arrangement, R_inf, n_r, r_min, r_max, n_gamma):
        self.op = op
        self.arrangement = arrangement
        self.R_inf = R_inf
        self.r, self.dr, self.L, self.wall = O.radial_grid(r_min, r_max, n_r)
        self.x, self.w = O.gauss_legendre(n_gamma)
        self.mu, self.m = product_masses(op.spec, arrangement)
        self.jmax = n_gamma - 1
        self.T, self.e = O.sine_kinetic(n_r, self.L, self.m, op.spec["rad_cut"])
        self.Br = 1.0 / (2.0 * self.m * self.r ** 2)
        self.P = O.legendre_table(self.jmax, 0, self.x, self.w)
        RP, XP = np.meshgrid(self.r, self.x)              # [n_gamma'][n_r']
        rr, RR, xx = reactant_from_product(op.spec, arrangement, RP, np.full_like(RP, R_inf), XP)
        self.points = (rr, RR, xx)
        # r' R' / (r R) and the product DVR weights sqrt(dr' w'_n)
        self.factor = (RP * R_inf) / (rr * RR) * np.sqrt(self.dr * self.w)[:, None]
        # the reactant DVR functions at the line's points (the interpolation weights)
        self.weights = dvr_functions(op, self.points)

    def diatomic_states(self, v_asym, j, n_states):
        """Lowest n_states eigenpairs of T_r' + V(r') + min(j(j+1)/(2 m' r'^2), rotcut)
        on the product grid; DVR-normalised, first component above 1e-3 of the
        maximum made positive (the reactant channels' convention)."""
        rot = self.Br * j * (j + 1)
        if self.op.spec["rot_cut"] > 0:
            rot = np.minimum(rot, self.op.spec["rot_cut"])
        e, vecs = np.linalg.eigh(self.T + np.diag(np.asarray(v_asym, float) + rot))
        chis = []
        for v in range(n_states):
            c = vecs[:, v].copy()
            first = np.nonzero(np.abs(c) > 1e-3 * np.max(np.abs(c)))[0][0]
            if c[first] < 0:
                c = -c
            chis.append(c / np.linalg.norm(c))
        return e[:n_states].copy(), np.array(chis)


def sine_dvr_functions(n, wall, length, pts):
    """t_i(x) at points pts (any shape) -> array [n][...]: sum_k S_ki sqrt(2/L)
    sin(k pi (x - wall)/L), zero outside (wall, wall + L)."""
    S = O.sine_dvr(n)
    pts = np.asarray(pts, float)
    k = np.arange(1, n + 1)
    phi = math.sqrt(2.0 / length) * np.sin(np.pi * np.multiply.outer(k, pts - wall) / length)
    inside = (pts > wall) & (pts < wall + length)
    return np.tensordot(S.T, phi, axes=(1, 0)) * inside


def legendre_dvr_functions(op, pts):
    """L_n(x) at points pts -> array [n_gamma][...]: sum_j P[j][n] P~_j(x)."""
    pts = np.asarray(pts, float)
    Pt = O.assoc_legendre_normalised(op.jmax, 0, pts.ravel()).reshape((op.jmax + 1,) + pts.shape)
    return np.tensordot(op.P[0].T, Pt, axes=(1, 0))


def dvr_functions(op, pts):
    """(t_i(r), t_m(R), L_n(x)) at the points pts = (r, R, x)."""
    r, R, x = pts
    return (sine_dvr_functions(op.spec["n_r"], op.r_wall, op.Lr, r),
            sine_dvr_functions(op.spec["n_R"], op.R_wall, op.LR, R),
            legendre_dvr_functions(op, x))


def interpolate(op, u_state, pts, weights=None):
    """Phi(r, R, x) at the points pts = (r, R, x) (arrays of one shape) from one
    state's DVR coefficients u_state[n_gamma][n_R][n_r]."""
    tr, tR, Ln = dvr_functions(op, pts) if weights is None else weights
    return np.einsum("nmi,i...,m...,n...->...", u_state, tr, tR, Ln, optimize=True)


def product_line(op, prod, u):
    """[n_Lambda][n_gamma'][n_r'] product line of a J = 0 packet u[1][n_Lambda][...]:
    sqrt(dr' w'_n) Phi'(r'_i, R'_inf, x'_n) per diabatic state."""
    return np.array([prod.factor * interpolate(op, u[0, le], prod.points, prod.weights)
                     for le in range(u.shape[1])])


def analyse_products(op, prod, packet, lines, E_v0j0, channels):
    """|S'_f(E)|^2 on the collision-energy grid for product channels
    (elec, v, j, energy, chi[n_r']) from the product lines of k = 0..K."""
    ecol = O.collision_energies(op.spec)
    E_tot = ecol + E_v0j0
    lines = np.asarray(lines)
    K = lines.shape[0] - 1
    c = O.chebyshev_energy_coeffs(op, E_tot, K)
    K0 = np.sqrt(2.0 * op.mu * ecol)
    gh = O.ghat(op, O.gaussian_R(op, packet), K0)
    out = np.zeros((len(channels), ecol.size))
    for f, ch in enumerate(channels):
        Cf = np.einsum("kni,n,i->k", lines[:, ch["elec"]], prod.P[ch["j"]], np.asarray(ch["chi"]))
        phi = c @ Cf
        Ef = E_tot - ch["energy"]
        open_ = Ef > 0
        Kf = np.sqrt(np.where(open_, 2.0 * prod.mu * Ef, 0.0))
        out[f] = np.where(open_, K0 * Kf * np.abs(phi) ** 2 / (op.mu * prod.mu * np.abs(gh) ** 2), 0.0)
    return out
