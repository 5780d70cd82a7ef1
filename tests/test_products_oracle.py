"""Pins of the product-arrangement oracle (reactant-coordinate-based analysis,
Sec. "Analysis of final states"): coordinate changes, DVR interpolation,
normalisation across coordinate sets (no GPU needed).

A plausible slip breaks at least one of them:
  - a wrong mass ratio or atom label in a coordinate change: distances;
  - a wrong sine or Legendre DVR function (phase, wall, normalisation): the
    basis-function interpolation;
  - a wrong or missing r'R'/(rR) factor or product quadrature weight: the
    norm of a packet computed in both coordinate sets.
"""
import math

import numpy as np
import pytest

from oracle import products_oracle as PR
from oracle import tdwp_oracle as O
from workloads import config
from workloads import pes as PES


def _spec(n_R=20, n_r=18, n_gamma=10):
    s = config(1)
    s.update(n_R=n_R, n_r=n_r, n_gamma=n_gamma, rad_cut=0.0, rot_cut=0.0)
    s["R_min"], s["R_max"], s["r_min"], s["r_max"] = 0.5, 9.0, 0.5, 9.0
    return s


@pytest.mark.parametrize("arr", PR.ARRANGEMENTS)
def test_coordinate_change_keeps_interatomic_distances(arr):
    """The three interatomic distances of a configuration are the same from reactant
    Jacobi (the PES fixture's distance relations) and from product Jacobi (the law
    of cosines in the product frame with the product masses); the round trip is the
    identity."""
    s = _spec()
    mA, mB, mC = s["mass_A"], s["mass_B"], s["mass_C"]
    rng = np.random.default_rng(7)
    r = rng.uniform(0.6, 6.0, 200)
    R = rng.uniform(0.6, 6.0, 200)
    x = rng.uniform(-0.99, 0.99, 200)
    rab, rbc, rac = PES.atom_distances(r, R, x, mA, mB, mC)
    rp, Rp, xp = PR.product_from_reactant(s, arr, r, R, x)
    mX, mY = (mA, mB) if arr == "C" else (mA, mC)
    dX, dY = mY * rp / (mX + mY), mX * rp / (mX + mY)
    d_XZ = np.sqrt(Rp ** 2 + dX ** 2 + 2 * Rp * dX * xp)
    d_YZ = np.sqrt(Rp ** 2 + dY ** 2 - 2 * Rp * dY * xp)
    if arr == "C":   # X = A, Y = B, Z = C
        got = (rp, d_YZ, d_XZ)
    else:            # X = A, Y = C, Z = B
        got = (d_XZ, d_YZ, rp)
    for a, b in zip(got, (rab, rbc, rac)):
        assert np.max(np.abs(a - b)) < 1e-12
    r2, R2, x2 = PR.reactant_from_product(s, arr, rp, Rp, xp)
    assert max(np.max(np.abs(r2 - r)), np.max(np.abs(R2 - R)), np.max(np.abs(x2 - x))) < 1e-12


@pytest.mark.parametrize("k,l,j", [(1, 1, 0), (3, 5, 2), (17, 2, 9), (9, 20, 4)])
def test_interpolation_exact_on_basis_functions(k, l, j):
    """A product of one sine mode in r, one in R and one normalised Legendre function
    in gamma lies in the DVR basis: interpolated anywhere inside the box it equals
    the closed form; outside the box it is zero."""
    s = _spec()
    op = O.Operator(s)

    def mode(n, q, L, wall, pts):
        return math.sqrt(2.0 / L) * np.sin(q * math.pi * (pts - wall) / L)

    Pj = O.assoc_legendre_normalised(j, 0, op.x)[j]
    u = (np.sqrt(op.w * op.dR * op.dr)[:, None, None] * Pj[:, None, None]
         * mode(s["n_R"], l, op.LR, op.R_wall, op.R)[None, :, None]
         * mode(s["n_r"], k, op.Lr, op.r_wall, op.r)[None, None, :])
    rng = np.random.default_rng(7)
    pr = rng.uniform(op.r_wall + 1e-3, op.r_wall + op.Lr - 1e-3, 300)
    pR = rng.uniform(op.R_wall + 1e-3, op.R_wall + op.LR - 1e-3, 300)
    px = rng.uniform(-1.0, 1.0, 300)
    got = PR.interpolate(op, u, (pr, pR, px))
    want = (mode(0, k, op.Lr, op.r_wall, pr) * mode(0, l, op.LR, op.R_wall, pR)
            * O.assoc_legendre_normalised(j, 0, px)[j])
    assert np.max(np.abs(got - want)) < 1e-11 * max(1.0, np.max(np.abs(want)))
    out = PR.interpolate(op, u, (np.array([op.r_wall - 0.1, 4.0]), np.array([3.0, op.R_wall + op.LR + 0.2]),
                                 np.array([0.1, 0.2])))
    assert np.all(out == 0.0)


@pytest.mark.parametrize("arr", PR.ARRANGEMENTS)
def test_packet_norm_equal_in_both_coordinate_sets(arr):
    """sum_k dR' sum (product line at R'_k)^2 approximates the integral of |Phi'|^2 over
    the product coordinates, which the unit Jacobian makes equal to the packet's
    norm sum u^2 in reactant coordinates: a packet inside both grids."""
    s = _spec(n_R=36, n_r=36, n_gamma=16)
    op = O.Operator(s)
    # a smooth packet around a geometry inside both arrangements' grids
    rr, RR, xx = op.r[None, None, :], op.R[None, :, None], op.x[:, None, None]
    phi = np.exp(-((rr - 3.2) / 0.45) ** 2 - ((RR - 2.6) / 0.45) ** 2) * (1.0 + 0.4 * xx) * np.exp(-2.0 * (xx - 0.3) ** 2)
    u = (np.sqrt(op.dr * op.dR * op.w)[:, None, None] * phi)[None, None]
    norm_reactant = float(np.sum(u * u))
    Rps = np.linspace(0.3, 7.5, 100)
    dRp = Rps[1] - Rps[0]
    total = 0.0
    for Rp in Rps:
        prod = PR.Products(op, arr, Rp, 64, 0.2, 7.5, 20)
        line = PR.product_line(op, prod, u)
        total += dRp * float(np.sum(line ** 2))
    assert abs(total / norm_reactant - 1.0) < 1e-4
