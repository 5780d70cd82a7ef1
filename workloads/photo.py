"""Synthetic photodissociation inputs: a transition dipole times an initial bound
state, sampled on a plan's grid (the product inside Eq. initial-photo-wvp), and
a ground-state surface whose lowest state can serve as that bound state.

The initial bound state and the dipole surfaces of a real system are not part
of these workloads.  Either a localised function stands in for the bound state
(a Gaussian around r = 1.4, R = 3.0 bohr in the interaction region with a
smooth angular factor; photo_packet), or the lowest state of a harmonic
ground-state well (ground_state_table) computed by the caller multiplies the
dipole (dipole_times).  The dipole of helicity block Omega is a smooth function
of (r, R, gamma) with its own amplitude.  Nothing here follows the method's
arithmetic: the values are inputs, given as the DVR-weighted coefficients
sqrt(dr dR w_n) f(r_i, R_m, gamma_n) of the library's packet layout.
"""
import numpy as np


def photo_packet(spec, unit, r, R, x, w, seed=0):
    """u[n_omega][n_elec][n_gamma][n_R][n_r] for unit `unit` of spec, on the grid
    (r, R, cos gamma = x, Gauss-Legendre weights w)."""
    u = spec["units"][unit]
    lo = 0 if u["parity"] * (-1) ** u["J"] == 1 else 1
    n_om = u["omega_max"] - lo + 1
    rng = np.random.default_rng(seed)
    rr, RR, xx = r[None, None, :], R[None, :, None], x[:, None, None]
    bound = (np.exp(-((rr - 1.4) / 0.25) ** 2 - ((RR - 3.0) / 0.4) ** 2)
             * (1.0 + 0.3 * xx + 0.1 * xx * xx))
    dr, dR = r[1] - r[0], R[1] - R[0]
    wgt = np.sqrt(dr * dR * np.asarray(w))[:, None, None]
    out = np.zeros((n_om, spec["n_elec"], len(x), len(R), len(r)))
    for b in range(n_om):
        amp = rng.uniform(0.5, 1.0) / (1 + b)
        for el in range(spec["n_elec"]):
            if el != spec["n_elec"] - 1:     # the transition reaches the last state only
                continue
            dip = amp * np.tanh(0.5 * (RR - 1.0)) * (1.0 + 0.2 * (rr - 1.4)) * (1.0 + 0.1 * b * xx)
            out[b, el] = wgt * dip * bound
    return out


def _dipole(b, amp, rr, RR, xx):
    return amp * np.tanh(0.5 * (RR - 1.0)) * (1.0 + 0.2 * (rr - 1.4)) * (1.0 + 0.1 * b * xx)


def ground_state_table(spec, r, R, x):
    """Potential table [1][n_gamma][n_R][n_r] (hartree) of a ground-state well at
    r = 1.4, R = 3.0 bohr and a linear geometry (cos gamma = 1 at the bottom, a
    single well): 0.35/2 (r - 1.4)^2 + 0.10/2 (R - 3.0)^2 + 0.05 (1 - cos gamma),
    capped at spec["v_cut"]."""
    rr, RR, xx = r[None, None, :], R[None, :, None], x[:, None, None]
    v = 0.175 * (rr - 1.4) ** 2 + 0.05 * (RR - 3.0) ** 2 + 0.05 * (1.0 - xx)
    return np.minimum(v, spec["v_cut"])[None]


def dipole_times(spec, unit, r, R, x, psi, seed=0):
    """Packet of unit `unit` (last diabatic state) = dipole times a bound state psi
    given as DVR-weighted coefficients [n_gamma][n_R][n_r] on the same grid (the
    dipole is local, so it multiplies the coefficients point by point)."""
    u = spec["units"][unit]
    lo = 0 if u["parity"] * (-1) ** u["J"] == 1 else 1
    n_om = u["omega_max"] - lo + 1
    rng = np.random.default_rng(seed)
    rr, RR, xx = r[None, None, :], R[None, :, None], x[:, None, None]
    psi = np.asarray(psi, dtype=np.float64).reshape(len(x), len(R), len(r))
    out = np.zeros((n_om, spec["n_elec"], len(x), len(R), len(r)))
    for b in range(n_om):
        amp = rng.uniform(0.5, 1.0) / (1 + b)
        out[b, spec["n_elec"] - 1] = _dipole(b, amp, rr, RR, xx) * psi
    return out


def bound_spec(spec):
    """The workload's grid with one electronic state and J = 0: the plan of the
    ground-state surface."""
    s = dict(spec)
    s["n_elec"] = 1
    s["units"] = [dict(J=0, parity=1, omega_max=0, n_packets=1)]
    s["packets"] = []
    s["pes"] = dict(spec["pes"], shifts=[0.0], couplings={})
    return s


def bound_components(r, R, x, w, n_om_i):
    """Stand-in bound-state helicity components [n_om_i][n_gamma][n_R][n_r]
    (DVR-weighted): a Gaussian in the interaction region with an angular factor
    that differs per component."""
    rr, RR, xx = r[None, None, :], R[None, :, None], x[:, None, None]
    dr, dR = r[1] - r[0], R[1] - R[0]
    wgt = np.sqrt(dr * dR * np.asarray(w))[:, None, None]
    out = np.empty((n_om_i, len(x), len(R), len(r)))
    for b in range(n_om_i):
        ang = (1.0 - xx * xx) ** (0.5 * b) * (1.0 + 0.3 * xx + 0.1 * (b + 1) * xx * xx)
        out[b] = wgt * np.exp(-((rr - 1.4) / 0.25) ** 2 - ((RR - 3.0) / 0.4) ** 2) * ang / (1 + b)
    return out


def dipole_components(r, R, x):
    """Body-frame spherical components d_q, q = -1, 0, +1 [3][n_gamma][n_R][n_r], of
    a stand-in transition dipole in the molecular x-z plane: d_z along R, d_x
    across it, smooth in (r, R, gamma); d_{+1} = -d_x / sqrt 2, d_{-1} = d_x / sqrt 2,
    d_0 = d_z."""
    rr, RR, xx = r[None, None, :], R[None, :, None], x[:, None, None]
    dz = np.tanh(0.5 * (RR - 1.0)) * (1.0 + 0.2 * (rr - 1.4)) * (0.6 + 0.4 * xx)
    dx = 0.5 * np.sqrt(np.maximum(1.0 - xx * xx, 0.0)) * np.exp(-0.1 * (RR - 3.0) ** 2) * (1.0 + 0.1 * rr)
    s2 = np.sqrt(2.0)
    shape = (len(x), len(R), len(r))
    return np.stack([np.broadcast_to(dx / s2, shape), np.broadcast_to(dz, shape),
                     np.broadcast_to(-dx / s2, shape)]).copy()
