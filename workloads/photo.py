"""Synthetic photodissociation packet: a transition dipole times an initial bound
state, sampled on a plan's grid (the product inside Eq. initial-photo-wvp).

The initial bound state and the dipole surfaces of a real system are not part
of these workloads; a localised function stands in for the bound state (a
Gaussian around r = 1.4, R = 3.0 bohr in the interaction region with a smooth
angular factor), and the dipole of helicity block Omega is a smooth function of
(r, R, gamma) with its own amplitude.  Nothing here follows the method's
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
