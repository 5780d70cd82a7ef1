"""Seeded synthetic state-resolved probabilities for the partial-wave sums.

Shaped like the output of the batched partial-wave workload: one curve per
computed total angular momentum, initial-helicity/parity family and final
state, on the collision-energy grid.  Each curve is a smooth threshold rise to
a random plateau in [0, 1) with small oscillations on top, clipped to [0, 1];
thresholds rise with J by a random increasing sequence.  Nothing here follows
the paper's arithmetic: these are inputs only.
"""
import numpy as np

from .configs import config


def families(j0):
    """(Omega0, parity) families of initial rotational state j0 and their smallest J:
    Omega0 = 0 once, Omega0 = 1..j0 with both parities."""
    fams = [(0, +1)] + [(om, s) for om in range(1, j0 + 1) for s in (+1, -1)]
    return fams, [om for om, _ in fams]


def energy_grid(n_e, e_lo, e_hi, seed=None):
    """Ascending grid of n_e points in [e_lo, e_hi]: uniform, or jittered when seeded."""
    e = np.linspace(e_lo, e_hi, n_e)
    if seed is not None and n_e > 2:
        rng = np.random.default_rng(seed)
        h = (e_hi - e_lo) / (n_e - 1)
        e[1:-1] += rng.uniform(-0.3 * h, 0.3 * h, n_e - 2)
    return e


def probability_curves(n_calc, n_fam, n_f, energies, seed, fam_jmin=None, J_calc=None):
    """p[n_calc][n_fam][n_f][n_e] in [0, 1]; zeros where J_calc[c] < fam_jmin[fam]."""
    rng = np.random.default_rng(seed)
    e = np.asarray(energies, dtype=np.float64)
    span = e[-1] - e[0] if e.size > 1 else 1.0
    steps = rng.uniform(0.0, 0.08 * span, size=n_calc)
    thr = e[0] + 0.1 * span + np.cumsum(steps)                # rising with J
    p = np.zeros((n_calc, n_fam, n_f, e.size))
    for c in range(n_calc):
        for fam in range(n_fam):
            if fam_jmin is not None and J_calc is not None and J_calc[c] < fam_jmin[fam]:
                continue
            plateau = rng.uniform(0.0, 1.0, n_f)
            width = rng.uniform(0.01, 0.1, n_f) * span
            offs = rng.uniform(-0.05, 0.05, n_f) * span
            wig = rng.uniform(0.0, 0.05, n_f)
            freq = rng.uniform(5.0, 30.0, n_f) / span
            for f in range(n_f):
                x = (e - thr[c] - offs[f]) / width[f]
                rise = 0.5 * (1.0 + np.tanh(x))
                p[c, fam, f] = np.clip(plateau[f] * rise * (1.0 + wig[f] * np.sin(freq[f] * e)),
                                       0.0, 1.0)
    return p


def batch_shape(n_f=64):
    """Computed J, families (for j0 = 2), energies and reduced-mass inputs of the
    batched workload: J = 0, 2, ..., 40 computed, J_max = 40, its collision-energy
    grid, n_f final states."""
    spec = config(4)
    J_calc = sorted({u["J"] for u in spec["units"]})
    fams, jmin = families(2)
    e = energy_grid(spec["n_energy"], spec["ecol_min"], spec["ecol_max"])
    mA, mB, mC = spec["mass_A"], spec["mass_B"], spec["mass_C"]
    return dict(J_calc=J_calc, J_max=J_calc[-1], n_fam=len(fams), fam_jmin=jmin, n_f=n_f,
                energies=e, masses=(mA, mB, mC))
