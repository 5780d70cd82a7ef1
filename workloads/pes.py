"""Synthetic diabatic potential-energy surfaces (the user-supplied PES of the
preparatory stage, Sec. 4 "System dependent programs": a routine that returns
the diabatic electronic matrix at a geometry).

State 1 is a London-Eyring-Polanyi-Sato surface for three identical Morse
pairs.  Further diabatic states are copies shifted upward by a constant, and
off-diagonal couplings are Gaussians in the mass-scaled hyperradius.  Energies
are returned in hartree relative to the reactant diatomic minimum (the
asymptotic A + BC(r = r_e) value of state 1); diagonal entries are capped at
the potential cut (Sec. 2.1, item 5 of the list; Table tab:parameters,
VcutmaxeV), off-diagonal entries are not cut.

Geometry (Sec. 4, distance relations): r is the B-C distance, R joins the BC
centre of mass to A, and gamma is the angle between the B->C vector and R.
"""
import numpy as np


def morse_singlet(d, De, a, re):
    x = np.exp(-a * (d - re))
    return De * (x * x - 2.0 * x)


def morse_triplet(d, De, a, re):
    x = np.exp(-a * (d - re))
    return 0.5 * De * (x * x + 2.0 * x)


def leps(rab, rbc, rac, De, a, re, sato):
    """Textbook LEPS energy (hartree, zero at separated atoms) for identical pairs."""
    def qj(d):
        e1 = morse_singlet(d, De, a, re)
        e3 = morse_triplet(d, De, a, re)
        q = 0.5 * (e1 * (1.0 + sato) + e3 * (1.0 - sato))
        j = 0.5 * (e1 * (1.0 + sato) - e3 * (1.0 - sato))
        return q, j
    q1, j1 = qj(rab)
    q2, j2 = qj(rbc)
    q3, j3 = qj(rac)
    exch = np.sqrt(0.5 * ((j1 - j2) ** 2 + (j2 - j3) ** 2 + (j3 - j1) ** 2))
    return (q1 + q2 + q3 - exch) / (1.0 + sato)


def atom_distances(r, R, cosg, mA, mB, mC):
    """(r_AB, r_BC, r_AC) from Jacobi (r, R, cos gamma) of the A + BC arrangement."""
    mbc = mB + mC
    dB = mC * r / mbc          # distance from the BC centre of mass to B
    dC = mB * r / mbc          # ... to C
    rab = np.sqrt(np.maximum(R * R + dB * dB + 2.0 * R * dB * cosg, 0.0))
    rac = np.sqrt(np.maximum(R * R + dC * dC - 2.0 * R * dC * cosg, 0.0))
    return rab, r, rac


def hyperradius(r, R, mA, mB, mC):
    """Delves mass-scaled hyperradius rho^2 = (mu R^2 + m r^2) / mu3."""
    M = mA + mB + mC
    mu = mA * (mB + mC) / M
    m = mB * mC / (mB + mC)
    mu3 = np.sqrt(mA * mB * mC / M)
    return np.sqrt((mu * R * R + m * r * r) / mu3)


def _npack(n):
    return n * (n + 1) // 2


def diabatic_matrix(spec, r, R, cosg):
    """Packed upper triangle (11, 12, .., 1n, 22, .., nn) of the capped diabatic
    matrix at broadcastable arrays r, R, cosg.  Returns shape (npack,) + shape."""
    pes = spec["pes"]
    mA, mB, mC = spec["mass_A"], spec["mass_B"], spec["mass_C"]
    r, R, cosg = np.broadcast_arrays(np.asarray(r, float), np.asarray(R, float),
                                     np.asarray(cosg, float))
    rab, rbc, rac = atom_distances(r, R, cosg, mA, mB, mC)
    v1 = leps(rab, rbc, rac, pes["De"], pes["a"], pes["re"], pes["sato"]) + pes["De"]
    n = spec["n_elec"]
    out = np.empty((_npack(n),) + r.shape)
    rho = hyperradius(r, R, mA, mB, mC) if n > 1 else None
    p = 0
    for a in range(n):
        for b in range(a, n):
            if a == b:
                v = v1 + pes["shifts"][a]
                if spec["v_cut"] > 0:
                    v = np.minimum(v, spec["v_cut"])
                out[p] = v
            else:
                c = pes["couplings"].get((a, b), 0.0)
                out[p] = c * np.exp(-((rho - pes["rho0"]) ** 2) / pes["rho_width"] ** 2)
            p += 1
    return out


def asymptotic_potential(spec, r, elec):
    """R -> infinity limit of diagonal entry `elec` (capped), a function of r only.

    For r > 0 the LEPS A + BC limit equals the singlet Morse curve exactly
    (the BC exchange integral is negative there)."""
    pes = spec["pes"]
    v = morse_singlet(np.asarray(r, float), pes["De"], pes["a"], pes["re"]) + pes["De"]
    v = v + pes["shifts"][elec]
    if spec["v_cut"] > 0:
        v = np.minimum(v, spec["v_cut"])
    return v
