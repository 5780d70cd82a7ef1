"""The five synthetic workloads, as plain problem definitions in atomic units.

Every workload is A + BC with masses 1.008 / 2.014 / 1.008 amu (an H + DH
analogue of the paper's Sec. 6 example) on a LEPS surface.  Field names follow
the paper's input namelists (Table tab:parameters) where one exists:
  n_r, r_min, r_max            npun1, rmis1, rfin1    (first/last r grid point)
  n_R, R_min, R_max            npun2, rmis2, rfin2
  n_gamma                      nangu
  v_cut, rad_cut, rot_cut      VcutmaxeV, radcutmaxeV, rotcutmaxeV (hartree)
  abs_*_start/strength/power   absr, absalp, nexpo    (Eq. imaginary-potential)
  r_flux                       r1flux (default: r absorber start - 1 angstrom)
  n_energy, ecol_min/max       netot, ekinmin, ekinmax (collision energy)
  units                        Jtot, iparity, iommax per partial wave
  packets                      nvref, jref, iomref, ielecref + inputcol
"""
import copy

from .constants import ANG_BOHR, amu, ev

# Absorber strength: phi at the grid edge for the quadratic absorbers over the
# last 20% of each radial range.  Chosen once from the oracle's config-1 study
# (final norm and closure of the probability sum).
PHI_EDGE = 0.5

# Reactant analysis line (bohr): beyond the initial packet, before the R absorber.
R_INF = 9.5

# First Chebyshev index entering the elastic-channel sum (kminelastic): the end
# of the 1/4 norm plateau, after the outgoing half of the initial packet has
# crossed R_INF and before the reflected incoming half returns.  Chosen once
# from the oracle's norm trace and its separable-potential elastic test.
K_MIN_ELASTIC = 250


def _absorber(xmin, xmax):
    start = xmax - 0.2 * (xmax - xmin)
    return start, PHI_EDGE / (xmax - start) ** 2, 2


def _base(n_R, n_r, n_gamma, steps, units, n_elec=1, shifts=None, couplings=None):
    R_min, R_max, r_min, r_max = 0.5, 12.0, 0.5, 8.0
    rs, ra, rp = _absorber(r_min, r_max)
    Rs, Ra, Rp = _absorber(R_min, R_max)
    spec = dict(
        n_r=n_r, r_min=r_min, r_max=r_max,
        n_R=n_R, R_min=R_min, R_max=R_max,
        n_gamma=n_gamma,
        mass_A=amu(1.008), mass_B=amu(2.014), mass_C=amu(1.008),
        n_elec=n_elec,
        v_cut=ev(2.5), rad_cut=ev(2.5), rot_cut=ev(5.0),
        abs_r_start=rs, abs_r_strength=ra, abs_r_power=rp,
        abs_R_start=Rs, abs_R_strength=Ra, abs_R_power=Rp,
        r_flux=rs - ANG_BOHR, R_inf=R_INF,
        n_energy=200, ecol_min=ev(0.2), ecol_max=ev(1.5),
        steps=steps,
        units=units,
        pes=dict(De=ev(4.747), a=1.0435, re=1.401, sato=0.15,
                 shifts=shifts or [0.0], couplings=couplings or {},
                 rho0=3.0, rho_width=1.0),
    )
    return spec


def _unit(J, omega_max, n_packets=1):
    # p = (-1)^J so that the Omega = 0 block exists (p (-1)^J = +1).
    return dict(J=J, parity=(-1) ** J, omega_max=omega_max, n_packets=n_packets)


def _packet(unit, slot, j0=0, v0=0, elec0=0):
    return dict(unit=unit, slot=slot, v0=v0, j0=j0, omega0=0, elec0=elec0,
                R0=8.0, width=0.3, ecol_mean=ev(0.5), k_min_elastic=K_MIN_ELASTIC)


def _cfg1():
    s = _base(64, 48, 24, 2000, [_unit(0, 0)])
    s["packets"] = [_packet(0, 0)]
    s["name"] = "fp64_J0_64x48x24"
    return s


def _cfg2():
    s = _base(256, 192, 80, 20000, [_unit(0, 0)])
    s["packets"] = [_packet(0, 0)]
    s["name"] = "J0_256x192x80"
    return s


def _cfg3():
    s = _base(192, 160, 64, 10000, [_unit(20, 8)], n_elec=2,
              shifts=[0.0, ev(0.5)], couplings={(0, 1): ev(0.1)})
    s["packets"] = [_packet(0, 0)]
    s["name"] = "J20_omega0-8_2state_192x160x64"
    return s


def _cfg4():
    units = [_unit(J, min(J, 6), 3) for J in range(0, 41, 2)]
    s = _base(128, 128, 48, 8000, units)
    s["packets"] = [_packet(u, j0, j0=j0) for u in range(len(units)) for j0 in range(3)]
    s["name"] = "batch_J0-40_x3packets_128x128x48"
    return s


def _cfg5():
    s = _base(256, 256, 96, 10000, [_unit(4, 4)], n_elec=3,
              shifts=[0.0, ev(0.5), ev(1.0)],
              couplings={(0, 1): ev(0.10), (0, 2): ev(0.05), (1, 2): ev(0.075)})
    s["packets"] = [_packet(0, 0)]
    s["name"] = "mlp_J4_3state_256x256x96"
    return s


CONFIGS = {1: _cfg1, 2: _cfg2, 3: _cfg3, 4: _cfg4, 5: _cfg5}


def config(i):
    """A fresh copy of workload i (1..5)."""
    return copy.deepcopy(CONFIGS[i]())


def small_variant(i, n_R=None, n_r=None, n_gamma=None, steps=None, units=None,
                  packets=None, n_energy=None):
    """Workload i with its physics kept but smaller grids / fewer steps (tests)."""
    s = config(i)
    if n_R:
        s["n_R"] = n_R
    if n_r:
        s["n_r"] = n_r
    if n_gamma:
        s["n_gamma"] = n_gamma
    if steps:
        s["steps"] = steps
    if units is not None:
        s["units"] = units
    if packets is not None:
        s["packets"] = packets
    if n_energy:
        s["n_energy"] = n_energy
    s["name"] = s["name"] + "_small"
    return s
