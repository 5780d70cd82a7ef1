"""Sets up a library plan for a workload definition: evaluates the caller's
potential-energy surface on the plan's own grid, solves the diatomic channel
problems with the library's preparatory-stage entry point and installs the
initial packets.  Marshalling only; no step of the method runs here."""
import numpy as np

from workloads import asymptotic_potential, diabatic_matrix

from .tdwp import Plan


def potential_table(plan, spec):
    r, R, x, _ = plan.grid()
    return diabatic_matrix(spec, r[None, None, :], R[None, :, None], x[:, None, None])


def build(spec, precision="fp64", bounds=None, stream="current", vtable=None, mlp=None,
          autotune=0):
    """Plan + potential + every initial packet.  Returns (plan, info) where info
    holds the grid, E_v0j0 per packet and the initial channel functions.
    mlp: None (tabulated potential) or a dict of set_potential_mlp arguments
    (sample_idx, init_params, order, batch, epochs, lr); the table is then the
    training data and info["mlp_report"] the training report."""
    plan = Plan(spec, precision=precision, bounds=bounds, stream=stream)
    r, R, x, w = plan.grid()
    if vtable is None:
        vtable = potential_table(plan, spec)
    info = dict(r=r, R=R, x=x, w=w, e0={}, chi0={})
    if mlp is None:
        plan.set_potential(vtable)
    else:
        info["mlp_report"] = plan.set_potential_mlp(vtable, **mlp)
    if autotune:
        info["autotune"] = plan.autotune(autotune)
    install_packets(plan, spec, info)
    return plan, info


def install_packets(plan, spec, info=None):
    """(Re)installs every initial packet of the workload: propagation restarts at k = 0."""
    r = plan.grid()[0]
    for pk in spec["packets"]:
        va = asymptotic_potential(spec, r, pk["elec0"])
        e, chi = plan.diatomic_states(va, pk["j0"], pk["v0"] + 1)
        E, c = e[pk["v0"]], chi[pk["v0"]]
        plan.set_initial_packet(pk, c, E)
        if info is not None:
            info["e0"][(pk["unit"], pk["slot"])] = E
            info["chi0"][(pk["unit"], pk["slot"])] = c


def channels(plan, spec, unit, jmax, vmax, elecs=None, omegas=None):
    """Reactant-arrangement channels (elec, v, j, omega) with the library's
    channel functions and energies."""
    r = plan.grid()[0]
    u = spec["units"][unit]
    lo = 0 if u["parity"] * (-1) ** u["J"] == 1 else 1
    oms = omegas if omegas is not None else list(range(lo, u["omega_max"] + 1))
    out = []
    for el in (elecs if elecs is not None else range(spec["n_elec"])):
        va = asymptotic_potential(spec, r, el)
        for j in range(jmax + 1):
            e, chi = plan.diatomic_states(va, j, vmax + 1)
            for v in range(vmax + 1):
                for om in oms:
                    if om <= j:
                        out.append(dict(elec=el, v=v, j=j, omega=om, energy=float(e[v]),
                                        chi=np.array(chi[v])))
    return out
