"""Physical invariants of the oracle's full pipeline on the 64x48x24 J = 0 workload
(separable elastic limit, probability sum rule, r*-independence of the flux,
norm trace).  Several seconds each."""
import numpy as np
import pytest

from oracle import tdwp_oracle as O
from workloads import asymptotic_potential, config

pytestmark = pytest.mark.slow


def _channels(op, spec, jmax, vmax):
    va = asymptotic_potential(spec, op.r, 0)
    out = []
    for j in range(jmax + 1):
        e, chi = O.diatomic_states(op, va, j, vmax + 1)
        for v in range(vmax + 1):
            out.append(dict(elec=0, v=v, j=j, omega=0, energy=e[v], chi=chi[v]))
    return out


@pytest.fixture(scope="module")
def leps_run():
    s = config(1)
    op = O.Operator(s)
    va = asymptotic_potential(s, op.r, 0)
    e0, chi0 = O.diatomic_states(op, va, 0, 1)
    pk = s["packets"][0]
    u0 = O.initial_packet(op, 0, pk, chi0[0])
    run = O.propagate(op, 0, u0, s["steps"], extra_r_flux=(4.2,))
    chans = _channels(op, s, 14, 3)
    res = O.analyse(op, 0, pk, run, e0[0], chans)
    return dict(op=op, run=run, res=res, pk=pk, e0=e0[0], chans=chans)


def test_separable_potential_is_purely_elastic():
    """V = V_asym(r) only, J = 0: the packet can only bounce off the R wall; the
    elastic |S|^2 is 1 up to the kminelastic window error, every other channel
    and the reactive flux vanish.  Pins the S-matrix and flux normalisations."""
    s = config(1)
    op0 = O.Operator(s)
    va = asymptotic_potential(s, op0.r, 0)
    vt = np.broadcast_to(va[None, None, None, :], (1, s["n_gamma"], s["n_R"], s["n_r"])).copy()
    op = O.Operator(s, vtable=vt)
    e0, chi0 = O.diatomic_states(op, va, 0, 1)
    pk = s["packets"][0]
    run = O.propagate(op, 0, O.initial_packet(op, 0, pk, chi0[0]), s["steps"])
    res = O.analyse(op, 0, pk, run, e0[0], _channels(op, s, 2, 2))
    pel = res["p_inel"][0]
    assert abs(pel.mean() - 1.0) < 0.02
    assert np.max(np.abs(pel - 1.0)) < 0.12
    assert np.max(np.abs(res["p_inel"][1:])) < 1e-12
    assert np.max(np.abs(res["p_reac"])) < 1e-10


def test_probability_sum_rule(leps_run):
    """Reactive + all inelastic = 1 (the unity column of the S2prod output)."""
    res = leps_run["res"]
    tot = res["p_reac"].sum(0) + res["p_inel"].sum(0)
    assert abs(tot.mean() - 1.0) < 0.02
    assert np.max(np.abs(tot - 1.0)) < 0.10
    assert np.min(res["p_inel"]) >= 0.0
    assert 0.0 <= np.min(res["p_reac"]) + 1e-3 and np.max(res["p_reac"]) < 1.0


def test_reactive_flux_independent_of_r_star(leps_run):
    run, op = leps_run["run"], leps_run["op"]
    r2 = O.analyse(op, 0, leps_run["pk"], run, leps_run["e0"], (), flux_slices=run["extra"][0])
    p1, p2 = leps_run["res"]["p_reac"][0], r2["p_reac"][0]
    assert np.max(np.abs(p1 - p2)) < 0.03
    assert np.max(p1) > 0.3


def test_norm_trace_plateaus():
    """Norm of the Chebyshev components: ~1/2 plateau, then ~1/4 once the outgoing
    half is absorbed, then decay towards zero."""
    s = config(1)
    op = O.Operator(s)
    va = asymptotic_potential(s, op.r, 0)
    e0, chi0 = O.diatomic_states(op, va, 0, 1)
    run = O.propagate(op, 0, O.initial_packet(op, 0, s["packets"][0], chi0[0]), 1000)
    n = run["norms"]
    assert abs(n[0] - 1.0) < 1e-14
    assert 0.38 < np.mean(n[20:60]) < 0.6
    assert 0.2 < np.mean(n[100:300]) < 0.3
    assert np.max(n[900:]) < 0.02
