"""Cross sections from propagated partial waves (Sec. "Cross sections"): the
HIP path's probabilities of a batch of J summed by the library, against the
oracle's probabilities of the same batch summed by the oracle.

Bar: the probabilities agree to 1e-8 absolute at every energy, so the cumulative
probability over J = 0..J_max agrees to (J_max + 1)^2 1e-8 and the cross section
to pi / K0^2 times that.
"""
import math

import numpy as np
import pytest

from oracle import tdwp_oracle as O
from oracle import xsection_oracle as X
from workloads import asymptotic_potential, ev, small_variant

pytestmark = pytest.mark.gpu

PE_TOL = 1e-8


@pytest.fixture(scope="module", autouse=True)
def _device():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2412_10167_amd import load_library
    load_library()


def test_cross_sections_from_batched_partial_waves():
    print("\n[case] partial-wave sums: units J=0,2,4,6 (Omega<=2), reactive + Omega'=0 "
          "inelastic channels, J_max=7", flush=True)
    from paper_2412_10167_amd import cross_section, cumulative_probability, problem
    spec = small_variant(4, n_R=20, n_r=16, n_gamma=10)
    Js = [0, 2, 4, 6]
    spec["units"] = [dict(J=J, parity=1, omega_max=min(J, 2), n_packets=1) for J in Js]
    base = spec["packets"][0]
    spec["packets"] = [dict(base, unit=u, slot=0, j0=0, omega0=0, k_min_elastic=30)
                       for u in range(len(Js))]
    K = 200
    plan, _ = problem.build(spec)
    plan.propagate(K, norms=False)

    op = O.Operator(spec)
    p_dev, p_ref = [], []
    for u, pk in enumerate(spec["packets"]):
        chans = problem.channels(plan, spec, u, 3, 1, omegas=[0])
        p_inel, p_reac = plan.state_to_state(u, 0, chans)
        p_dev.append(np.vstack([p_reac, p_inel]))
        va = asymptotic_potential(spec, op.r, pk["elec0"])
        e0, chi0 = O.diatomic_states(op, va, pk["j0"], 1)
        run = O.propagate(op, u, O.initial_packet(op, u, pk, chi0[0]), K)
        och = []
        for c in chans:
            vc = asymptotic_potential(spec, op.r, c["elec"])
            ec, chic = O.diatomic_states(op, vc, c["j"], c["v"] + 1)
            och.append(dict(c, energy=ec[c["v"]], chi=chic[c["v"]]))
        res = O.analyse(op, u, pk, run, e0[0], och)
        p_ref.append(np.vstack([res["p_reac"], res["p_inel"]]))
    plan.close()
    p_dev = np.stack(p_dev)[:, None]          # [J][family][final state][energy]
    p_ref = np.stack(p_ref)[:, None]
    assert np.max(np.abs(p_dev - p_ref)) < PE_TOL

    e = np.linspace(spec["ecol_min"], spec["ecol_max"], spec["n_energy"])
    B = np.full(len(Js), ev(1.7e-3))
    J_max = 7
    C_dev = cumulative_probability(Js, B, p_dev, e, J_max)
    C_ref = X.cumulative_probability(Js, B, p_ref, e, J_max)
    assert np.max(np.abs(C_dev - C_ref)) < (J_max + 1) ** 2 * PE_TOL
    mA, mB, mC = spec["mass_A"], spec["mass_B"], spec["mass_C"]
    mu = mA * (mB + mC) / (mA + mB + mC)
    s_dev = cross_section(C_dev, e, mu, 0)
    s_ref = X.cross_section(C_ref, e, mu, 0)
    bound = math.pi / (2 * mu * e) * (J_max + 1) ** 2 * PE_TOL
    assert np.all(np.abs(s_dev - s_ref) < bound[None, :])
