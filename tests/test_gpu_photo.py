"""Photodissociation packets on the HIP path (through the C ABI) against the
oracle: the autocorrelation C_k = <u_0|u_k> formed on the device after every
step (Eqs. fourier-transform, chebyshev-transform), and the energy content
a_0(E) from it.

Bar: FP64 forms within 1e-10 C_0 at every k (the packet bar, 1e-10 of the
largest value, bounds the overlap far below that); the mixed forms within 1e-4
C_0.  a_0(E) within the bound those differences imply through Eq.
chebyshev-transform.  Each case prints its name first.
"""
import math

import numpy as np
import pytest

from oracle import photo_oracle as PH
from oracle import tdwp_oracle as O
from workloads import asymptotic_potential, config, small_variant
from workloads.photo import photo_packet

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2412_10167_amd import load_library
    load_library()


def banner(name):
    print(f"\n[case] {name}", flush=True)


def _photo_plan(spec, precision="fp64"):
    from paper_2412_10167_amd import problem
    from paper_2412_10167_amd.tdwp import Plan
    plan = Plan(spec, precision=precision)
    plan.set_potential(problem.potential_table(plan, spec))
    return plan


def _device_packet(plan, spec, unit, seed=0):
    r, R, x, w = plan.grid()
    return photo_packet(spec, unit, r, R, x, w, seed=seed)


def _oracle_series(spec, unit, K, seed=0):
    op = O.Operator(spec)
    u0 = photo_packet(spec, unit, op.r, op.R, op.x, op.w, seed=seed)
    return op, PH.autocorrelation(op, unit, u0, K)


def _spec_2state_J1(n_R=21, n_r=17, n_gamma=9):
    s = small_variant(3, n_R=n_R, n_r=n_r, n_gamma=n_gamma)
    s["units"] = [dict(J=1, parity=-1, omega_max=1, n_packets=1)]
    s["packets"] = []
    return s


CASES = [
    ("J=0 24x20x10 fp64 (matrix-core kernels)", lambda: small_variant(1, n_R=24, n_r=20, n_gamma=10),
     "fp64", 150, 1e-10),
    ("J=1 Omega 0..1, 2 states, 21x17x9 fp64 (general kernels)", _spec_2state_J1, "fp64", 80, 1e-10),
    ("J=0 24x20x10 fp16x3", lambda: small_variant(1, n_R=24, n_r=20, n_gamma=10), "fp16x3", 150, 1e-4),
    ("J=1 Omega 0..1, 2 states, 22x18x10 fp64 (matrix-core kernels, overlaps in the R pass)",
     lambda: _spec_2state_J1(22, 18, 10), "fp64", 80, 1e-10),
    ("J=1 Omega 0..1, 2 states, 22x18x10 bf16x3", lambda: _spec_2state_J1(22, 18, 10), "bf16x3", 80,
     1e-4),
    ("J=0 24x20x10 fp32", lambda: small_variant(1, n_R=24, n_r=20, n_gamma=10), "fp32", 150, 1e-4),
]


@pytest.mark.parametrize("name, spec_fn, precision, K, tol", CASES)
def test_autocorrelation_matches_oracle(name, spec_fn, precision, K, tol):
    banner(f"photodissociation autocorrelation: {name}, {K} steps")
    spec = spec_fn()
    spec["units"] = [dict(u, n_packets=1) for u in spec["units"]][:1]
    plan = _photo_plan(spec, precision)
    plan.set_packet_values(0, 0, _device_packet(plan, spec, 0))
    plan.propagate(K // 2, norms=False)      # two calls: the series continues across them
    plan.propagate(K - K // 2, norms=False)
    C = plan.autocorrelation(0, 0)
    e_min, e_max = plan.spectral_bounds()
    plan.close()
    op, ref = _oracle_series(spec, 0, K)
    assert C.shape == (K + 1,)
    assert abs(C[0] - ref[0]) <= 1e-13 * ref[0]
    err = float(np.max(np.abs(C - ref)))
    assert err <= tol * ref[0], err
    # energy content from both series
    E = np.linspace(op.Emin + 0.05 * (op.Emax - op.Emin), op.Emin + 0.5 * (op.Emax - op.Emin), 41)
    from paper_2412_10167_amd import energy_content
    a_dev = energy_content(C, e_min, e_max, E)
    a_ref = PH.energy_content(ref, op.Emin, op.Emax, E)
    th = np.arccos((E - op.E0) / op.dE)
    bound = (2 * K + 1) * max(err, 1e-300) / (math.pi * op.dE * np.sin(th)) \
        + 1e-12 * np.max(np.abs(a_ref))
    assert np.all(np.abs(a_dev - a_ref) <= bound)


@pytest.mark.parametrize("precision, tol", [("fp64", 1e-10), ("fp16x3", 1e-4)])
def test_full_size_workload2_photo_first_steps(precision, tol):
    banner(f"photodissociation at full size 256x192x80, {precision}, autotuned launch form: 6 steps")
    spec = config(2)
    plan = _photo_plan(spec, precision)
    plan.autotune(2)                          # the benchmark's launch configuration
    plan.set_packet_values(0, 0, _device_packet(plan, spec, 0))
    K = 6
    plan.propagate(K, norms=False)
    C = plan.autocorrelation(0, 0)
    lo, hi = plan.spectral_bounds()
    plan.close()
    op = O.Operator(spec, bounds=(lo, hi))
    ref = PH.autocorrelation(op, 0, photo_packet(spec, 0, op.r, op.R, op.x, op.w), K)
    err = float(np.max(np.abs(C - ref)))
    print(f"[result] max |C_k - oracle| / C_0 = {err / ref[0]:.2e}", flush=True)
    assert err <= tol * ref[0]


def test_autocorrelation_across_readback_chunks():
    # 4,100 steps in one call: the partial sums are read back every 4,096 steps
    banner("photodissociation autocorrelation over 4100 steps in one call, J=0 15x12x6 fp64 "
           "(general kernels)")
    spec = small_variant(1, n_R=15, n_r=12, n_gamma=6)
    plan = _photo_plan(spec)
    plan.set_packet_values(0, 0, _device_packet(plan, spec, 0))
    K = 4100
    plan.propagate(K, norms=False)
    C = plan.autocorrelation(0, 0)
    assert plan.autocorrelation(0, 0, n=0).shape == (0,)
    plan.close()
    _, ref = _oracle_series(spec, 0, K)
    assert C.shape == (K + 1,)
    assert float(np.max(np.abs(C - ref))) <= 1e-10 * ref[0]


def test_photo_and_collision_packets_share_a_plan():
    banner("batch: collision packet (slot 0) and photodissociation packet (slot 1), J=0 24x20x10")
    from paper_2412_10167_amd import problem
    from paper_2412_10167_amd.tdwp import TdwpError
    spec = small_variant(1, n_R=24, n_r=20, n_gamma=10)
    spec["units"] = [dict(spec["units"][0], n_packets=2)]
    spec["packets"] = [dict(spec["packets"][0], k_min_elastic=30)]
    plan, info = problem.build(spec)                  # installs the collision packet, slot 0
    plan.set_packet_values(0, 1, _device_packet(plan, spec, 0))
    K = 60
    plan.propagate(K, norms=False)
    C = plan.autocorrelation(0, 1)
    with pytest.raises(TdwpError):
        plan.autocorrelation(0, 0)                    # not a photodissociation packet
    chans = problem.channels(plan, spec, 0, 2, 0)
    with pytest.raises(TdwpError):
        plan.state_to_state(0, 1, chans)              # no collision analysis for it
    p_inel, p_reac = plan.state_to_state(0, 0, chans)
    plan.close()
    op, ref = _oracle_series(spec, 0, K)
    assert float(np.max(np.abs(C - ref))) <= 1e-10 * ref[0]
    # the collision packet is unaffected by its neighbour
    pk = spec["packets"][0]
    va = asymptotic_potential(spec, op.r, pk["elec0"])
    e0, chi0 = O.diatomic_states(op, va, pk["j0"], 1)
    run = O.propagate(op, 0, O.initial_packet(op, 0, pk, chi0[0]), K)
    och = []
    for c in chans:
        vc = asymptotic_potential(spec, op.r, c["elec"])
        ec, chic = O.diatomic_states(op, vc, c["j"], c["v"] + 1)
        och.append(dict(c, energy=ec[c["v"]], chi=chic[c["v"]]))
    res = O.analyse(op, 0, pk, run, e0[0], och)
    assert np.max(np.abs(p_reac - res["p_reac"])) < 1e-8
    assert np.max(np.abs(p_inel - res["p_inel"])) < 1e-8


def test_photo_packet_errors():
    banner("photodissociation entry points: invalid values and order")
    from paper_2412_10167_amd.tdwp import TdwpError
    spec = small_variant(1, n_R=16, n_r=12, n_gamma=6)
    plan = _photo_plan(spec)
    u = _device_packet(plan, spec, 0)
    with pytest.raises(TdwpError):
        plan.set_packet_values(0, 0, np.zeros_like(u))      # zero packet
    bad = u.copy()
    bad.flat[3] = np.nan
    with pytest.raises(TdwpError):
        plan.set_packet_values(0, 0, bad)                     # not finite
    with pytest.raises(TdwpError):
        plan.set_packet_values(0, 5, u)                       # no such slot
    plan.set_packet_values(0, 0, u)
    plan.propagate(3, norms=False)
    assert plan.autocorrelation(0, 0).shape == (4,)
    with pytest.raises(TdwpError):
        plan.autocorrelation(0, 0, n=5)                       # beyond the current step
    plan.close()


def test_photodissociation_from_a_lanczos_bound_state():
    banner("photodissociation: Lanczos bound state on a ground-state well, times the dipole, "
           "propagated; J=0 24x20x10 fp64")
    from paper_2412_10167_amd.tdwp import Plan
    from workloads.photo import bound_spec, dipole_times, ground_state_table
    spec = small_variant(1, n_R=24, n_r=20, n_gamma=10)
    bspec = bound_spec(spec)
    bplan = Plan(bspec)
    r, R, x, _ = bplan.grid()
    bplan.set_potential(ground_state_table(bspec, r, R, x))
    guess = np.exp(-((R[:, None] - 3.0) / 0.5) ** 2 - ((r[None, :] - 1.4) / 0.3) ** 2)
    guess = np.broadcast_to(guess, (len(x),) + guess.shape).copy()
    E_i, psi, res = bplan.lowest_state(guess, n_iter=300)
    bplan.close()
    psi = psi * np.sign(psi.flat[np.argmax(np.abs(psi))])
    opb0 = O.Operator(bspec)
    opb = O.Operator(bspec, vtable=ground_state_table(bspec, opb0.r, opb0.R, opb0.x))
    E_ref, psi_ref = PH.lowest_state(opb, 0)
    ov = abs(float(np.sum(psi * psi_ref.reshape(psi.shape))))
    print(f"[result] bound state E {E_i:.12f} vs dense {E_ref:.12f}; overlap {ov:.12f}; "
          f"residual {res:.1e}", flush=True)
    assert abs(E_i - E_ref) <= 1e-9 * abs(E_ref) and ov > 1 - 1e-8
    # the photodissociation packet from each side's bound state
    plan = _photo_plan(spec)
    rr, RR, xx, _ = plan.grid()
    u_dev = dipole_times(spec, 0, rr, RR, xx, psi)
    plan.set_packet_values(0, 0, u_dev)
    K = 120
    plan.propagate(K, norms=False)
    C = plan.autocorrelation(0, 0)
    lo, hi = plan.spectral_bounds()
    plan.close()
    op = O.Operator(spec, bounds=(lo, hi))
    u_ref = dipole_times(spec, 0, op.r, op.R, op.x, psi_ref)
    ref = PH.autocorrelation(op, 0, u_ref, K)
    err = float(np.max(np.abs(C - ref)))
    # the two bound states agree to an overlap of 1 - O(1e-13), i.e. vectors to
    # O(1e-7); C_k = <u_0|u_k> is bilinear in the packet and the damped recursion
    # does not grow it, so |dC_k| <= (2 |u_0| + |du_0|) |du_0|, plus the FP64 step's bar
    du = float(np.linalg.norm(u_dev - u_ref))
    bound = (2 * np.sqrt(ref[0]) + du) * du + 1e-10 * ref[0]
    print(f"[result] autocorrelation max |C - oracle| / C_0 = {err / ref[0]:.2e} "
          f"(packets differ by {du:.1e}; bound {bound / ref[0]:.1e} C_0)", flush=True)
    assert err <= bound


def test_photo_packet_replaced_by_a_collision_packet():
    banner("slot switched from a photodissociation packet to a collision packet, J=0 24x20x10 fp64")
    from paper_2412_10167_amd import problem
    from paper_2412_10167_amd.tdwp import TdwpError
    spec = small_variant(1, n_R=24, n_r=20, n_gamma=10)
    plan = _photo_plan(spec)
    plan.set_packet_values(0, 0, _device_packet(plan, spec, 0))
    plan.propagate(30, norms=False)                 # overlaps in the R pass, graphs captured
    problem.install_packets(plan, spec)             # the same slot as a collision packet
    with pytest.raises(TdwpError):
        plan.autocorrelation(0, 0)
    K = 60
    plan.propagate(K)
    got = plan.get_packet(0, 0, 0)
    lo, hi = plan.spectral_bounds()
    plan.close()
    op = O.Operator(spec, bounds=(lo, hi))
    pk = spec["packets"][0]
    va = asymptotic_potential(spec, op.r, pk["elec0"])
    e, chi = O.diatomic_states(op, va, pk["j0"], 1)
    run = O.propagate(op, 0, O.initial_packet(op, 0, pk, chi[0]), K, keep_vectors=(K,))
    ref = run["vectors"][K]
    assert float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))) < 1e-10


# ---- the initial packet of Eq. initial-photo-wvp built by the library ------------------------

@pytest.mark.parametrize("J,par,omega_max,Ji,Mi,pari,om_lo_i,n_om_i,pol", [
    (1, -1, 1, 0, 0, 1, 0, 1, 0),     # J_i = 0 -> J = 1, linear
    (2, 1, 2, 1, 1, -1, 1, 1, -1),    # J_i = 1 (Omega_i = 1) -> J = 2, circular
    (3, -1, 2, 2, 0, 1, 0, 3, 0),     # three bound helicities, final helicities truncated at 2
    (2, 1, 2, 2, -1, -1, 1, 2, 1),    # same J, p_i (-1)^J_i = -1 (no Omega_i = 0)
])
def test_photo_packet_matches_oracle(J, par, omega_max, Ji, Mi, pari, om_lo_i, n_om_i, pol):
    banner(f"photodissociation packet J_i={Ji} M_i={Mi} p_i={pari} -> J={J} p={par} "
           f"(Omega <= {omega_max}), polarisation {pol}: library vs oracle, then 30 steps")
    from workloads.photo import bound_components, dipole_components
    spec = small_variant(3, n_R=21, n_r=17, n_gamma=9)
    spec["units"] = [dict(J=J, parity=par, omega_max=omega_max, n_packets=1)]
    spec["packets"] = []
    plan = _photo_plan(spec)
    r, R, x, w = plan.grid()
    bound = bound_components(r, R, x, w, n_om_i)
    dip = dipole_components(r, R, x)
    elec = spec["n_elec"] - 1
    plan.photo_packet(0, 0, elec, Ji, Mi, pari, om_lo_i, bound, dip, pol)
    got = plan.get_packet(0, 0, 0)
    want = PH.photo_packet(spec, 0, elec, Ji, Mi, pari, list(range(om_lo_i, om_lo_i + n_om_i)),
                           bound, dip, pol)
    err = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    print(f"[result] packet rel {err:.2e}; block norms "
          + " ".join(f"{float(np.sum(want[a] ** 2)):.3e}" for a in range(want.shape[0])), flush=True)
    assert err < 1e-14
    K = 30
    plan.propagate(K, norms=False)
    C = plan.autocorrelation(0, 0)
    op = O.Operator(spec)
    Cref = PH.autocorrelation(op, 0, want, K)
    dc = float(np.max(np.abs(C - Cref)) / Cref[0])
    print(f"[result] autocorrelation rel {dc:.2e}", flush=True)
    assert dc < 1e-10
    plan.close()


def test_photo_packet_rejects_invalid_transitions():
    banner("photodissociation packet: invalid quantum numbers and forbidden transitions rejected")
    from paper_2412_10167_amd.tdwp import TdwpError
    from workloads.photo import bound_components, dipole_components
    spec = small_variant(3, n_R=21, n_r=17, n_gamma=9)
    spec["units"] = [dict(J=1, parity=1, omega_max=1, n_packets=1)]
    spec["packets"] = []
    plan = _photo_plan(spec)
    r, R, x, w = plan.grid()
    b1, dip = bound_components(r, R, x, w, 1), dipole_components(r, R, x)
    bad = [dict(Ji=0, Mi=1, pari=1, om=0, pol=0),      # |M_i| > J_i
           dict(Ji=1, Mi=0, pari=1, om=0, pol=0),      # Omega_i = 0 with p_i (-1)^J_i = -1
           dict(Ji=3, Mi=3, pari=1, om=0, pol=1),      # |M_i + pol| above the final J
           dict(Ji=0, Mi=0, pari=1, om=0, pol=0)]      # in-plane dipole cannot reach p = +1, J = 1
    for c in bad:
        with pytest.raises(TdwpError) as e:
            plan.photo_packet(0, 0, 0, c["Ji"], c["Mi"], c["pari"], c["om"], b1, dip, c["pol"])
        assert e.value.code == -1
    plan.close()
