"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

FP64 bars: packet 1e-10 relative (max |diff| / max |u|), P(E) 1e-8 absolute,
index maps and integer layout exact.  Every case prints its name first so a
failing GPU run names it.
"""
import numpy as np
import pytest

from oracle import tdwp_oracle as O
from workloads import asymptotic_potential, config, ev, small_variant

pytestmark = pytest.mark.gpu

PKT_TOL = 1e-10
PE_TOL = 1e-8


@pytest.fixture(scope="module", autouse=True)
def _device():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2412_10167_amd import load_library
    load_library()


def _problem():
    from paper_2412_10167_amd import problem
    return problem


def banner(name):
    print(f"\n[case] {name}", flush=True)


def oracle_packets(spec, K, keep=()):
    """Oracle runs of every packet: dict (unit, slot) -> (op, run, e0, chi0)."""
    op = O.Operator(spec)
    out = {}
    for pk in spec["packets"]:
        va = asymptotic_potential(spec, op.r, pk["elec0"])
        e, chi = O.diatomic_states(op, va, pk["j0"], pk["v0"] + 1)
        u0 = O.initial_packet(op, pk["unit"], pk, chi[pk["v0"]])
        run = O.propagate(op, pk["unit"], u0, K, keep_vectors=keep)
        out[(pk["unit"], pk["slot"])] = (run, e[pk["v0"]], chi[pk["v0"]])
    return op, out


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def oracle_channels(op, spec, chans):
    out = []
    for c in chans:
        va = asymptotic_potential(spec, op.r, c["elec"])
        e, chi = O.diatomic_states(op, va, c["j"], c["v"] + 1)
        out.append(dict(c, energy=e[c["v"]], chi=chi[c["v"]]))
    return out


# ---------------------------------------------------------------------------

def test_plan_tables_match_oracle():
    banner("plan tables: grid, quadrature, bounds, diatomic states")
    spec = small_variant(3, n_R=20, n_r=18, n_gamma=12, steps=10)
    spec["units"] = [dict(J=5, parity=1, omega_max=4, n_packets=1)]
    spec["packets"] = [dict(spec["packets"][0], omega0=1, j0=2)]
    problem = _problem()
    plan, info = problem.build(spec)
    op = O.Operator(spec)
    r, R, x, w = plan.grid()
    assert np.max(np.abs(r - op.r)) < 1e-14 and np.max(np.abs(R - op.R)) < 1e-14
    assert np.max(np.abs(x - op.x)) < 1e-14 and np.max(np.abs(w - op.w)) < 1e-14
    lo, hi = plan.spectral_bounds()
    assert abs(lo - op.Emin) < 1e-13 and abs(hi - op.Emax) < 1e-13 * abs(op.Emax)
    for el in range(spec["n_elec"]):
        va = asymptotic_potential(spec, op.r, el)
        for j in (0, 3):
            eg, cg = plan.diatomic_states(va, j, 4)
            eo, co = O.diatomic_states(op, va, j, 4)
            assert np.max(np.abs(eg - eo)) < 1e-12
            assert np.max(np.abs(cg - co)) < 1e-10
    # odd-parity unit: helicities 1..4 (integer layout)
    assert plan.get_packet(0, 0, 0).shape == (4, 2, 12, 20, 18)
    plan.close()


def test_first_step_packet_j0():
    banner("one step, J=0, 64x48x24")
    spec = config(1)
    problem = _problem()
    plan, _ = problem.build(spec)
    plan.propagate(1)
    op, ref = oracle_packets(spec, 1, keep=(0, 1))
    run = ref[(0, 0)][0]
    assert rel_err(plan.get_packet(0, 0, 1), run["vectors"][0]) < PKT_TOL
    assert rel_err(plan.get_packet(0, 0, 0), run["vectors"][1]) < PKT_TOL
    plan.close()


@pytest.mark.parametrize("name,spec_fn,K", [
    ("J=0 small ragged 24x20x10", lambda: small_variant(1, n_R=24, n_r=20, n_gamma=10), 150),
    ("J=5 p(-1)^J=-1, Omega 1..3, 2 states", lambda: _coriolis_spec(5, 1, 3, 2), 60),
    ("J=20 Omega 0..8, 2 states (config-3 physics)", lambda: _coriolis_spec(20, 1, 8, 2), 60),
    ("J=4 Omega 0..4, 3 states (config-5 physics)", lambda: _coriolis_spec(4, 1, 4, 3, cfg=5), 40),
])
def test_packet_parity(name, spec_fn, K):
    banner(name)
    spec = spec_fn()
    problem = _problem()
    plan, _ = problem.build(spec)
    norms = plan.propagate(K)
    op, ref = oracle_packets(spec, K, keep=(K - 1, K))
    run = ref[(0, 0)][0]
    assert rel_err(plan.get_packet(0, 0, 0), run["vectors"][K]) < PKT_TOL
    assert rel_err(plan.get_packet(0, 0, 1), run["vectors"][K - 1]) < PKT_TOL
    assert np.max(np.abs(norms[0] - run["norms"][1:])) < 1e-12
    plan.close()


def _coriolis_spec(J, parity, omega_max, n_elec, cfg=3):
    s = small_variant(cfg, n_R=22, n_r=18, n_gamma=14)
    s["n_elec"] = n_elec
    s["units"] = [dict(J=J, parity=parity, omega_max=omega_max, n_packets=1)]
    lo = 0 if parity * (-1) ** J == 1 else 1
    s["packets"] = [dict(s["packets"][0], omega0=lo, j0=max(lo, 1))]
    return s


def test_full_config1_probabilities():
    banner("config 1 full: 64x48x24, 2000 steps, P(E) on 200 energies")
    spec = config(1)
    problem = _problem()
    plan, info = problem.build(spec)
    K = spec["steps"]
    norms = plan.propagate(K)
    op, ref = oracle_packets(spec, K, keep=(K,))
    run, e0, chi0 = ref[(0, 0)]
    assert rel_err(plan.get_packet(0, 0, 0), run["vectors"][K]) < PKT_TOL
    assert np.max(np.abs(norms[0] - run["norms"][1:])) < 1e-12
    chans = problem.channels(plan, spec, 0, 10, 2)
    p_inel, p_reac = plan.state_to_state(0, 0, chans)
    res = O.analyse(op, 0, spec["packets"][0], run, e0, oracle_channels(op, spec, chans))
    assert np.max(np.abs(p_reac - res["p_reac"])) < PE_TOL
    assert np.max(np.abs(p_inel - res["p_inel"])) < PE_TOL
    # the same plan continues bit-identically after an analysis call
    plan.close()


def test_chunked_propagation_is_bit_identical():
    banner("chunked == single call (bit-exact)")
    spec = small_variant(1, n_R=24, n_r=20, n_gamma=10)
    problem = _problem()
    a, _ = problem.build(spec)
    b, _ = problem.build(spec)
    na = a.propagate(130)
    nb = np.concatenate([b.propagate(n) for n in (1, 63, 2, 64)], axis=1)
    assert np.array_equal(na, nb)
    assert np.array_equal(a.get_packet(0, 0, 0), b.get_packet(0, 0, 0))
    chans = problem.channels(a, spec, 0, 3, 1)
    pa = a.state_to_state(0, 0, chans)
    pb = b.state_to_state(0, 0, chans)
    assert np.array_equal(pa[0], pb[0]) and np.array_equal(pa[1], pb[1])
    a.close()
    b.close()


def test_batched_units_match_standalone_oracle():
    banner("batch: J=0,2,5(odd) units x 2 packets, uneven helicity counts")
    spec = small_variant(4, n_R=20, n_r=16, n_gamma=10)
    spec["units"] = [dict(J=0, parity=1, omega_max=0, n_packets=2),
                     dict(J=2, parity=1, omega_max=2, n_packets=2),
                     dict(J=5, parity=1, omega_max=3, n_packets=2)]
    base = spec["packets"][0]
    spec["packets"] = []
    for u, lo in ((0, 0), (1, 0), (2, 1)):
        for slot in range(2):
            spec["packets"].append(dict(base, unit=u, slot=slot, j0=max(lo, slot + lo),
                                        omega0=lo, k_min_elastic=30))
    problem = _problem()
    plan, _ = problem.build(spec)
    K = 50
    norms = plan.propagate(K)
    op, ref = oracle_packets(spec, K, keep=(K,))
    for i, pk in enumerate(spec["packets"]):
        run = ref[(pk["unit"], pk["slot"])][0]
        assert rel_err(plan.get_packet(pk["unit"], pk["slot"], 0), run["vectors"][K]) < PKT_TOL
        assert np.max(np.abs(norms[i] - run["norms"][1:])) < 1e-12
    for pk in spec["packets"][::3]:
        run, e0, _ = ref[(pk["unit"], pk["slot"])]
        chans = problem.channels(plan, spec, pk["unit"], 3, 1)
        p_inel, p_reac = plan.state_to_state(pk["unit"], pk["slot"], chans)
        res = O.analyse(op, pk["unit"], pk, run, e0, oracle_channels(op, spec, chans))
        assert np.max(np.abs(p_reac - res["p_reac"])) < PE_TOL
        assert np.max(np.abs(p_inel - res["p_inel"])) < PE_TOL
    plan.close()


def test_two_state_probabilities():
    banner("J=3 Omega 0..2, 2 coupled states: P_reac per state and inelastic")
    spec = _coriolis_spec(3, -1, 2, 2)   # p(-1)^J = +1: Omega 0..2
    spec["steps"] = 300
    spec["n_energy"] = 40
    spec["packets"][0]["k_min_elastic"] = 60
    problem = _problem()
    plan, _ = problem.build(spec)
    plan.propagate(spec["steps"])
    op, ref = oracle_packets(spec, spec["steps"])
    run, e0, _ = ref[(0, 0)]
    chans = problem.channels(plan, spec, 0, 4, 1)
    p_inel, p_reac = plan.state_to_state(0, 0, chans)
    res = O.analyse(op, 0, spec["packets"][0], run, e0, oracle_channels(op, spec, chans))
    assert np.max(np.abs(p_reac - res["p_reac"])) < PE_TOL
    assert np.max(np.abs(p_inel - res["p_inel"])) < PE_TOL
    plan.close()


def test_full_size_config2_first_steps():
    banner("config 2 full size 256x192x80: 6 steps")
    spec = config(2)
    problem = _problem()
    plan, _ = problem.build(spec)
    K = 6
    norms = plan.propagate(K)
    op, ref = oracle_packets(spec, K, keep=(K,))
    run = ref[(0, 0)][0]
    assert rel_err(plan.get_packet(0, 0, 0), run["vectors"][K]) < PKT_TOL
    assert np.max(np.abs(norms[0] - run["norms"][1:])) < 1e-12
    plan.close()


@pytest.mark.parametrize("K", [0, 1])
def test_zero_and_one_step_probabilities(K):
    banner(f"{K} steps: packet, norms and P(E) from the k <= {K} terms (J=5 Omega 1..3, 2 states)")
    spec = _coriolis_spec(5, 1, 3, 2)
    problem = _problem()
    plan, _ = problem.build(spec)
    norms = plan.propagate(K)
    assert norms.shape == (1, K)
    op, ref = oracle_packets(spec, K, keep=(K,))
    run, e0, _ = ref[(0, 0)]
    assert rel_err(plan.get_packet(0, 0, 0), run["vectors"][K]) < PKT_TOL
    chans = problem.channels(plan, spec, 0, 3, 1)
    p_inel, p_reac = plan.state_to_state(0, 0, chans)
    res = O.analyse(op, 0, spec["packets"][0], run, e0, oracle_channels(op, spec, chans))
    assert np.max(np.abs(p_reac - res["p_reac"])) < PE_TOL
    assert np.max(np.abs(p_inel - res["p_inel"])) < PE_TOL
    # no channels: the reactive probabilities alone
    p_none, p_reac2 = plan.state_to_state(0, 0, [])
    assert p_none.shape == (0, spec["n_energy"]) and np.array_equal(p_reac2, p_reac)
    plan.close()


def _full_size_sampled(wl, K, keep):
    """Full-size plan of workload wl on the GPU; the packets in `keep` ((unit, slot)
    pairs) against an oracle run of just their units with the plan's bounds."""
    spec = config(wl)
    problem = _problem()
    plan, _ = problem.build(spec)
    plan.propagate(K)
    lo, hi = plan.spectral_bounds()
    units = sorted({u for u, _ in keep})
    sub = dict(spec)
    sub["units"] = [spec["units"][u] for u in units]
    sub["packets"] = [dict(p, unit=units.index(p["unit"])) for p in spec["packets"]
                      if (p["unit"], p["slot"]) in keep]
    op = O.Operator(sub, bounds=(lo, hi))
    for pk in sub["packets"]:
        va = asymptotic_potential(sub, op.r, pk["elec0"])
        e, chi = O.diatomic_states(op, va, pk["j0"], pk["v0"] + 1)
        u0 = O.initial_packet(op, pk["unit"], pk, chi[pk["v0"]])
        run = O.propagate(op, pk["unit"], u0, K, keep_vectors=(K,))
        got = plan.get_packet(units[pk["unit"]], pk["slot"], 0)
        err = rel_err(got, run["vectors"][K])
        print(f"[result] unit {units[pk['unit']]} slot {pk['slot']}: packet rel {err:.2e}", flush=True)
        assert err < PKT_TOL
    plan.close()


def test_full_size_config3_first_steps():
    banner("config 3 full size 192x160x64, J=20 Omega 0..8, 2 states: 2 steps")
    _full_size_sampled(3, 2, {(0, 0)})


def test_full_size_config4_sampled_packets():
    banner("config 4 full size (21 units x 3 packets, 128x128x48): 2 steps, J=0 and J=40 packets")
    _full_size_sampled(4, 2, {(0, 0), (20, 2)})


def test_full_size_config5_first_step():
    banner("config 5 full size 256x256x96, J=4 Omega 0..4, 3 states: 1 step")
    _full_size_sampled(5, 1, {(0, 0)})


def test_errors_are_reported():
    banner("error paths: ESTATE, ERANGE, EINVAL")
    from paper_2412_10167_amd.tdwp import Plan, TdwpError
    spec = small_variant(1, n_R=16, n_r=12, n_gamma=6)
    plan = Plan(spec)
    with pytest.raises(TdwpError) as e:
        plan.propagate(1)
    assert e.value.code == -4
    plan.close()
    # E_max far below the true spectrum: the recursion diverges and is caught
    problem = _problem()
    plan, _ = problem.build(spec, bounds=(0.0, ev(0.5)))
    with pytest.raises(TdwpError) as e:
        plan.propagate(400)
    assert e.value.code == -5
    with pytest.raises(TdwpError) as e:
        plan.state_to_state(0, 0, [dict(elec=3, v=0, j=0, omega=0, energy=0.0,
                                         chi=np.zeros(spec["n_r"]))])
    assert e.value.code == -1
    plan.close()


def test_graph_replay_bit_identical_to_direct_launches():
    banner("HIP graph replay == direct launches (bit-exact), config-1 shape")
    spec = config(1)
    spec["steps"] = 700
    problem = _problem()
    a, _ = problem.build(spec)
    b, _ = problem.build(spec)
    b.set_option("graphs", 0)
    na = a.propagate(300)
    na2 = a.propagate(400)
    nb = b.propagate(700)
    assert a.stat("graph_steps") > 500 and b.stat("graph_steps") == 0
    assert np.array_equal(np.concatenate([na, na2], axis=1), nb)
    assert np.array_equal(a.get_packet(0, 0, 0), b.get_packet(0, 0, 0))
    chans = problem.channels(a, spec, 0, 4, 1)
    pa, pb = a.state_to_state(0, 0, chans), b.state_to_state(0, 0, chans)
    assert np.array_equal(pa[0], pb[0]) and np.array_equal(pa[1], pb[1])
    a.close()
    b.close()


@pytest.mark.parametrize("nt", [1, 2, 4])
def test_angular_tile_variants(nt):
    banner(f"angular tile {nt}: J=0 24x20x10 and J=5 Omega 1..3 2 states")
    problem = _problem()
    for spec in (small_variant(1, n_R=24, n_r=20, n_gamma=10), _coriolis_spec(5, 1, 3, 2)):
        plan, _ = problem.build(spec)
        try:
            plan.set_option("ang_tile", nt)
        except Exception:
            plan.close()
            continue    # variant not feasible for this shape
        K = 40
        plan.propagate(K)
        op, ref = oracle_packets(spec, K, keep=(K,))
        assert rel_err(plan.get_packet(0, 0, 0), ref[(0, 0)][0]["vectors"][K]) < PKT_TOL
        assert plan.stat("ang_tile") == nt
        plan.close()


@pytest.mark.parametrize("fuse", [1, 0])
@pytest.mark.parametrize("kernel", [1, 2])
def test_angular_kernels(kernel, fuse):
    banner(f"angular kernel {kernel}, r pass {'in the same launch' if fuse else 'after it'}: "
           "J=0, J=5 Omega 1..3 2 states, J=20 Omega 0..8 2 states")
    problem = _problem()
    for spec in (small_variant(1, n_R=24, n_r=20, n_gamma=10), _coriolis_spec(5, 1, 3, 2),
                 _coriolis_spec(20, 1, 8, 2)):
        plan, _ = problem.build(spec)
        plan.set_option("ang_kernel", kernel)
        plan.set_option("fuse_r", fuse)
        plan.set_option("ang_xcd", fuse)   # both block orders of the angular pass
        assert plan.stat("ang_kernel") == kernel and plan.stat("fuse_r") == fuse
        K = 40
        plan.propagate(K)
        op, ref = oracle_packets(spec, K, keep=(K,))
        assert rel_err(plan.get_packet(0, 0, 0), ref[(0, 0)][0]["vectors"][K]) < PKT_TOL
        plan.close()


@pytest.mark.parametrize("grid", [1, 7])
def test_radial_grid_is_bit_identical(grid):
    banner(f"radial passes on {grid} looping workgroups == one workgroup per block")
    spec = _coriolis_spec(5, 1, 3, 2)
    problem = _problem()
    a, _ = problem.build(spec)
    b, _ = problem.build(spec)
    b.set_option("radial_grid", grid)
    na, nb = a.propagate(45), b.propagate(45)
    assert np.array_equal(na, nb)
    assert np.array_equal(a.get_packet(0, 0, 0), b.get_packet(0, 0, 0))
    chans = problem.channels(a, spec, 0, 3, 1)
    pa, pb = a.state_to_state(0, 0, chans), b.state_to_state(0, 0, chans)
    assert np.array_equal(pa[0], pb[0]) and np.array_equal(pa[1], pb[1])
    a.close()
    b.close()


def test_autotune_then_parity():
    banner("autotune before packets, then FP64 parity")
    spec = _coriolis_spec(4, 1, 4, 3, cfg=5)
    problem = _problem()
    plan, info = problem.build(spec, autotune=2)
    print("[result] autotune", info["autotune"], flush=True)
    K = 30
    plan.propagate(K)
    op, ref = oracle_packets(spec, K, keep=(K,))
    assert rel_err(plan.get_packet(0, 0, 0), ref[(0, 0)][0]["vectors"][K]) < PKT_TOL
    plan.close()


def test_step_variant_options_are_checked():
    banner("launch-form and block-order options: values checked, state reported")
    from paper_2412_10167_amd.tdwp import TdwpError
    problem = _problem()
    plan, _ = problem.build(small_variant(1, n_R=24, n_r=20, n_gamma=10))
    for name in ("fuse_r", "ang_xcd"):
        for bad in (-1, 2):
            with pytest.raises(TdwpError):
                plan.set_option(name, bad)
    for fuse in (0, 1):
        plan.set_option("fuse_r", fuse)
        assert plan.stat("fuse_r") == fuse
    plan.close()
