"""Mixed-precision forms (FP32, BF16x3, FP16x3 contractions with FP64 recursion)
against the FP64 oracle: every state-to-state P(E) within 1e-3 absolute.  Each
case also prints its measured errors."""
import numpy as np
import pytest

from oracle import tdwp_oracle as O
from workloads import asymptotic_potential, config, small_variant

pytestmark = pytest.mark.gpu

PE_MIXED_TOL = 1e-3


@pytest.fixture(scope="module", autouse=True)
def _device():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _oracle(spec, K):
    op = O.Operator(spec)
    pk = spec["packets"][0]
    va = asymptotic_potential(spec, op.r, pk["elec0"])
    e, chi = O.diatomic_states(op, va, pk["j0"], pk["v0"] + 1)
    run = O.propagate(op, 0, O.initial_packet(op, 0, pk, chi[pk["v0"]]), K, keep_vectors=(K,))
    return op, run, e[pk["v0"]]


def _ochans(op, spec, chans):
    out = []
    for c in chans:
        va = asymptotic_potential(spec, op.r, c["elec"])
        e, chi = O.diatomic_states(op, va, c["j"], c["v"] + 1)
        out.append(dict(c, energy=e[c["v"]], chi=chi[c["v"]]))
    return out


@pytest.fixture(scope="module")
def config1_oracle():
    spec = config(1)
    op, run, e0 = _oracle(spec, spec["steps"])
    return spec, op, run, e0


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3", "fp16x3"])
def test_config1_probabilities_per_precision(precision, config1_oracle):
    from paper_2412_10167_amd import problem
    spec, op, run, e0 = config1_oracle
    print(f"\n[case] config 1, {precision}", flush=True)
    plan, _ = problem.build(spec, precision=precision)
    plan.propagate(spec["steps"])
    u = plan.get_packet(0, 0, 0)
    chans = problem.channels(plan, spec, 0, 10, 2)
    p_inel, p_reac = plan.state_to_state(0, 0, chans)
    res = O.analyse(op, 0, spec["packets"][0], run, e0, _ochans(op, spec, chans))
    K = spec["steps"]
    du = np.max(np.abs(u - run["vectors"][K])) / np.max(np.abs(run["vectors"][K]))
    dr = np.max(np.abs(p_reac - res["p_reac"]))
    di = np.max(np.abs(p_inel - res["p_inel"]))
    print(f"[result] {precision}: packet rel {du:.2e}  P_reac {dr:.2e}  P_inel {di:.2e}", flush=True)
    plan.close()
    tol = 1e-8 if precision == "fp64" else PE_MIXED_TOL
    assert dr < tol and di < tol


@pytest.mark.parametrize("fuse", [1, 0])
@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16x3"])
def test_coriolis_two_state_packet_per_precision(precision, fuse):
    from paper_2412_10167_amd import problem
    s = small_variant(3, n_R=22, n_r=18, n_gamma=14)
    s["units"] = [dict(J=5, parity=1, omega_max=3, n_packets=1)]
    s["packets"] = [dict(s["packets"][0], omega0=1, j0=1)]
    K = 60
    print(f"\n[case] J=5 Omega 1..3 2 states, {precision}, r pass "
          f"{'in the angular launch' if fuse else 'after it'}", flush=True)
    plan, _ = problem.build(s, precision=precision)
    plan.set_option("fuse_r", fuse)
    plan.propagate(K)
    op, run, _ = _oracle(s, K)
    du = np.max(np.abs(plan.get_packet(0, 0, 0) - run["vectors"][K])) / np.max(np.abs(run["vectors"][K]))
    print(f"[result] {precision}: packet rel {du:.2e}", flush=True)
    plan.close()
    assert du < {"fp32": 1e-5, "bf16x3": 1e-4, "fp16x3": 1e-4}[precision]


def test_general_path_odd_sizes():
    """Odd grid sizes take the general (non-split) kernels; FP64 parity as usual."""
    from paper_2412_10167_amd import problem
    s = small_variant(1, n_R=21, n_r=17, n_gamma=9)
    K = 80
    print("\n[case] odd sizes 21x17x9 FP64", flush=True)
    plan, _ = problem.build(s)
    plan.propagate(K)
    op, run, _ = _oracle(s, K)
    du = np.max(np.abs(plan.get_packet(0, 0, 0) - run["vectors"][K])) / np.max(np.abs(run["vectors"][K]))
    plan.close()
    assert du < 1e-10


def _wave_cases():
    """(name, spec) cases for the per-wave angular kernel: one helicity, Coriolis
    coupling over two states, and 48 / 40 gamma nodes (three j tiles, capped
    rotational energies at small r) with up to eight helicities."""
    a = small_variant(1, n_R=24, n_r=20, n_gamma=10)
    b = small_variant(3, n_R=22, n_r=18, n_gamma=14)
    b["units"] = [dict(J=5, parity=1, omega_max=3, n_packets=1)]
    b["packets"] = [dict(b["packets"][0], omega0=1, j0=1)]
    c = small_variant(1, n_R=24, n_r=20, n_gamma=48)
    c["units"] = [dict(J=4, parity=1, omega_max=4, n_packets=1)]
    c["packets"] = [dict(c["packets"][0], omega0=0, j0=2)]
    d = small_variant(1, n_R=20, n_r=16, n_gamma=40)
    d["units"] = [dict(J=8, parity=1, omega_max=7, n_packets=1)]
    d["packets"] = [dict(d["packets"][0], omega0=2, j0=3)]
    return [("J=0 24x20x10", a), ("J=5 Omega 1..3, 2 states, 22x18x14", b),
            ("J=4 Omega 0..4, 24x20x48", c), ("J=8 Omega 0..7, 20x16x40", d)]


@pytest.mark.parametrize("precision", ["bf16x3", "fp16x3"])
def test_wave_angular_kernel_per_precision(precision):
    """Angular kernel 3 (columns held per wave) against the FP64 oracle and against
    kernel 2 on the same plan: packets after 60 steps, r pass after the angular
    pass (and the plane pass where the form allows it)."""
    from paper_2412_10167_amd import problem
    K = 60
    for name, s in _wave_cases():
        print(f"\n[case] angular kernel 3, {name}, {precision}", flush=True)
        got = {}
        for kern in (3, 2):
            plan, _ = problem.build(s, precision=precision)
            plan.set_option("fuse_r", 0)
            plan.set_option("ang_kernel", kern)
            assert plan.stat("ang_kernel") == kern
            plan.propagate(K)
            got[kern] = plan.get_packet(0, 0, 0)
            plan.close()
        op, run, _ = _oracle(s, K)
        ref = run["vectors"][K]
        scale = np.max(np.abs(ref))
        du = np.max(np.abs(got[3] - ref)) / scale
        d32 = np.max(np.abs(got[3] - got[2])) / scale
        print(f"[result] {precision}: packet rel {du:.2e}; kernel 3 vs kernel 2 {d32:.2e}", flush=True)
        assert du < 1e-4 and d32 < 1e-4


def test_wave_angular_kernel_is_checked():
    """Kernel 3 is refused where it does not apply: the FP64 form, more than eight
    helicities; with the r pass fused into the angular launch kernel 2 runs."""
    from paper_2412_10167_amd import problem
    from paper_2412_10167_amd.tdwp import TdwpError
    print("\n[case] angular kernel 3: refused for FP64 and for nine helicities", flush=True)
    s = _wave_cases()[1][1]
    plan, _ = problem.build(s)
    with pytest.raises(TdwpError):
        plan.set_option("ang_kernel", 3)
    plan.close()
    plan, _ = problem.build(s, precision="fp16x3")
    plan.set_option("ang_kernel", 3)
    plan.set_option("fuse_r", 1)
    assert plan.stat("ang_kernel") == 2
    plan.set_option("fuse_r", 0)
    assert plan.stat("ang_kernel") == 3
    plan.close()
    e = small_variant(3, n_R=22, n_r=18, n_gamma=24)
    e["units"] = [dict(J=10, parity=1, omega_max=8, n_packets=1)]
    e["packets"] = [dict(e["packets"][0], omega0=1, j0=2)]
    plan, _ = problem.build(e, precision="fp16x3")
    with pytest.raises(TdwpError):
        plan.set_option("ang_kernel", 3)
    plan.close()
