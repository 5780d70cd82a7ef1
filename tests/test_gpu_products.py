"""Product-arrangement analysis from reactant coordinates (J = 0) on the HIP path
against the oracle: the product grid and channel functions, and the product
state-to-state probabilities |S'|^2 after the same propagation.

Bar: FP64 within 1e-8 absolute (the collision probabilities' bar), the mixed
forms within 1e-3.  Each case prints its name first."""
import numpy as np
import pytest

from oracle import products_oracle as PR
from oracle import tdwp_oracle as O
from workloads import asymptotic_potential, config

pytestmark = pytest.mark.gpu

PE_TOL = 1e-8
PE_MIXED_TOL = 1e-3


@pytest.fixture(scope="module", autouse=True)
def _device():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def banner(name):
    print(f"\n[case] {name}", flush=True)


def _spec(arrangement="C", units=None, n_R=32, n_r=28, n_gamma=12):
    s = config(1)
    s.update(n_R=n_R, n_r=n_r, n_gamma=n_gamma, n_energy=40)
    s["R_min"], s["R_max"], s["r_min"], s["r_max"] = 0.5, 9.0, 0.5, 9.0
    for ax in ("r", "R"):
        st = 9.0 - 0.2 * 8.5
        s[f"abs_{ax}_start"], s[f"abs_{ax}_strength"] = st, 0.5 / (9.0 - st) ** 2
    s["r_flux"], s["R_inf"] = 4.5, 6.8
    s["units"] = units or [dict(J=0, parity=1, omega_max=0, n_packets=1)]
    base = dict(s["packets"][0], R0=5.2, k_min_elastic=0)
    s["packets"] = [dict(base, unit=u, slot=q, j0=q, omega0=0)
                    for u, un in enumerate(s["units"]) for q in range(un["n_packets"])]
    s["products"] = dict(arrangement=arrangement, R_inf=5.5, n_r=24, r_min=0.6, r_max=4.2, n_gamma=10)
    return s


def _oracle(spec, K, unit=0, slot=0):
    op = O.Operator(spec)
    pr = spec["products"]
    prod = PR.Products(op, pr["arrangement"], pr["R_inf"], pr["n_r"], pr["r_min"], pr["r_max"],
                       pr["n_gamma"])
    sub = dict(spec)
    sub["units"] = [spec["units"][unit]]
    pk = [dict(p, unit=0) for p in spec["packets"] if p["unit"] == unit and p["slot"] == slot][0]
    op1 = O.Operator(sub, bounds=(op.Emin, op.Emax))
    prod1 = PR.Products(op1, pr["arrangement"], pr["R_inf"], pr["n_r"], pr["r_min"], pr["r_max"],
                        pr["n_gamma"])
    va = asymptotic_potential(spec, op1.r, pk["elec0"])
    e, chi = O.diatomic_states(op1, va, pk["j0"], pk["v0"] + 1)
    run = O.propagate(op1, 0, O.initial_packet(op1, 0, pk, chi[pk["v0"]]), K,
                      line_fn=lambda u: PR.product_line(op1, prod1, u))
    return op1, prod1, pk, run, e[pk["v0"]]


def _channels(prod, spec, jmax=5, vmax=2):
    out = []
    va = asymptotic_potential(spec, prod.r, 0)
    for j in range(jmax + 1):
        e, chi = prod.diatomic_states(va, j, vmax + 1)
        for v in range(vmax + 1):
            out.append(dict(elec=0, v=v, j=j, energy=float(e[v]), chi=chi[v]))
    return out


@pytest.mark.parametrize("arr", ["C", "B"])
def test_product_grid_and_channels_match_oracle(arr):
    banner(f"product grid and channel functions, arrangement {arr}")
    from paper_2412_10167_amd import problem
    spec = _spec(arr)
    plan, _ = problem.build(spec)
    r, x, w = plan.product_grid()
    op = O.Operator(spec)
    pr = spec["products"]
    prod = PR.Products(op, arr, pr["R_inf"], pr["n_r"], pr["r_min"], pr["r_max"], pr["n_gamma"])
    assert np.max(np.abs(r - prod.r)) < 1e-14 and np.max(np.abs(x - prod.x)) < 1e-14
    assert np.max(np.abs(w - prod.w)) < 1e-14
    va = asymptotic_potential(spec, prod.r, 0)
    for j in (0, 4):
        eg, cg = plan.product_diatomic_states(va, j, 3)
        eo, co = prod.diatomic_states(va, j, 3)
        assert np.max(np.abs(eg - eo)) < 1e-12 and np.max(np.abs(cg - co)) < 1e-10
    plan.close()


@pytest.mark.parametrize("arr,precision,K", [("C", "fp64", 300), ("B", "fp64", 300),
                                             ("C", "fp16x3", 300)])
def test_product_probabilities_match_oracle(arr, precision, K):
    banner(f"product probabilities, arrangement {arr}, {precision}, {K} steps (32x28x12)")
    from paper_2412_10167_amd import problem
    spec = _spec(arr)
    plan, _ = problem.build(spec, precision=precision)
    if precision != "fp64":
        plan.set_option("plane_r", 1)
    plan.propagate(K)
    op, prod, pk, run, e0 = _oracle(spec, K)
    chans = _channels(prod, spec)
    got = plan.state_to_state_products(0, 0, chans)
    want = PR.analyse_products(op, prod, pk, run["lines"], e0, chans)
    err = float(np.max(np.abs(got - want)))
    print(f"[result] max |P'| {np.max(want):.3e}, sum over channels max "
          f"{np.max(want.sum(0)):.3e}; max |diff| {err:.2e}", flush=True)
    assert np.max(want) > 1e-6
    assert err < (PE_TOL if precision == "fp64" else PE_MIXED_TOL)
    plan.close()


def test_products_in_a_batch_and_graph_replay():
    banner("products in a batch (J=0 x2 with a line, J=2 without), graphs == direct launches")
    from paper_2412_10167_amd import problem
    from paper_2412_10167_amd.tdwp import TdwpError
    spec = _spec("C", units=[dict(J=0, parity=1, omega_max=0, n_packets=2),
                             dict(J=2, parity=1, omega_max=2, n_packets=1)])
    a, _ = problem.build(spec)
    b, _ = problem.build(spec)
    b.set_option("graphs", 0)
    K = 120
    na = np.concatenate([a.propagate(n) for n in (50, 1, 69)], axis=1)
    nb = b.propagate(K)
    assert np.array_equal(na, nb) and a.stat("graph_steps") > 60
    op, prod, pk, run, e0 = _oracle(spec, K, unit=0, slot=1)
    chans = _channels(prod, spec, jmax=3, vmax=1)
    ga = a.state_to_state_products(0, 1, chans)
    gb = b.state_to_state_products(0, 1, chans)
    assert np.array_equal(ga, gb)
    want = PR.analyse_products(op, prod, pk, run["lines"], e0, chans)
    err = float(np.max(np.abs(ga - want)))
    print(f"[result] J=0 slot 1 in the batch: max |diff| {err:.2e}", flush=True)
    assert err < PE_TOL
    with pytest.raises(TdwpError) as e:
        a.state_to_state_products(1, 0, chans)   # the J = 2 unit records no product line
    assert e.value.code == -1
    a.close()
    b.close()


def test_products_need_the_matrix_core_path():
    banner("a product arrangement on odd grid sizes (general kernels) is refused")
    from paper_2412_10167_amd.tdwp import Plan, TdwpError
    spec = _spec("C", n_R=31, n_r=27, n_gamma=11)
    with pytest.raises(TdwpError) as e:
        Plan(spec)
    assert e.value.code == -1
