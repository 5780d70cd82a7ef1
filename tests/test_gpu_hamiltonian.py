"""H u by the library's step kernels (tdwp_apply_hamiltonian; Eq. hamiltonian with
its caps, no damping) against the oracle's H application.

Bar: FP64 within 1e-11 of max |H u| (one application; the propagated packet's
bar is 1e-10 after many); fp16x3 within 1e-5 (split contractions, 2^-22 of the
contraction's scale).  A plan used for H u propagates afterwards as one that
never was (the damping restored), checked against the oracle.
"""
import numpy as np
import pytest

from oracle import tdwp_oracle as O
from workloads import asymptotic_potential, small_variant

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


def _coriolis_spec(J, parity, omega_max, n_elec, n_R, n_r, n_gamma, cfg=3):
    s = small_variant(cfg, n_R=n_R, n_r=n_r, n_gamma=n_gamma)
    s["n_elec"] = n_elec
    s["units"] = [dict(J=J, parity=parity, omega_max=omega_max, n_packets=1)]
    lo = 0 if parity * (-1) ** J == 1 else 1
    s["packets"] = [dict(s["packets"][0], omega0=lo, j0=max(lo, 1))]
    return s


def _bare_plan(spec, precision):
    from paper_2412_10167_amd import problem
    from paper_2412_10167_amd.tdwp import Plan
    plan = Plan(spec, precision=precision)
    plan.set_potential(problem.potential_table(plan, spec))
    return plan


CASES = [
    ("J=0 24x20x10 fp64 (matrix-core kernels)", lambda: small_variant(1, n_R=24, n_r=20, n_gamma=10),
     "fp64", 1e-11),
    ("J=5 p(-1)^J=-1 Omega 1..3, 2 states, 22x18x14 fp64 (matrix-core kernels)",
     lambda: _coriolis_spec(5, 1, 3, 2, 22, 18, 14), "fp64", 1e-11),
    ("J=2 Omega 0..2, 2 states, 21x17x9 fp64 (general kernels)",
     lambda: _coriolis_spec(2, 1, 2, 2, 21, 17, 9), "fp64", 1e-11),
    ("J=0 24x20x10 fp16x3", lambda: small_variant(1, n_R=24, n_r=20, n_gamma=10), "fp16x3", 1e-5),
]


@pytest.mark.parametrize("name, spec_fn, precision, tol", CASES)
def test_apply_hamiltonian_matches_oracle(name, spec_fn, precision, tol):
    banner(f"H u: {name}")
    spec = spec_fn()
    plan = _bare_plan(spec, precision)
    lo, hi = plan.spectral_bounds()
    op = O.Operator(spec, bounds=(lo, hi))
    rng = np.random.default_rng(17)
    shape = op.unit_shape(0)
    for trial in range(2):                    # the second call reuses the plan
        u = rng.standard_normal(shape)
        got = plan.apply_hamiltonian(u)
        ref = O.apply_H(op, 0, u)
        err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
        print(f"[result] trial {trial}: max |Hu - oracle| / max |Hu| = {err:.2e}", flush=True)
        assert err < tol
    plan.close()


def test_apply_hamiltonian_order_and_propagation_after_it():
    banner("H u refused with a packet installed; propagation after H u matches the oracle")
    from paper_2412_10167_amd import problem
    from paper_2412_10167_amd.tdwp import TdwpError
    spec = small_variant(1, n_R=24, n_r=20, n_gamma=10)
    plan = _bare_plan(spec, "fp64")
    u = np.random.default_rng(3).standard_normal(O.Operator(spec).unit_shape(0))
    plan.apply_hamiltonian(u)
    with pytest.raises(TdwpError):
        plan.apply_hamiltonian(u, unit=0, slot=3)             # no such packet
    problem.install_packets(plan, spec)
    with pytest.raises(TdwpError):
        plan.apply_hamiltonian(u)                              # a packet is installed
    K = 40
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


@pytest.mark.parametrize("name, spec_fn, n_iter", [
    ("J=0 16x12x6 (matrix-core kernels)", lambda: small_variant(1, n_R=16, n_r=12, n_gamma=6), 400),
    ("J=1 Omega 0..1, 2 states, 13x11x5 (general kernels)",
     lambda: _coriolis_spec(1, -1, 1, 2, 13, 11, 5), 400),
])
def test_lowest_state_matches_dense_eigensolver(name, spec_fn, n_iter):
    banner(f"bound state by the library's Lanczos iteration: {name}, {n_iter} steps")
    from oracle import photo_oracle as PH
    spec = spec_fn()
    plan = _bare_plan(spec, "fp64")
    lo, hi = plan.spectral_bounds()
    op = O.Operator(spec, bounds=(lo, hi))
    guess = np.random.default_rng(5).standard_normal(op.unit_shape(0))
    E, psi, res = plan.lowest_state(guess, n_iter=n_iter)
    plan.close()
    E_ref, psi_ref = PH.lowest_state(op, 0)
    ov = abs(float(np.sum(psi * psi_ref)))
    print(f"[result] E {E:.12f} vs dense {E_ref:.12f} (rel {abs(E - E_ref) / abs(E_ref):.1e}); "
          f"|<psi|psi_ref>| = {ov:.12f}; residual {res:.1e}", flush=True)
    assert abs(E - E_ref) <= 1e-9 * abs(E_ref)
    assert ov > 1 - 1e-8
    assert res < 1e-5 * abs(E_ref)


def test_lowest_state_mixed_form_and_errors():
    banner("bound state in the fp16x3 form; invalid iteration counts, guesses and order")
    from oracle import photo_oracle as PH
    from paper_2412_10167_amd import problem
    from paper_2412_10167_amd.tdwp import TdwpError
    spec = small_variant(1, n_R=16, n_r=12, n_gamma=6)
    plan = _bare_plan(spec, "fp16x3")
    lo, hi = plan.spectral_bounds()
    op = O.Operator(spec, bounds=(lo, hi))
    guess = np.random.default_rng(5).standard_normal(op.unit_shape(0))
    E, psi, res = plan.lowest_state(guess, n_iter=300)
    E_ref, psi_ref = PH.lowest_state(op, 0)
    ov = abs(float(np.sum(psi * psi_ref)))
    print(f"[result] fp16x3: E rel {abs(E - E_ref) / abs(E_ref):.1e}, overlap 1 - {1 - ov:.1e}",
          flush=True)
    # the split contractions carry 2^-22 of the contraction scale into H u
    assert abs(E - E_ref) <= 1e-5 * abs(E_ref) and ov > 1 - 1e-6
    with pytest.raises(TdwpError):
        plan.lowest_state(guess, n_iter=1)                   # fewer than two steps
    with pytest.raises(TdwpError):
        plan.lowest_state(np.zeros_like(guess), n_iter=10)   # zero start vector
    problem.install_packets(plan, spec)
    with pytest.raises(TdwpError):
        plan.lowest_state(guess, n_iter=10)                  # a packet is installed
    plan.close()
