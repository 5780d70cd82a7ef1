"""The network inference entry point that allocates nothing
(tdwp_mlp_eval_noalloc) against the allocating one (tdwp_mlp_eval), through
the C ABI: two calls in a row, the second smaller, each compared with the
allocating call on the same points; an input beyond the fixed scratch is
refused before any device work."""
import numpy as np
import pytest

from workloads import small_variant
from workloads import pes as PES
from workloads.mlp_inputs import init_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _distances(spec, n, seed):
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.5, 8.0, n)
    R = rng.uniform(0.5, 12.0, n)
    x = rng.uniform(-1.0, 1.0, n)
    rab, rbc, rac = PES.atom_distances(r, R, x, spec["mass_A"], spec["mass_B"], spec["mass_C"])
    return np.stack([rab, rbc, rac], axis=1)


def test_noalloc_inference_equals_allocating_inference():
    from paper_2412_10167_amd import problem
    from paper_2412_10167_amd.tdwp import TdwpError
    print("\n[case] mlp_eval_noalloc vs mlp_eval: 3000 then 700 points, 3 states", flush=True)
    spec = small_variant(5, n_R=24, n_r=20, n_gamma=12)
    plan, _ = problem.build(spec, mlp=dict(sample_idx=np.arange(64), init_params=init_params(6),
                                            order=np.arange(64), batch=64, epochs=0, lr=1e-3))
    try:
        for n, seed in ((3000, 11), (700, 12)):
            d = _distances(spec, n, seed)
            ref = plan.mlp_eval(d)
            got = plan.mlp_eval_noalloc(d)
            print(f"[result] {n} points: max |diff| {np.max(np.abs(got - ref)):.3e}", flush=True)
            assert got.shape == ref.shape == (n, 6)
            assert np.array_equal(got, ref)
        # n_pts (3 + n_pair) above 2^19 doubles: refused on the host
        big = np.ones(((1 << 19) // 9 + 1, 3))
        with pytest.raises(TdwpError) as e:
            plan.mlp_eval_noalloc(big)
        assert e.value.code == -6
        # the plan is still usable afterwards
        d = _distances(spec, 50, 13)
        assert np.array_equal(plan.mlp_eval_noalloc(d), plan.mlp_eval(d))
    finally:
        plan.close()
