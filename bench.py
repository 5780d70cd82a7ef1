"""Throughput of the Chebyshev wave-packet hot path on one MI355X.

Workload: J = 0 A + BC (masses 1.008/2.014/1.008 amu) on the synthetic LEPS
surface, grid R x r x gamma = 256 x 192 x 80 (3,932,160 values), one diabatic
state, one packet.  A step is one full Chebyshev iteration: angular + potential,
both radial kinetic terms, scaling/recursion/damping, norm, flux and analysis
lines, and the (amortised) Chebyshev-to-energy accumulation.  Inputs are
resident in HBM before the timed region; the timed region is K calls' worth of
steps bracketed by device synchronisation and HIP events on the library's
stream.

Prints one JSON line.  Also reports the dominant kernel against its roofline
(per-kernel device time from HIP events inside the library) and the FP64 oracle
timed on a bounded sample of the same workload on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Chebyshev steps/s (grid-pt·steps/s) mixed vs FP64 at ≤1e-3 |ΔP(E)|"
PEAKS = {  # MI355X published dense peaks
    "hbm": (8000.0, "GB/s"),
    "fp64": (78.6, "TFLOP/s"),
    "fp32": (157.3, "TFLOP/s"),
    "bf16": (2500.0, "TFLOP/s"),
}


def kernel_model(spec, name, precision):
    """Algorithmic work of one launch of kernel `name` on the workload, as
    (bound, amount, unit, peak): flops for dense contractions, bytes for streams."""
    nr, nR, ng, ne = spec["n_r"], spec["n_R"], spec["n_gamma"], spec["n_elec"]
    n_om = sum(u["omega_max"] + 1 for u in spec["units"])   # parity-even units: 0..omega_max
    values = n_om * ne * ng * nR * nr
    if name == "radial_epi":
        flops = values * 2.0 * (nR + nr)
        return "alu", flops / 1e12, "TFLOP/s", PEAKS["fp64"][0]
    if name == "angular_pot":
        flops = values * 4.0 * ng
        return "alu", flops / 1e12, "TFLOP/s", PEAKS["fp64"][0]
    if name == "slices":
        return "hbm", values * 8.0 / 1e9, "GB/s", PEAKS["hbm"][0]
    return None


def cpu_baseline(spec, budget_s=15.0):
    """The oracle, untuned, on a bounded sample: as many full-size Chebyshev steps
    as fit in about budget_s seconds after one warm-up step."""
    import numpy as np
    from oracle import tdwp_oracle as O
    from workloads import asymptotic_potential
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max([i.get("num_threads", 1) for i in info] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    op = O.Operator(spec)
    va = asymptotic_potential(spec, op.r, 0)
    e0, chi0 = O.diatomic_states(op, va, 0, 1)
    u0 = O.initial_packet(op, 0, spec["packets"][0], chi0[0])
    u_prev, u = u0, op.D * O.apply_Hs(op, 0, u0)
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < budget_s:
        u_prev, u = u, op.D * (2.0 * O.apply_Hs(op, 0, u) - op.D * u_prev)
        n += 1
    dt = time.perf_counter() - t0
    assert np.isfinite(np.sum(u * u))
    return dict(value=n / dt, unit="Chebyshev steps/s", cores=cores, kind="oracle",
                sample=f"{n} full-size steps (256x192x80, J=0) of the FP64 numpy oracle "
                       f"(H application, recursion and damping; no slices) in {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-steps", type=int, default=50)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(independent partial waves would shard across GPUs with no per-step traffic)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2412_10167_amd import problem
    from workloads import config

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    spec = config(2)
    plan, _ = problem.build(spec, precision=args.precision)
    values = spec["n_R"] * spec["n_r"] * spec["n_gamma"]
    plan.propagate(args.warmup, norms=False)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    plan.propagate(args.steps, norms=False)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    steps_per_s = args.steps / (ms / 1e3)

    kt = plan.time_kernels(args.kernel_steps)
    per_step = {k: v for k, v in kt.items()}
    dom = max((k for k in per_step if kernel_model(spec, k, args.precision)), key=lambda k: per_step[k])
    bound, amount, unit, peak = kernel_model(spec, dom, args.precision)
    achieved = amount / (per_step[dom] * 1e-6)
    roofline = dict(bound=bound, achieved=round(achieved, 3), peak=peak, unit=unit,
                    frac=round(achieved / peak, 4), traffic=None, kernel=dom,
                    kernel_avg_us=round(per_step[dom], 2),
                    kernels_avg_us={k: round(v, 2) for k, v in per_step.items()})
    plan.close()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(spec)

    out = {
        "metric": METRIC,
        "value": round(steps_per_s, 2),
        "unit": "Chebyshev steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16x3": "bf16x3+f64", "fp16x3": "f16x3+f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "J=0 A+BC LEPS, R x r x gamma = 256x192x80, 1 state, 1 packet",
                   "precision": args.precision, "grid_values": values,
                   "grid_pt_steps_per_s": round(steps_per_s * values, 1),
                   "wall_s": round(wall, 3)},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
