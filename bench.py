"""Throughput of the Chebyshev wave-packet hot path on one MI355X.

Default workload: the batched one, 21 partial waves J = 0, 2, ..., 40 (helicities
Omega <= min(J, 6): 135 helicity blocks) x 3 initial states BC(v=0, j=0,1,2) of
A + BC (masses 1.008/2.014/1.008 amu) on the synthetic LEPS surface, grid
R x r x gamma = 128 x 128 x 48 (318,504,960 values per step), in the
mixed-precision form chosen by the library's autotuner, with the plain FP64 form
timed beside it.  A step is one full Chebyshev iteration of every packet:
angular + Coriolis, both radial kinetic terms, potential, scaling/recursion/
damping, norm, flux and analysis lines, and the Chebyshev-to-energy
accumulation.  The accumulation runs once per ring of buffered steps; its
HIP-event time for one flush, divided by the ring length, is added to the
timed per-step time.  Inputs are resident in HBM before the timed region; the
timed region is K steps bracketed by device synchronisation and HIP events on
the library's stream.

Prints one JSON line.  Also reports the dominant kernel against the HBM
roofline (algorithmic bytes: read u_k and u_{k-1}, write u_{k+1}, 24 bytes per
value, plus the potential once per grid point), the whole step against the
same bytes, the largest P(E) difference of the timed form from the FP64 form
after the workload's full step count (per partial wave), and the FP64 oracle
timed on a bounded sample of the same workload on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD_NAMES = {
    2: "J=0 A+BC LEPS, R x r x gamma = 256x192x80, 1 state, 1 packet",
    3: "J=20 Omega 0..8, 2 coupled states, 192x160x64",
    4: "21 partial waves J=0..40 (Omega<=6) x 3 packets, 128x128x48",
    5: "J=4 Omega 0..4, 3 coupled states, 256x256x96 (tabulated V)",
}
METRIC = "Chebyshev steps/s (grid-pt·steps/s) mixed vs FP64 at ≤1e-3 |ΔP(E)|"
PEAKS = {  # MI355X published dense peaks
    "hbm": (8000.0, "GB/s"),
    "fp64": (78.6, "TFLOP/s"),
    "fp32": (157.3, "TFLOP/s"),
    "bf16": (2500.0, "TFLOP/s"),
}


def kernel_model(spec, name, precision, fused=False, photo=False):
    """Algorithmic work of one launch of kernel `name` on this single-unit workload:
    (bound, amount, unit, peak).  Flops count the executed multiply-adds of the
    even/odd-split contractions (2 per MAC); bytes count each HBM array the
    kernel must touch once (packet FP64, H-partials FP64 or FP32, potential FP64).
    fused: the r pass shares the angular launch and writes T_r u to a buffer of
    its own, which the R pass reads.  photo: the R pass also reads u_0 to form the
    photodissociation overlaps."""
    nr, nR, ng, ne = spec["n_r"], spec["n_R"], spec["n_gamma"], spec["n_elec"]
    n_blk = sum((u["omega_max"] - (0 if u["parity"] * (-1) ** u["J"] == 1 else 1) + 1) * u["n_packets"]
                for u in spec["units"])
    values = n_blk * ne * ng * nR * nr
    hb = 8 if precision == "fp64" else 4
    fp64 = precision == "fp64"
    if name == "radial_R_epilogue":
        # T_R split: nR flops per value; bytes: u_k, h, u_{k-1}, V (in h's
        # precision, shared by the helicity blocks of a point), u_{k+1}
        flops, byts = values * nR, values * (8 + hb + 8 + hb * ne * (ne + 1) / 2 / (n_blk * ne) + 8)
        if fused:
            byts += values * hb
        if photo:
            byts += values * 8
    elif name == "radial_rR_epilogue":
        # both radial terms over whole planes (one state): T_R and T_r full-size,
        # nR + nr flops per value; bytes: u_k, h, u_{k-1}, u_{k+1}, and V (FP32)
        # once per grid point
        flops, byts = values * (nR + nr), values * (8 + hb + 8 + 8) + hb * nR * nr * ng
    elif name == "radial_r" and not fused:
        # T_r split: nr flops per value; bytes: u_k, h read and written
        flops, byts = values * nr, values * (8 + 2 * hb)
    elif name == "autocorrelation":
        # <u_0|u_k> of the photodissociation packets: u_0 and u_k read once
        flops, byts = values * 2, values * 16
    elif name == "angular":
        # forward by absolute j (2 ng flops per value), back by parity class (ng);
        # bytes: u_k, h written
        flops, byts = values * 3 * ng, values * (8 + hb)
        if fused:   # plus the r pass: u_k read again, T_r u written
            flops, byts = flops + values * nr, byts + values * (8 + hb)
    else:
        return None
    if fp64 and flops / byts > PEAKS["fp64"][0] * 1e3 / PEAKS["hbm"][0]:
        return "mfma", flops / 1e12, "TFLOP/s", PEAKS["fp64"][0], byts
    return "hbm", byts / 1e9, "GB/s", PEAKS["hbm"][0], byts


KERNEL_SOURCES = ("paper_2412_10167_amd/csrc/fast_kernels.hpp", "paper_2412_10167_amd/csrc/mfma.hpp",
                  "paper_2412_10167_amd/csrc/plane_kernels.hpp",
                  "paper_2412_10167_amd/csrc/angw_kernels.hpp",
                  "paper_2412_10167_amd/csrc/step_kernels.hpp", "paper_2412_10167_amd/csrc/tdwp.hip")


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, precision):
    """HBM bytes per launch of `kernel` from the committed PMC summary of this
    workload and precision (FETCH_SIZE and WRITE_SIZE scaled by a device copy of
    known size), or None when there is none or the kernel sources have changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"step_kernels_w{workload}_{precision}_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    digest, table = None, {}
    for line in open(path):
        if line.startswith("kernel sources sha256/16:"):
            digest = line.split(":", 1)[1].strip()
        elif line.startswith("traffic_bytes "):
            _, name, val = line.split()
            table[name] = float(val)
    if digest != kernel_source_digest():
        return None
    return table.get(kernel)


def pe_difference(problem, spec, precision, steps, autotune, jmax=10, vmax=2):
    """Largest |P(E)| difference between the timed form and the FP64 form after the
    same number of steps, each built as it is timed (the autotuner's variant):
    reactive probability per state and every reactant-channel probability
    (v <= vmax, j <= jmax, all helicities) of every packet, on all collision
    energies; also the largest difference per partial wave J."""
    import numpy as np
    res, per_pk, chosen = {}, {}, {}
    for prec in (precision, "fp64"):
        plan, info = problem.build(spec, precision=prec, autotune=autotune)
        chosen[prec] = (info.get("autotune") or "").split("chosen=")[-1] or None
        plan.propagate(steps, norms=False)
        parts = []
        for pk in spec["packets"]:
            chans = problem.channels(plan, spec, pk["unit"], min(jmax, spec["n_gamma"] - 1), vmax)
            p_inel, p_reac = plan.state_to_state(pk["unit"], pk["slot"], chans)
            v = np.concatenate([p_inel.ravel(), p_reac.ravel()])
            per_pk.setdefault(prec, []).append(v)
            parts.append(v)
        res[prec] = np.concatenate(parts)
        plan.close()
        print(f"pe_vs_fp64: {prec} propagated {steps} steps", file=sys.stderr, flush=True)
    d = np.abs(res[precision] - res["fp64"])
    by_J = {}
    for i, pk in enumerate(spec["packets"]):
        J = spec["units"][pk["unit"]]["J"]
        dj = float(np.max(np.abs(per_pk[precision][i] - per_pk["fp64"][i])))
        by_J[J] = max(by_J.get(J, 0.0), dj)
    return dict(steps=steps, probabilities=int(d.size), max_abs_diff=float(d.max()),
                max_probability=float(np.max(np.abs(res["fp64"]))),
                variants=chosen,
                max_abs_diff_by_J={str(k): float("%.3g" % v) for k, v in sorted(by_J.items())})


def mlp_bench(args, torch, problem, config):
    """Learned potential: device training from the tabulated surface (timed apart),
    grid error of the network, and the step with the network evaluated on the fly
    against the tabulated step of the same plan shape.  Prints one JSON line."""
    import numpy as np
    from workloads.mlp_inputs import batch_order, init_params, sample_indices
    spec = config(args.workload)
    torch.cuda.set_device(0)
    torch.cuda.set_stream(torch.cuda.Stream())
    stream = torch.cuda.current_stream()
    plan_t, _ = problem.build(spec, precision=args.precision, autotune=args.autotune)
    vtab = problem.potential_table(plan_t, spec)
    n_pair = vtab.shape[0]
    n_pts = vtab[0].size
    idx = sample_indices(n_pts, n_samples=args.mlp_samples)
    mlp = dict(sample_idx=idx, init_params=init_params(n_pair), order=batch_order(idx.size),
               batch=args.mlp_batch, epochs=args.mlp_epochs, lr=args.mlp_lr,
               lr_final=args.mlp_lr_final)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan_m, info = problem.build(spec, precision=args.precision, vtable=vtab, mlp=mlp,
                                 autotune=args.autotune)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    loss, rms, mx = info["mlp_report"]
    print(f"trained in {train_s:.1f} s: grid rms {rms * 27211.386:.2f} meV", file=sys.stderr, flush=True)

    def rate(plan):
        plan.propagate(args.warmup, norms=False)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.propagate(args.steps, norms=False)
        e1.record(stream)
        torch.cuda.synchronize()
        return args.steps / (e0.elapsed_time(e1) / 1e3)

    r_table, r_mlp = rate(plan_t), rate(plan_m)
    kt = plan_m.time_kernels(args.kernel_steps)
    pe = None
    if args.mlp_pe_steps > 0:
        res = {}
        for key, plan in (("table", plan_t), ("mlp", plan_m)):
            problem.install_packets(plan, spec)
            plan.propagate(args.mlp_pe_steps, norms=False)
            print(f"{key}: {args.mlp_pe_steps} steps propagated", file=sys.stderr, flush=True)
            parts = []
            for pk in spec["packets"]:
                chans = problem.channels(plan, spec, pk["unit"], min(10, spec["n_gamma"] - 1), 2)
                p_inel, p_reac = plan.state_to_state(pk["unit"], pk["slot"], chans)
                parts += [p_inel.ravel(), p_reac.ravel()]
            res[key] = np.concatenate(parts)
        d = np.abs(res["mlp"] - res["table"])
        pe = dict(steps=args.mlp_pe_steps, probabilities=int(d.size), max_abs_diff=float(d.max()),
                  mean_abs_diff=float(d.mean()), max_probability=float(np.max(np.abs(res["table"]))))
    plan_t.close()
    plan_m.close()
    eh_mev = 27211.386245988
    values = n_pts * sum((u["omega_max"] - (0 if u["parity"] * (-1) ** u["J"] == 1 else 1) + 1)
                         * u["n_packets"] for u in spec["units"]) * spec["n_elec"]
    out = {
        "metric": "Chebyshev steps/s with the learned potential evaluated on the fly",
        "value": round(r_mlp, 2), "unit": "Chebyshev steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16x3": "bf16x3+f64",
                  "fp16x3": "f16x3+f64"}[args.precision] + ", network bf16/f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_NAMES.get(wl, spec["name"]), "grid_values": values,
                   "table_steps_per_s": round(r_table, 2),
                   "table_bytes_per_step": int(vtab.size * (8 if args.precision == "fp64" else 4)),   # the R pass reads the table at h's width
                   "network_flops_per_step": int(n_pts * 2 * (3 * 128 + 2 * 128 * 128 + 128 * n_pair)),
                   "training": {"samples": int(idx.size), "epochs": args.mlp_epochs,
                                "batch": args.mlp_batch, "lr": args.mlp_lr,
                                "lr_final": args.mlp_lr_final,
                                "seconds": round(train_s, 2), "final_loss": loss,
                                "grid_rms_meV": round(rms * eh_mev, 3),
                                "grid_max_meV": round(mx * eh_mev, 3)},
                   "pe_network_vs_table": pe,
                   "kernels_avg_us": {k: round(v, 2) for k, v in kt.items()}},
    }
    print(json.dumps(out))


def n_blocks(spec):
    """Helicity blocks x packets of a workload (the units of work of one step)."""
    return sum((u["omega_max"] - (0 if u["parity"] * (-1) ** u["J"] == 1 else 1) + 1) * u["n_packets"]
               for u in spec["units"])


def cpu_baseline(spec, min_steps=100, budget_s=20.0):
    """The oracle, untuned, on a bounded sample: one packet of the workload's unit
    with the most helicity blocks, at least min_steps full-size Chebyshev steps
    (more while within budget_s) after one warm-up step.  The rate is scaled to
    steps/s of the whole workload by the blocks the sample holds against the
    workload's total (the oracle's cost per block and step is nearly uniform)."""
    import numpy as np
    from oracle import tdwp_oracle as O
    from workloads import asymptotic_potential
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max([i.get("num_threads", 1) for i in info] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    ui = max(range(len(spec["units"])), key=lambda i: (spec["units"][i]["omega_max"], spec["units"][i]["J"]))
    sub = dict(spec)
    sub["units"] = [dict(spec["units"][ui], n_packets=1)]
    pk = [dict(p, unit=0) for p in spec["packets"] if p["unit"] == ui][0]
    sub["packets"] = [pk]
    op = O.Operator(sub)
    va = asymptotic_potential(sub, op.r, pk["elec0"])
    e0, chi0 = O.diatomic_states(op, va, pk["j0"], pk["v0"] + 1)
    u0 = O.initial_packet(op, 0, pk, chi0[pk["v0"]])
    u_prev, u = u0, op.D * O.apply_Hs(op, 0, u0)
    t0 = time.perf_counter()
    n = 0
    while n < min_steps or time.perf_counter() - t0 < budget_s:
        u_prev, u = u, op.D * (2.0 * O.apply_Hs(op, 0, u) - op.D * u_prev)
        n += 1
    dt = time.perf_counter() - t0
    assert np.isfinite(np.sum(u * u))
    blk = n_blocks(sub)
    total = n_blocks(spec)
    U = spec["units"][ui]
    return dict(value=n * blk / dt / total, unit="Chebyshev steps/s", cores=cores, kind="oracle",
                sample=f"{n} full-size steps of one packet of the J={U['J']} unit ({blk} helicity "
                       f"blocks of {spec['n_R']}x{spec['n_r']}x{spec['n_gamma']}) of the FP64 numpy "
                       f"oracle (H application, recursion and damping; no slices) in {dt:.1f} s = "
                       f"{n * blk / dt:.3f} block-steps/s, scaled to the workload's {total} blocks")


def spectrum_timing(plan, skip_oracle, E_i):
    """Energy content a_0(E) and cross section sigma(h nu) (host functions of the
    library) from the packet's whole autocorrelation series on 2,000 energies, with
    the oracle's time beside them."""
    import numpy as np
    from paper_2412_10167_amd import energy_content, photo_cross_section
    C = plan.autocorrelation(0, 0)
    lo, hi = plan.spectral_bounds()
    E = np.linspace(lo, hi, 2002)[1:-1]
    hnu = E[E > E_i] - E_i
    t0 = time.perf_counter()
    a0 = energy_content(C, lo, hi, E)
    sigma = photo_cross_section(C, lo, hi, E_i, hnu) if hnu.size else np.zeros(0)
    t_lib = time.perf_counter() - t0
    out = dict(components=int(C.size), energies=int(E.size), library_ms=round(t_lib * 1e3, 3))
    if sigma.size:
        k = int(np.argmax(sigma))
        out.update(sigma_peak_bohr2=float(sigma[k]),
                   sigma_peak_hnu_eV=float(hnu[k] * 27.211386245988))
    if not skip_oracle:
        from oracle import photo_oracle as PH
        t0 = time.perf_counter()
        ref = PH.energy_content(C, lo, hi, E)
        out["oracle_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
        out["max_rel_diff"] = float(np.max(np.abs(a0 - ref)) / np.max(np.abs(ref)))
    return out


def partial_waves_bench(args):
    """Partial-wave sums on the batched workload's output shape (host functions of
    the library): a fitted B per computed J, the cumulative probability over
    J = 0..40 from the 21 computed J, and the cross section.  The probabilities
    are seeded synthetic curves of that shape; the oracle runs the same sums."""
    import numpy as np
    from paper_2412_10167_amd import cross_section, cumulative_probability, fit_jshift_b
    from workloads import ev
    from workloads.partial_waves import batch_shape, probability_curves

    s = batch_shape(n_f=args.pw_final_states)
    J, e, jmin = s["J_calc"], s["energies"], s["fam_jmin"]
    p = probability_curves(len(J), s["n_fam"], s["n_f"], e, 2024, fam_jmin=jmin, J_calc=J)
    mA, mB, mC = s["masses"]
    mu = mA * (mB + mC) / (mA + mB + mC)
    B_max = ev(5e-3)
    fam_total = p[:, 0].sum(axis=1)            # Omega0 = 0 family, summed over final states

    def fits():
        B = [fit_jshift_b(fam_total[c], fam_total[c + 1], e, J[c], J[c + 1], B_max)
             for c in range(len(J) - 1)]
        return np.array(B + [B[-1]])

    def sums(B):
        C = cumulative_probability(J, B, p, e, s["J_max"], fam_jmin=jmin)
        return cross_section(C, e, mu, 2)

    def rate(fn, budget):
        fn()
        t0, n = time.perf_counter(), 0
        while time.perf_counter() - t0 < budget:
            out = fn()
            n += 1
        return (time.perf_counter() - t0) / n, out

    t_fit, B = rate(fits, 1.0)
    t_sum, sigma = rate(lambda: sums(B), 2.0)
    terms = sum(1 for Jv in range(s["J_max"] + 1) for jm in jmin if Jv >= jm) * s["n_f"] * e.size
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import xsection_oracle as X
        t_or, ref = rate(lambda: X.cross_section(
            X.cumulative_probability(J, B, p, e, s["J_max"], fam_jmin=jmin), e, mu, 2), 10.0)
        err = float(np.max(np.abs(sigma - ref)) / np.max(np.abs(ref)))
        cpu = dict(value=round(terms / t_or, 1), unit="terms/s", cores=1, kind="oracle",
                   sample=f"the same sums (numpy oracle) repeated for about 10 s; "
                          f"max relative difference of sigma {err:.1e}")
    out = {
        "metric": "partial-wave sum terms/s (Eq. cumulative-probability + cross section)",
        "value": round(terms / t_sum, 1),
        "unit": "terms/s",
        "n_gpus": 0,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": round(t_sum * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"J=0..40 from 21 computed J, {s['n_fam']} (Omega0, p) families "
                               f"(j0=2), {s['n_f']} final states, {e.size} energies",
                   "terms": terms, "fit_ms_per_interval": round(t_fit * 1e3 / (len(J) - 1), 4),
                   "host_threads": min(16, os.cpu_count() or 1, max(1, s["n_f"] // 16))},
        "roofline": None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="fp16x3",
                    help="contraction precision of the timed form: fp64, fp32, bf16x3, fp16x3")
    ap.add_argument("--no-fp64-reference", action="store_true",
                    help="skip timing the plain FP64 form beside a mixed form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-steps", type=int, default=None,
                    help="steps of the per-kernel HIP-event timing (default: past two ring "
                         "flushes, so the energy accumulation is timed)")
    ap.add_argument("--autotune", type=int, default=5,
                    help="steps per tile variant timed by the library's autotuner (0: off)")
    ap.add_argument("--workload", type=int, default=None,
                    help="workload number 1..5 (default 4: 21 partial waves x 3 packets, "
                         "128x128x48; 2 with --photo, 5 with --mlp)")
    ap.add_argument("--no-side-workload", action="store_true",
                    help="skip timing workload 2 (J=0 256x192x80) beside the batched workload")
    ap.add_argument("--radial-grid", type=int, default=0,
                    help="workgroups of the radial passes (0: one per block)")
    ap.add_argument("--pe-steps", type=int, default=None,
                    help="steps of the P(E) comparison of the timed form with the FP64 form "
                         "(default: the workload's full step count on workloads 2 and 4, else "
                         "0 = off)")
    ap.add_argument("--mlp", action="store_true",
                    help="learned-potential run: train the network on the device from the "
                         "tabulated surface, then time the step with the network evaluated on "
                         "the fly beside the tabulated step (default workload 5)")
    ap.add_argument("--mlp-samples", type=int, default=200000)
    ap.add_argument("--mlp-epochs", type=int, default=40)
    ap.add_argument("--mlp-batch", type=int, default=1024)
    ap.add_argument("--mlp-lr", type=float, default=2e-3)
    ap.add_argument("--mlp-lr-final", type=float, default=2e-5)
    ap.add_argument("--mlp-pe-steps", type=int, default=0,
                    help="also propagate both plans from k = 0 for this many steps and report "
                         "the largest P(E) difference between the network and the table")
    ap.add_argument("--photo", action="store_true",
                    help="propagate a photodissociation packet (synthetic dipole times bound "
                         "state) with its autocorrelation formed after every step")
    ap.add_argument("--lanczos-steps", type=int, default=300,
                    help="Lanczos steps of the bound state (--photo)")
    ap.add_argument("--partial-waves", action="store_true",
                    help="time the host partial-wave sums (J-shifting interpolation, cumulative "
                         "probability, cross section) on the batched workload's output shape")
    ap.add_argument("--pw-final-states", type=int, default=64)
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="also run one device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.workload is None:
        args.workload = 2 if args.photo else 5 if args.mlp else 4
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(independent partial waves would shard across GPUs with no per-step traffic)",
              file=sys.stderr)
        sys.exit(2)
    if args.partial_waves:
        return partial_waves_bench(args)

    import torch
    from paper_2412_10167_amd import problem
    from workloads import config

    if args.mlp:
        return mlp_bench(args, torch, problem, config)

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    # a dedicated (non-default, default-priority) stream: the library enqueues on it,
    # the timing events are recorded on it, and HIP graphs can be captured on it
    bench_stream = torch.cuda.Stream()
    torch.cuda.set_stream(bench_stream)
    tune_reports = {}
    spec = config(args.workload)
    values = sum(
        (u["omega_max"] - (0 if u["parity"] * (-1) ** u["J"] == 1 else 1) + 1) * u["n_packets"]
        for u in spec["units"]) * spec["n_elec"] * spec["n_R"] * spec["n_r"] * spec["n_gamma"]

    bound_cache = {}

    def build(precision):
        if not args.photo:
            return problem.build(spec, precision=precision, autotune=args.autotune)
        # photodissociation: the bound state of a ground-state well by the
        # library's Lanczos iteration (FP64, same grid), times the dipole; the
        # autocorrelation formed on the device after every step
        import numpy as np
        from paper_2412_10167_amd.tdwp import Plan
        from workloads.photo import bound_spec, dipole_times, ground_state_table
        if "bound" not in bound_cache:
            bspec = bound_spec(spec)
            bplan = Plan(bspec)
            r, R, x, _ = bplan.grid()
            bplan.set_potential(ground_state_table(bspec, r, R, x))
            g = np.exp(-((R[:, None] - 3.0) / 0.5) ** 2 - ((r[None, :] - 1.4) / 0.3) ** 2)
            g = np.broadcast_to(g, (len(x),) + g.shape).copy()
            t0 = time.perf_counter()
            E_i, psi, res = bplan.lowest_state(g, n_iter=args.lanczos_steps)
            t_lz = time.perf_counter() - t0
            bplan.close()
            bound_cache["bound"] = (E_i, psi, (r, R, x))
            bound_cache["info"] = dict(energy=E_i, residual=res, lanczos_steps=args.lanczos_steps,
                                       seconds=round(t_lz, 3))
        E_i, psi, (r, R, x) = bound_cache["bound"]
        plan = Plan(spec, precision=precision)
        plan.set_potential(problem.potential_table(plan, spec))
        info = {}
        if args.autotune:
            info["autotune"] = plan.autotune(args.autotune)
        plan.set_packet_values(0, 0, dipole_times(spec, 0, r, R, x, psi))
        return plan, info

    def timed(precision, steps, warmup, sp=None):
        if sp is None:
            plan, info = build(precision)
        else:
            plan, info = problem.build(sp, precision=precision, autotune=args.autotune)
        if args.radial_grid:
            plan.set_option("radial_grid", args.radial_grid)
        if info.get("autotune") and sp is None:
            tune_reports[precision] = info["autotune"]
        plan.propagate(warmup, norms=False)
        stream = torch.cuda.current_stream()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        plan.propagate(steps, norms=False)
        e1.record(stream)
        torch.cuda.synchronize()
        return plan, e0.elapsed_time(e1), time.perf_counter() - t0

    def per_step_kernels(plan):
        """Kernel averages (us per launch, HIP events on the library's stream) over
        enough steps to include two energy accumulations (ring flushes)."""
        ring = plan.stat("ring_len")
        n = args.kernel_steps or 2 * ring + 8
        kt = plan.time_kernels(n)
        fz = bool(plan.stat("fuse_r"))
        return {k: v for k, v in kt.items()
                if not (fz and k == "radial_r") and not (k == "autocorrelation" and v == 0.0)}, ring

    plan, ms, wall = timed(args.precision, args.steps, args.warmup)
    per_step, ring = per_step_kernels(plan)
    fused = bool(plan.stat("fuse_r"))
    # the energy accumulation runs once per ring of buffered steps: its time per
    # flush over the ring length is added to the timed steps
    acc_us = per_step.get("accumulate", 0.0)
    ms_step = ms / args.steps + acc_us * 1e-3 / ring
    steps_per_s = 1e3 / ms_step
    in_pass = args.photo and not per_step.get("autocorrelation")
    step_kernels = {k: v for k, v in per_step.items() if k not in ("accumulate", "slices")}
    dom = max((k for k in step_kernels if kernel_model(spec, k, args.precision, fused)),
              key=lambda k: step_kernels[k])
    traffic = measured_traffic(dom, args.workload, args.precision) if not args.photo else None
    _, _, _, _, own_bytes = kernel_model(spec, dom, args.precision, fused, in_pass)
    # algorithmic bytes of a step: u_k and u_{k-1} read, u_{k+1} written (FP64),
    # the potential once per grid point (8 bytes per stored entry)
    n_pair = spec["n_elec"] * (spec["n_elec"] + 1) // 2
    alg_bytes = 24.0 * values + 8.0 * n_pair * spec["n_R"] * spec["n_r"] * spec["n_gamma"]
    peak = PEAKS["hbm"][0]
    achieved = alg_bytes / 1e9 / (step_kernels[dom] * 1e-6)
    step_gbps = alg_bytes / 1e9 / (ms_step * 1e-3)
    roofline = dict(bound="hbm", achieved=round(achieved, 3), peak=peak, unit="GB/s",
                    frac=round(achieved / peak, 4), traffic=traffic, kernel=dom,
                    kernel_avg_us=round(step_kernels[dom], 2),
                    algorithmic_bytes_per_step=alg_bytes,
                    kernel_own_bytes=own_bytes,
                    kernel_own_frac=round(own_bytes / 1e9 / (step_kernels[dom] * 1e-6) / peak, 4),
                    step=dict(achieved=round(step_gbps, 3), frac=round(step_gbps / peak, 4),
                              ms=round(ms_step, 5)),
                    kernels_avg_us={k: round(v, 2) for k, v in per_step.items()},
                    ring_len=ring)
    acf = None
    if args.photo:
        if in_pass:   # formed by the R pass (u_0 read there, 8 bytes per value)
            acf = dict(formed_in="radial_R_epilogue")
        else:
            _, gb, _, pk_bw, _ = kernel_model(spec, "autocorrelation", args.precision, fused)
            a_bw = gb / (per_step["autocorrelation"] * 1e-6)
            acf = dict(formed_in="autocorrelation kernel",
                       kernel_avg_us=round(per_step["autocorrelation"], 2),
                       achieved_GBps=round(a_bw, 1), frac=round(a_bw / pk_bw, 4))
        acf["bound_state"] = bound_cache.get("info")
        acf["spectrum"] = spectrum_timing(plan, args.no_cpu_baseline, bound_cache["bound"][0])
    plan.close()
    print(f"timed {args.precision}: {steps_per_s:.2f} steps/s", file=sys.stderr, flush=True)
    fp64_rate = None
    if args.precision != "fp64" and not args.no_fp64_reference:
        p64, ms64, _ = timed("fp64", args.steps, args.warmup)
        k64, ring64 = per_step_kernels(p64)
        p64.close()
        fp64_rate = 1e3 / (ms64 / args.steps + k64.get("accumulate", 0.0) * 1e-3 / ring64)
        print(f"timed fp64: {fp64_rate:.2f} steps/s", file=sys.stderr, flush=True)
    side = None
    if args.workload != 2 and not args.no_side_workload and not args.photo:
        s2 = config(2)
        side = {"workload": WORKLOAD_NAMES[2]}
        for prec in ([args.precision, "fp64"] if args.precision != "fp64" else ["fp64"]):
            pp, m2, _ = timed(prec, 400, 20, sp=s2)
            k2, r2 = per_step_kernels(pp)
            pp.close()
            side[prec + "_steps_per_s"] = round(1e3 / (m2 / 400 + k2.get("accumulate", 0.0) * 1e-3 / r2), 2)
        if "fp64_steps_per_s" in side and args.precision != "fp64":
            side["speedup_vs_fp64"] = round(side[args.precision + "_steps_per_s"] / side["fp64_steps_per_s"], 3)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()

    pe_steps = args.pe_steps if args.pe_steps is not None else (
        spec["steps"] if args.workload in (2, 4) else 0)
    if args.photo:
        pe_steps = 0
    pe = None
    if pe_steps > 0 and args.precision != "fp64":
        pe = pe_difference(problem, spec, args.precision, pe_steps, args.autotune)

    cpu = None
    if not args.no_cpu_baseline and not args.photo:
        cpu = cpu_baseline(spec)

    out = {
        "metric": METRIC if not args.photo else
        "Chebyshev steps/s of a photodissociation packet with its per-step autocorrelation",
        "value": round(steps_per_s, 2),
        "unit": "Chebyshev steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16x3": "bf16x3+f64", "fp16x3": "f16x3+f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": WORKLOAD_NAMES.get(args.workload, spec["name"]),
                   "precision": args.precision, "grid_values": values,
                   "grid_pt_steps_per_s": round(steps_per_s * values, 1),
                   "timed_steps_ms": round(ms, 4),
                   "accumulate_in_step": f"one energy accumulation per {ring} steps: "
                                         f"{acc_us:.1f} us per flush, {acc_us / ring:.2f} us per step "
                                         "added to the timed steps",
                   "fp64_steps_per_s": round(fp64_rate, 2) if fp64_rate else None,
                   "speedup_vs_fp64": round(steps_per_s / fp64_rate, 3) if fp64_rate else None,
                   "autotune": tune_reports or None,
                   "fused_r": fused,
                   "autocorrelation": acf,
                   "pe_vs_fp64": pe,
                   "workload_2": side,
                   "wall_s": round(wall, 3)},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
