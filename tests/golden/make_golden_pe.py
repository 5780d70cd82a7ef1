"""Writes the oracle's state-to-state probabilities of full-length workload runs
to tests/golden/ (one JSON file per packet).

Only oracle/ and workloads/ are used: the stored values are the FP64 oracle's
(Eq. wvp-k propagated for the workload's step count, then Eqs. total-flux and
S-matrix-from-chebyshev on its collision-energy grid).  The GPU tests read the
files and compare the library's probabilities with them.

Each file records the workload, the unit and slot, the step count, a hash of
the workload definition, the commit of the oracle source, the spectral bounds
(taken from the whole workload, as a batched plan computes them), the channel
list with energies, the reactive probability per diabatic state, the inelastic
probabilities per channel and the norm trace every 50 steps.

    python tests/golden/make_golden_pe.py WORKLOAD UNIT SLOT [--steps K]
        [--jmax 10] [--vmax 2]

Runs take hours for the full-size workloads (one packet per process).
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import tdwp_oracle as O  # noqa: E402
from workloads import asymptotic_potential, config  # noqa: E402

NORM_STRIDE = 50


def spec_hash(spec):
    """sha256/16 of a canonical text of the workload definition (tuple keys as text)."""
    def canon(x):
        if isinstance(x, dict):
            return {str(k): canon(v) for k, v in sorted(x.items(), key=lambda kv: str(kv[0]))}
        if isinstance(x, (list, tuple)):
            return [canon(v) for v in x]
        if isinstance(x, float):
            return repr(x)
        return x
    return hashlib.sha256(json.dumps(canon(spec), sort_keys=True).encode()).hexdigest()[:16]


def oracle_commit():
    try:
        return subprocess.run(["git", "log", "-1", "--format=%H", "--", "oracle/tdwp_oracle.py"],
                              cwd=ROOT, capture_output=True, text=True, check=True).stdout.strip()
    except Exception:
        return "unknown"


def golden_name(wl, unit, slot, steps):
    return os.path.join(ROOT, "tests", "golden", f"pe_w{wl}_u{unit}_s{slot}_k{steps}.json")


def reactant_channels(op, spec, unit_index, jmax, vmax):
    """(elec, v, j, Omega) with Omega <= j over the unit's helicities, each with the
    oracle's channel function and energy."""
    oms = O.omega_range(spec["units"][unit_index])
    out = []
    for el in range(spec["n_elec"]):
        va = asymptotic_potential(spec, op.r, el)
        for j in range(jmax + 1):
            e, chi = O.diatomic_states(op, va, j, vmax + 1)
            for v in range(vmax + 1):
                for om in oms:
                    if om <= j:
                        out.append(dict(elec=el, v=v, j=j, omega=om, energy=float(e[v]), chi=chi[v]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", type=int)
    ap.add_argument("unit", type=int)
    ap.add_argument("slot", type=int)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--jmax", type=int, default=10)
    ap.add_argument("--vmax", type=int, default=2)
    a = ap.parse_args()
    spec = config(a.workload)
    K = a.steps or spec["steps"]
    full = O.Operator(spec)
    bounds = (full.Emin, full.Emax)
    del full
    sub = dict(spec)
    sub["units"] = [spec["units"][a.unit]]
    pk = [dict(p, unit=0) for p in spec["packets"] if p["unit"] == a.unit and p["slot"] == a.slot][0]
    sub["packets"] = [pk]
    op = O.Operator(sub, bounds=bounds)
    va = asymptotic_potential(sub, op.r, pk["elec0"])
    e, chi = O.diatomic_states(op, va, pk["j0"], pk["v0"] + 1)
    u0 = O.initial_packet(op, 0, pk, chi[pk["v0"]])
    t0 = time.time()
    print(f"workload {a.workload} unit {a.unit} slot {a.slot}: {K} steps, shape {u0.shape}", flush=True)
    run = O.propagate(op, 0, u0, K)
    t1 = time.time()
    chans = reactant_channels(op, sub, 0, a.jmax, a.vmax)
    res = O.analyse(op, 0, pk, run, e[pk["v0"]], chans)
    doc = dict(
        what="FP64 oracle state-to-state probabilities (reactive per diabatic state, "
             "reactant-arrangement inelastic per channel)",
        script="tests/golden/make_golden_pe.py",
        workload=a.workload, workload_name=spec["name"], unit=a.unit, slot=a.slot,
        J=spec["units"][a.unit]["J"], j0=pk["j0"], v0=pk["v0"], steps=K,
        spec_sha16=spec_hash(spec), oracle_commit=oracle_commit(),
        oracle_seconds=round(t1 - t0, 1),
        bounds=[repr(bounds[0]), repr(bounds[1])], E_v0j0=repr(float(e[pk["v0"]])),
        energies=[repr(float(x)) for x in res["energies"]],
        channels=[dict(elec=c["elec"], v=c["v"], j=c["j"], omega=c["omega"], energy=repr(c["energy"]))
                  for c in chans],
        p_reac=[[repr(float(x)) for x in row] for row in res["p_reac"]],
        p_inel=[[repr(float(x)) for x in row] for row in res["p_inel"]],
        norm_stride=NORM_STRIDE,
        norms=[repr(float(x)) for x in run["norms"][::NORM_STRIDE]],
    )
    path = golden_name(a.workload, a.unit, a.slot, K)
    with open(path + ".tmp", "w") as f:
        json.dump(doc, f, indent=0)
    os.replace(path + ".tmp", path)
    print(f"wrote {path} ({t1 - t0:.0f} s of propagation)", flush=True)


if __name__ == "__main__":
    main()
