"""Parity of the library's partial-wave sums (C ABI, host functions) with the
oracle (Sec. "Cross sections": Eqs. collisional-xsection, cumulative-probability,
J-shifting-interpolation), on seeded threshold-shaped curves.

Both sides compute in FP64 and read curves by linear interpolation; they
differ only in the order of rounding, so the bar is 1e-12 relative to the
largest value (the sums of up to a few thousand terms of size <= 2J+1).
The fitted B is a minimiser found by different searches on both sides: the
bar there is that both reach the same minimum (B to 1e-7 B_max, misfit to
1e-12 relative).  These need the built library but no GPU.
"""
import numpy as np
import pytest

from oracle import xsection_oracle as X
from paper_2412_10167_amd import (cross_section, cumulative_probability, fit_jshift_b, jshift,
                                  jshift_interpolate)
from paper_2412_10167_amd.tdwp import TdwpError
from workloads import amu, ev
from workloads.partial_waves import batch_shape, energy_grid, families, probability_curves

B_FIG = ev(1.7e-3)


def close(got, ref, rel=1e-12):
    scale = max(1.0, float(np.max(np.abs(ref))))
    np.testing.assert_allclose(got, ref, rtol=0, atol=rel * scale)


@pytest.mark.parametrize("n_e, seed", [(1, 1), (2, 2), (33, 3), (200, 4)])
def test_jshift_matches_oracle(n_e, seed):
    rng = np.random.default_rng(seed)
    e = energy_grid(n_e, ev(0.2), ev(1.5), seed=seed)
    p = rng.uniform(size=n_e)
    for J_ref, J, B in ((0, 0, B_FIG), (0, 7, B_FIG), (12, 3, 2 * B_FIG), (5, 60, B_FIG),
                        (3, 9, 0.0)):
        close(jshift(p, e, J_ref, B, J), X.jshift(p, e, J_ref, B, J))


@pytest.mark.parametrize("n_e, seed", [(1, 5), (17, 6), (200, 7)])
def test_jshift_interpolate_matches_oracle(n_e, seed):
    rng = np.random.default_rng(seed)
    e = energy_grid(n_e, ev(0.2), ev(1.5), seed=seed)
    p1, p2 = rng.uniform(size=n_e), rng.uniform(size=n_e)
    for J in range(6, 15):
        close(jshift_interpolate(p1, p2, e, 6, 14, 3 * B_FIG, J),
              X.jshift_interpolate(p1, p2, e, 6, 14, 3 * B_FIG, J))
    np.testing.assert_array_equal(jshift_interpolate(p1, p2, e, 6, 14, B_FIG, 6), p1)
    np.testing.assert_array_equal(jshift_interpolate(p1, p2, e, 6, 14, B_FIG, 14), p2)


CASES = [
    # J_calc, J_max, j0 (families), n_f, n_e, seed
    ([0, 2, 4, 6], 6, 0, 1, 9, 10),              # even J computed, one family
    ([0, 3, 7, 12], 15, 2, 5, 33, 11),           # beyond the last computed J
    ([2, 5, 9], 11, 1, 3, 1, 12),                # below the first, one energy
    ([0, 1, 2, 3, 4, 5], 5, 3, 2, 17, 13),       # every J computed
    ([4], 9, 0, 2, 25, 14),                      # plain J-shifting from one J
    ([0, 10, 20], 20, 2, 7, 65, 15),             # wide intervals, ragged sizes
]


@pytest.mark.parametrize("J_calc, J_max, j0, n_f, n_e, seed", CASES)
def test_cumulative_probability_matches_oracle(J_calc, J_max, j0, n_f, n_e, seed):
    rng = np.random.default_rng(seed)
    e = energy_grid(n_e, ev(0.2), ev(1.5), seed=seed)
    fams, jmin = families(j0)
    p = probability_curves(len(J_calc), len(fams), n_f, e, seed, fam_jmin=jmin, J_calc=J_calc)
    B = rng.uniform(0.5, 4.0, len(J_calc)) * B_FIG
    got = cumulative_probability(J_calc, B, p, e, J_max, fam_jmin=jmin)
    close(got, X.cumulative_probability(J_calc, B, p, e, J_max, fam_jmin=jmin))
    # without family limits every family counts from J = 0
    close(cumulative_probability(J_calc, B, p, e, J_max),
          X.cumulative_probability(J_calc, B, p, e, J_max))


def test_cumulative_probability_batch_size_matches_oracle():
    # the batched workload's shape: J = 0, 2, ..., 40 computed, families of j0 = 2,
    # 64 final states, its 200-point collision-energy grid
    s = batch_shape()
    J_calc, e = s["J_calc"], s["energies"]
    p = probability_curves(len(J_calc), s["n_fam"], s["n_f"], e, 99, fam_jmin=s["fam_jmin"],
                           J_calc=J_calc)
    B = np.full(len(J_calc), B_FIG)
    got = cumulative_probability(J_calc, B, p, e, s["J_max"], fam_jmin=s["fam_jmin"])
    close(got, X.cumulative_probability(J_calc, B, p, e, s["J_max"], fam_jmin=s["fam_jmin"]))


def test_cross_section_matches_oracle():
    rng = np.random.default_rng(20)
    e = energy_grid(41, ev(0.2), ev(1.5), seed=21)
    C = rng.uniform(0.0, 500.0, (6, 41))
    mu = amu(1.008) * amu(3.022) / amu(4.030)
    for j0 in (0, 1, 4):
        close(cross_section(C, e, mu, j0), X.cross_section(C, e, mu, j0))


@pytest.mark.parametrize("seed", range(6))
def test_fit_jshift_b_matches_oracle(seed):
    e = energy_grid(120, ev(0.2), ev(1.5), seed=seed)
    p = probability_curves(2, 1, 1, e, seed=100 + seed)
    p1, p2 = p[0, 0, 0], p[1, 0, 0]
    J1, J2, B_max = 2 * seed, 2 * seed + 2, 20 * B_FIG
    got = fit_jshift_b(p1, p2, e, J1, J2, B_max)
    ref = X.fit_jshift_b(p1, p2, e, J1, J2, B_max)
    m_got = X.jshift_misfit(p1, p2, e, J1, J2, got)
    m_ref = X.jshift_misfit(p1, p2, e, J1, J2, ref)
    assert m_got <= m_ref * (1 + 1e-12) + 1e-300
    assert abs(got - ref) <= 1e-7 * B_max


def test_invalid_arguments_are_rejected():
    e = np.linspace(0.0, 1.0, 5)
    p = np.zeros(5)
    bad = [
        lambda: jshift(p, e[::-1], 0, B_FIG, 2),                         # grid not ascending
        lambda: jshift(p, e, 0, -B_FIG, 2),                              # negative B
        lambda: jshift(p, e, -1, B_FIG, 2),                              # negative J
        lambda: jshift_interpolate(p, p, e, 3, 3, B_FIG, 3),             # J2 == J1
        lambda: jshift_interpolate(p, p, e, 3, 6, B_FIG, 7),             # J outside [J1, J2]
        lambda: cumulative_probability([0, 0], [0, 0], np.zeros((2, 1, 1, 5)), e, 3),
        lambda: cumulative_probability([0, 2], [0, -1.0], np.zeros((2, 1, 1, 5)), e, 3),
        lambda: cumulative_probability([0, 2], [0, 0], np.zeros((2, 1, 1, 5)), e, -1),
        lambda: cumulative_probability([0, 2], [0, 0], np.zeros((2, 1, 1, 5)), e, 3,
                                       fam_jmin=[-1]),
        lambda: cross_section(np.ones((1, 5)), e, 1.0, 0),               # E = 0
        lambda: cross_section(np.ones((1, 5)), e + 1, 0.0, 0),           # mu = 0
        lambda: cross_section(np.ones((1, 5)), e + 1, 1.0, -1),          # j0 < 0
        lambda: fit_jshift_b(p, p, e, 2, 2, B_FIG),                      # J2 == J1
        lambda: fit_jshift_b(p, p, e, 0, 2, 0.0),                        # B_max = 0
    ]
    for k, call in enumerate(bad):
        with pytest.raises(TdwpError):
            call()
            pytest.fail(f"case {k} accepted")


def test_bench_partial_waves_line():
    # the host leg of bench.py runs without a GPU and prints one JSON line
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--partial-waves",
                          "--no-cpu-baseline", "--pw-final-states", "8"],
                         capture_output=True, text=True, timeout=300, check=True).stdout
    line = json.loads([ln for ln in out.splitlines() if ln.startswith("{")][-1])
    assert line["unit"] == "terms/s" and line["value"] > 0 and line["dtype"] == "f64"
    assert line["config"]["terms"] == 41 * 200 * 8 * 5 - 200 * 8 * (1 + 1 + 2 + 2)
