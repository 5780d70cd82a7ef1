"""Parity of the library's photodissociation spectra (C ABI, host functions) with
the oracle (Eqs. chebyshev-transform and spectrum), on seeded autocorrelation
series; no GPU needed.

Both sides compute in FP64; the library forms cos(k theta) by a rotation
restarted from the library cosine every 256 terms, the oracle calls cos(k theta)
directly.  The bar is 1e-12 of the sum of the magnitudes of the terms at each
energy, sum_k (2 - delta_k0) |C_k| / (pi dE sin theta): the rounding scale of
the sum itself.
"""
import math

import numpy as np
import pytest

from oracle import photo_oracle as PH
from paper_2412_10167_amd import energy_content, photo_cross_section
from paper_2412_10167_amd.tdwp import TdwpError


def _scale(C, e_min, e_max, E):
    E0, dE = 0.5 * (e_max + e_min), 0.5 * (e_max - e_min)
    th = np.arccos((np.asarray(E) - E0) / dE)
    w = np.full(len(C), 2.0)
    w[0] = 1.0
    return float(np.sum(w * np.abs(C))) / (math.pi * dE * np.sin(th))


def _series(K, seed):
    # a decaying, oscillating series like a damped packet's overlaps
    rng = np.random.default_rng(seed)
    k = np.arange(K)
    return np.exp(-k / (0.3 * K + 1)) * np.cos(0.37 * k + rng.uniform(0, 6)) + 0.01 * rng.standard_normal(K)


@pytest.mark.parametrize("K, n_e, seed", [(1, 5, 1), (2, 7, 2), (255, 33, 3), (257, 40, 4),
                                          (4000, 200, 5), (20001, 64, 6)])
def test_energy_content_matches_oracle(K, n_e, seed):
    e_min, e_max = -0.35, 1.25
    C = _series(K, seed)
    rng = np.random.default_rng(seed + 100)
    E = np.sort(rng.uniform(e_min, e_max, n_e))
    E[0] = e_min + 1e-6 * (e_max - e_min)            # close to both ends of the range
    E[-1] = e_max - 1e-6 * (e_max - e_min)
    got = energy_content(C, e_min, e_max, E)
    ref = PH.energy_content(C, e_min, e_max, E)
    assert np.all(np.abs(got - ref) <= 1e-12 * _scale(C, e_min, e_max, E))


@pytest.mark.parametrize("K, seed", [(3, 11), (300, 12), (8000, 13)])
def test_photo_cross_section_matches_oracle(K, seed):
    e_min, e_max, E_i = -0.2, 0.9, -0.45
    C = _series(K, seed)
    hnu = np.linspace(0.3, 1.3, 77)
    got = photo_cross_section(C, e_min, e_max, E_i, hnu)
    ref = PH.cross_section(C, e_min, e_max, E_i, hnu)
    bound = 1e-12 * _scale(C, e_min, e_max, E_i + hnu) * PH.A_AU * hnu * math.pi
    assert np.all(np.abs(got - ref) <= bound)


def test_invalid_spectrum_arguments_are_rejected():
    C = np.ones(4)
    bad = [
        lambda: energy_content(C, 0.0, 1.0, [1.0]),            # on the upper bound
        lambda: energy_content(C, 0.0, 1.0, [-0.1]),           # below the range
        lambda: energy_content(C, 1.0, 1.0, [1.0]),            # empty range
        lambda: energy_content([], 0.0, 1.0, [0.5]),           # no components
        lambda: photo_cross_section(C, 0.0, 1.0, -0.5, [0.0]),  # h nu = 0
        lambda: photo_cross_section(C, 0.0, 1.0, -0.5, [2.0]),  # final energy above the range
    ]
    for k, call in enumerate(bad):
        with pytest.raises(TdwpError):
            call()
            pytest.fail(f"case {k} accepted")
