"""Seeded random inputs of the learned-potential training: which grid points are
sampled, the initial network parameters and the minibatch order.  Random numbers
only; the network's arithmetic lives with each implementation."""
import numpy as np

HIDDEN = 128


def n_params(n_pair):
    return 3 * HIDDEN + HIDDEN + 2 * (HIDDEN * HIDDEN + HIDDEN) + HIDDEN * n_pair + n_pair


def sample_indices(n_points, n_samples=200000, seed=12345):
    """Flat grid indices drawn uniformly without replacement."""
    rng = np.random.default_rng(seed)
    n = min(n_samples, n_points)
    return np.sort(rng.choice(n_points, size=n, replace=False)).astype(np.int64)


def init_params(n_pair, seed=2024):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases, layout
    W1[3][128] b1 W2[128][128] b2 W3[128][128] b3 W4[128][n_pair] b4."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((3, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, n_pair)):
        lim = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-lim, lim, size=fan_in * fan_out))
        parts.append(rng.uniform(-lim, lim, size=fan_out))
    return np.concatenate(parts).astype(np.float32)


def batch_order(n_samples, seed=7):
    return np.random.default_rng(seed).permutation(n_samples).astype(np.int32)
