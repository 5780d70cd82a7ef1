"""FP64 CPU oracle of the learned diabatic-potential surrogate (test infrastructure only).

The surrogate maps the three internuclear distances (r_AB, r_BC, r_AC) of a
grid point to the packed upper triangle of its diabatic potential matrix
(the quantity the tabulated potential of Sec. 2.1 item 5 holds, evaluated on
the fly instead of read):

    f = (d - FEAT_CENTER) / FEAT_SCALE                       (3 features)
    a1 = silu(f W1 + b1), a2 = silu(a1 W2 + b2), a3 = silu(a2 W3 + b3)
    V = OUT_SCALE * (a3 W4 + b4)                              (hartree)

silu(x) = x / (1 + e^-x).  Loss: mean over batch and outputs of
(y - V/OUT_SCALE)^2.  Plain FP64 forward and reverse-mode gradients, written
from the chain rule; pinned by finite differences in the tests.
"""
import numpy as np

FEAT_CENTER = 4.0
FEAT_SCALE = 3.0
OUT_SCALE = 0.1
HIDDEN = 128


def layer_shapes(n_out):
    return [(3, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, n_out)]


def n_params(n_out):
    return sum(a * b + b for a, b in layer_shapes(n_out))


def unpack(theta, n_out):
    """Flat parameters -> [(W, b)] in the order W1, b1, W2, b2, W3, b3, W4, b4 (W row-major [in][out])."""
    out, p = [], 0
    for a, b in layer_shapes(n_out):
        W = np.asarray(theta[p:p + a * b], float).reshape(a, b)
        p += a * b
        bias = np.asarray(theta[p:p + b], float)
        p += b
        out.append((W, bias))
    return out


def features(d):
    return (np.asarray(d, float) - FEAT_CENTER) / FEAT_SCALE


def silu(x):
    return x / (1.0 + np.exp(-x))


def dsilu(x):
    s = 1.0 / (1.0 + np.exp(-x))
    return s * (1.0 + x * (1.0 - s))


def forward(theta, d, n_out):
    """Returns (normalised outputs y [B][n_out], cache)."""
    layers = unpack(theta, n_out)
    a = features(d)
    cache = [a]
    zs = []
    for k, (W, b) in enumerate(layers):
        z = a @ W + b
        zs.append(z)
        a = silu(z) if k < len(layers) - 1 else z
        cache.append(a)
    return a, (cache, zs)


def potential(theta, d, n_out):
    """Surrogate potential entries (hartree)."""
    return OUT_SCALE * forward(theta, d, n_out)[0]


def loss_and_grad(theta, d, v_target, n_out):
    """Mean-squared error on normalised targets and its gradient w.r.t. the flat parameters."""
    y, (acts, zs) = forward(theta, d, n_out)
    t = np.asarray(v_target, float) / OUT_SCALE
    B = y.shape[0]
    diff = y - t
    loss = float(np.mean(diff * diff))
    layers = unpack(theta, n_out)
    g = 2.0 * diff / (B * n_out)          # d loss / d z_last
    grads = []
    for k in range(len(layers) - 1, -1, -1):
        W, _ = layers[k]
        a_in = acts[k]
        grads.append((a_in.T @ g, g.sum(axis=0)))
        if k > 0:
            g = (g @ W.T) * dsilu(zs[k - 1])
    grads.reverse()
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat
