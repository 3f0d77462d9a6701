"""Float64 oracle of the coarse-grid MLP (test infrastructure).

Not in the paper: a small network that maps the coarsest-level residual to a
correction, used in place of the exact coarse solve of Alg. fmg.  Model:
four dense layers n_in -> H -> H -> H -> n_out with ReLU between them;
weights and the inputs of every layer are stored in bfloat16 (round to
nearest even), products are summed in higher precision.  Loss: mean squared
error over the n_out outputs of a batch.

`quantize=True` reproduces the bfloat16 storage points of the GPU model
(weights, layer inputs, and the output/hidden gradients that enter the
weight- and data-gradient products); `quantize=False` is the plain real
network, used for the finite-difference pins.
"""
import numpy as np


def bf16(x):
    """Round float64 values to bfloat16 (round to nearest even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if np.any(nan):
        out[nan] = np.nan
    return out


class MLP:
    """params: list [W1, b1, W2, b2, W3, b3, W4, b4], W_l of shape (out, in)."""

    def __init__(self, params, quantize=True):
        self.p = [np.asarray(a, dtype=np.float64) for a in params]
        self.q = quantize

    def _r(self, x):
        return bf16(x) if self.q else x

    def forward(self, X):
        """Returns the output and the cache of layer inputs / pre-activations."""
        a = self._r(X)
        cache = []
        n = len(self.p) // 2
        for l in range(n):
            W, b = self._r(self.p[2 * l]), self.p[2 * l + 1]
            z = a @ W.T + b
            cache.append((a, z))
            a = self._r(np.maximum(z, 0.0)) if l < n - 1 else z
        return a, cache

    def loss_and_grads(self, X, Y):
        """MSE loss (1 / (B n_out)) sum (out - Y)^2 and its gradient wrt params."""
        out, cache = self.forward(X)
        B, m = Y.shape
        diff = out - Y
        loss = float(np.sum(diff * diff) / (B * m))
        g = self._r(2.0 * diff / (B * m))          # d loss / d z_last
        grads = [None] * len(self.p)
        n = len(self.p) // 2
        for l in range(n - 1, -1, -1):
            a, z = cache[l]
            W = self._r(self.p[2 * l])
            grads[2 * l] = g.T @ a
            grads[2 * l + 1] = g.sum(axis=0)
            if l > 0:
                da = g @ W
                zprev = cache[l - 1][1]
                g = self._r(da * (zprev > 0))
        return loss, grads


def init_params(rng, n_in, H, n_out):
    """He-uniform weights and zero biases from a numpy Generator (the caller
    draws; both sides receive the same numbers)."""
    dims = [n_in, H, H, H, n_out]
    ps = []
    for l in range(4):
        fan_in = dims[l]
        lim = np.sqrt(6.0 / fan_in)
        ps.append(rng.uniform(-lim, lim, size=(dims[l + 1], dims[l])))
        ps.append(np.zeros(dims[l + 1]))
    return ps


def adam_step(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) on float64 master parameters."""
    out = []
    for k, (p, g) in enumerate(zip(params, grads)):
        m[k] = b1 * m[k] + (1 - b1) * g
        v[k] = b2 * v[k] + (1 - b2) * g * g
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        out.append(p - lr * mh / (np.sqrt(vh) + eps))
    return out
