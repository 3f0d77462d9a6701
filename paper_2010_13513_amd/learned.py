"""Learned coarse solve: training-pair collection, GPU training and held-out
evaluation around the C ABI.

Not in the paper.  A network stands in for the exact coarsest-level solve of
Alg. fmg: it maps [r / ||r||, log nu at the coarse P1 nodes] to the exact
correction A0(nu)^+ r / ||r|| (pressure at zero mean).  Pairs are recorded by
the library at the coarse-grid visits of plain (exact-coarse-solve) FMG solves
over seeded log-normal viscosity and Fourier forcing fields; the network is
trained by the library's own forward / backward / Adam kernels; the plain
solver stays the fallback (residual-ratio monitor of hhg_fmg_solve).  This
module only loops over seeds and calls the library; random numbers (initial
weights, minibatch order) are drawn here and passed in.
"""
import time

import numpy as np

from . import hhg, workloads as W
from .problem import Problem

# seeds: training fields from TRAIN_BASE, held-out fields from TEST_BASE
TRAIN_BASE = W.SEED_BASE + 5000 + 100000
TEST_BASE = W.SEED_BASE + 5000 + 900000


def forcing_seed(nu_seed):
    return nu_seed + 50000


def init_params(rng, n_in, hidden, n_out):
    """He-uniform weights, zero biases, in the library's parameter order."""
    dims = [n_in, hidden, hidden, hidden, n_out]
    out = []
    for l in range(4):
        lim = np.sqrt(6.0 / dims[l])
        out.append(rng.uniform(-lim, lim, size=(dims[l + 1], dims[l])).ravel())
        out.append(np.zeros(dims[l + 1]))
    return np.concatenate(out).astype(np.float32)


def solve_instance(P, nu_seed, prm, x=None, want_stats=True):
    """Set the seed's viscosity on every level, build its right-hand sides
    and boundary data, run hhg_fmg_solve.  Returns (x, stats, seconds of the
    solve) -- a solve that stops at max_cycles returns its stats too."""
    P.set_viscosity(W.lognormal_viscosity(nu_seed))
    prob = W.fourier_forcing(forcing_seed(nu_seed))
    bs = P.rhs(prob)
    x = P.boundary(prob) if x is None else x
    P.torch.cuda.synchronize()
    t0 = time.perf_counter()
    try:
        st = hhg.hhg_fmg_solve(P.h, x, bs, prm, want_stats=want_stats)
    except hhg.HHGError as e:
        if e.status != hhg.HHG_ERR_NOT_CONVERGED:
            raise
        st = None
    P.torch.cuda.synchronize()
    return x, st, time.perf_counter() - t0


def collect_pairs(P, seeds, prm, n_pairs, per_seed=None, log=None):
    """Record up to n_pairs (features, targets) from the exact coarse solves
    of plain FMG solves over the given viscosity seeds, at most per_seed from
    one seed (the first coarse-grid visits of its solve).  Returns device
    float32 tensors (n, n_in), (n, n_out) and the number of seeds used."""
    torch = P.torch
    n_in, n_out = hhg.hhg_mlp_dims(P.h)
    F = torch.zeros(n_pairs, n_in, dtype=torch.float32, device=P.dev)
    T = torch.zeros(n_pairs, n_out, dtype=torch.float32, device=P.dev)
    k, used = 0, 0
    t0 = time.perf_counter()
    for s in seeds:
        if k >= n_pairs:
            break
        cap = n_pairs - k if per_seed is None else min(per_seed, n_pairs - k)
        hhg.hhg_record_pairs(P.h, F[k:], T[k:], cap)
        solve_instance(P, s, prm)
        k += hhg.hhg_recorded_pairs(P.h)
        used += 1
        if log and used % 100 == 0:
            log(f"[pairs] {used} seeds, {k} pairs, {time.perf_counter() - t0:.1f} s")
    hhg.hhg_record_pairs(P.h, None, None, 0)
    return F[:k], T[:k], used


def train(ctx, F, T, hidden=512, batch=256, epochs=100, lr=1e-3, lr_final=1e-4, stages=4, seed=0, log=None):
    """Train a network on (F, T) with Adam, the learning rate stepped
    geometrically from lr to lr_final over `stages` stages.

    Inputs and outputs are normalised for training -- each feature group
    (the residual part, the log-viscosity part) and the targets divided by
    their root-mean-square -- and the scales are folded exactly into the
    first layer's columns and the last layer's rows afterwards, so the
    returned network takes the library's raw features.  Odd symmetry of the
    exact map (the correction of -r is minus the correction of r) is added
    to the data by appending (-r, log nu) -> -target pairs.

    Returns the handle (caller destroys it) and the loss history (mean batch
    loss of the last epoch of every stage, normalised units)."""
    import torch
    n, n_in = F.shape
    n_out = T.shape[1]
    rms = lambda a: float(a.double().pow(2).mean().sqrt().clamp_min(1e-30))
    s_r, s_n, s_t = rms(F[:, :n_out]), rms(F[:, n_out:]) if n_in > n_out else 1.0, rms(T)
    Fn = torch.cat([F[:, :n_out] / s_r, F[:, n_out:] / s_n], dim=1)
    Fn = torch.cat([Fn, torch.cat([-Fn[:, :n_out], Fn[:, n_out:]], dim=1)]).contiguous()
    Tn = torch.cat([T / s_t, -T / s_t]).contiguous()
    n2 = 2 * n
    rng = np.random.default_rng(seed)
    m = hhg.hhg_mlp_create(ctx, n_in, hidden, n_out, max(batch, 256))
    hhg.hhg_mlp_set_params(m, init_params(rng, n_in, hidden, n_out))
    hist = []
    per = max(1, epochs // stages)
    for st in range(stages):
        rate = lr * (lr_final / lr) ** (st / max(stages - 1, 1))
        order = np.concatenate([rng.permutation(n2) for _ in range(per)]).astype(np.int32)
        t0 = time.perf_counter()
        hist.append(hhg.hhg_mlp_train(m, Fn, Tn, n2, batch, per, rate, order))
        if log:
            log(f"[train] stage {st}: lr {rate:.2e}, {per} epochs, loss {hist[-1]:.4e}, "
                f"{time.perf_counter() - t0:.1f} s")
    # fold the normalisation into W1 (columns) and W4, b4 (rows)
    p = hhg.hhg_mlp_get_params(m).astype(np.float64)
    w1 = p[:hidden * n_in].reshape(hidden, n_in)
    w1[:, :n_out] /= s_r
    w1[:, n_out:] /= s_n
    o4 = hidden * n_in + hidden + 2 * (hidden * hidden + hidden)
    p[o4:o4 + n_out * hidden] *= s_t
    p[o4 + n_out * hidden:] *= s_t
    hhg.hhg_mlp_set_params(m, p.astype(np.float32))
    return m, hist


def pair_errors(P, m, F, T, chunk=256):
    """Relative error ||net(f) - t|| / ||t|| of every pair (device metrics)."""
    torch = P.torch
    n, n_out = T.shape
    Y = torch.empty(chunk, n_out, dtype=torch.float32, device=P.dev)
    errs = []
    for i in range(0, n, chunk):
        b = min(chunk, n - i)
        hhg.hhg_mlp_forward(m, F[i:i + b], b, Y)
        d = (Y[:b] - T[i:i + b]).double().norm(dim=1) / T[i:i + b].double().norm(dim=1).clamp_min(1e-300)
        errs.append(d)
    torch.cuda.synchronize()
    return torch.cat(errs).cpu().numpy()


def cycle_rates(P, nu_seed, prm, cycles=6):
    """Residual reduction per V-cycle (hhg_vcycle, then zero pressure mean)
    from the boundary data with zero interior, for the coarse treatment the
    hierarchy and prm select.  Returns the list of ratios."""
    P.set_viscosity(W.lognormal_viscosity(nu_seed))
    prob = W.fourier_forcing(forcing_seed(nu_seed))
    b = P.rhs(prob)[-1]
    x = P.boundary(prob)
    L = P.lmax
    r = P.torch.empty_like(x)
    out, prev = [], None
    for c in range(cycles + 1):
        hhg.hhg_residual(P.h, L, x, b, r)
        ru, rp = hhg.hhg_norms(P.h, L, r)
        rn = float(np.hypot(ru, rp))
        if prev is not None:
            out.append(rn / prev)
        prev = rn
        if c < cycles:
            hhg.hhg_vcycle(P.h, L, x, b, prm)
            hhg.hhg_project_mean_zero(P.h, L, x)
    return out
