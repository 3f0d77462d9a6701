"""Coarsest-grid solve (oracle; test infrastructure).

Alg. fmg solves calA_0 x_0 = b_0 exactly on the coarsest level (the paper uses
a sparse direct solver).  The coarse system on the unknowns -- interior
velocity DoFs and all pressure DoFs -- is singular (null vector (0, 1_p) for
an all-Dirichlet boundary), so the exact solve is taken as the minimum-norm
least-squares solution by the SVD pseudo-inverse with relative cut-off 1e-12,
followed by the mean-zero pressure projection.
"""
import numpy as np


def unknown_index(S):
    """Indices (into the oracle Stokes vector) of the coarse unknowns."""
    vi = np.nonzero(S.lev.vint)[0]
    nv = S.nv
    return np.concatenate([vi, nv + vi, 2 * nv + vi, 3 * nv + np.arange(S.np_)])


def dense_system(S):
    """calA restricted to the unknowns, assembled column by column."""
    idx = unknown_index(S)
    n = idx.size
    K = np.zeros((n, n))
    e = np.zeros(S.n)
    for c, j in enumerate(idx):
        e[:] = 0.0
        e[j] = 1.0
        K[:, c] = S.apply(e)[idx]
    return K, idx


class CoarseSolver:
    def __init__(self, S, rcond=1e-12):
        self.S = S
        self.K, self.idx = dense_system(S)
        U, s, Vt = np.linalg.svd(self.K)
        self.sv = s
        keep = s > rcond * s[0]
        self.rank = int(keep.sum())
        self.Kp = (Vt[keep].T / s[keep]) @ U[:, keep].T

    def solve(self, x, b):
        """x <- x + K^+ (b - calA x) on the unknowns, then mean-zero pressure."""
        r = self.S.residual(x, b)
        y = x.copy()
        y[self.idx] += self.Kp @ r[self.idx]
        return self.S.mean_zero(y)
