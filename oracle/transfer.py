"""Grid transfer (oracle; test infrastructure).

Paper Sec. 3.3: prolongation I_l^{l+1} evaluates the coarse finite-element
function at the fine nodes -- quadratic for P2 fields, linear otherwise,
velocity and pressure independently; restriction is its transpose.

The prolongation matrix is built by point location: every fine node is located
in a coarse Kuhn simplex and the coarse basis functions are evaluated at its
barycentric coordinates.
"""
import numpy as np
import scipy.sparse as sp

from . import fe, mesh


def locate(Nc, pts):
    """Containing coarse Kuhn simplex and barycentric coordinates.

    pts: (n, 3) float positions in coarse lattice units ([0, Nc]^3).  Returns
    (vertices (n, 4, 3) integer coarse coordinates, lam (n, 4)).  Inside a
    lattice cube the Kuhn simplex holding a point is the one whose step order
    sorts the local coordinates in decreasing order.
    """
    pts = np.asarray(pts, dtype=float)
    cube = np.clip(np.floor(pts), 0, Nc - 1).astype(np.int64)
    t = pts - cube
    order = np.argsort(-t, axis=1, kind="stable")
    ts = np.take_along_axis(t, order, axis=1)
    lam = np.stack([1.0 - ts[:, 0], ts[:, 0] - ts[:, 1], ts[:, 1] - ts[:, 2], ts[:, 2]], axis=1)
    n = pts.shape[0]
    V = np.zeros((n, 4, 3), dtype=np.int64)
    V[:, 0] = cube
    for s in range(3):
        step = np.zeros((n, 3), dtype=np.int64)
        step[np.arange(n), order[:, s]] = 1
        V[:, s + 1] = V[:, s] + step
    return V, lam


def _eval_basis(order, lam):
    """Values (n, nloc) of the barycentric basis at lam."""
    if order == 1:
        return lam.copy()
    cols = [lam[:, i] * (2 * lam[:, i] - 1) for i in range(4)]
    cols += [4 * lam[:, i] * lam[:, j] for (i, j) in mesh.P2_EDGES]
    return np.stack(cols, axis=1)


def prolongation(Nc, order):
    """Sparse I_l^{l+1}: fine lattice (2 Nc intervals) <- coarse lattice (Nc)."""
    Nf = 2 * Nc
    if order == 1:
        fc = mesh.p1_coords(Nf).astype(float) / 2.0          # in coarse units
        nf, ncs = (Nf + 1) ** 3, (Nc + 1) ** 3
    else:
        fc = mesh.p2_coords(Nf).astype(float) / 4.0
        nf, ncs = (2 * Nf + 1) ** 3, (2 * Nc + 1) ** 3
    V, lam = locate(Nc, fc)
    W = _eval_basis(order, lam)
    cols = fe.element_dofs(V, Nc, order)
    rows = np.repeat(np.arange(nf)[:, None], cols.shape[1], axis=1)
    keep = np.abs(W) > 1e-15
    P = sp.csr_matrix((W[keep], (rows[keep], cols[keep])), shape=(nf, ncs))
    return P


class Transfer:
    """Prolongation / restriction of whole Stokes vectors between two levels."""

    def __init__(self, Sc, Sf):
        self.Sc, self.Sf = Sc, Sf
        Nc = Sc.lev.N
        vo = Sc.lev.vorder
        self.Pv = prolongation(Nc, vo)
        self.Pp = prolongation(Nc, 1)
        self.Rv = self.Pv.T.tocsr()
        self.Rp = self.Pp.T.tocsr()

    def prolong(self, xc):
        us, p = self.Sc.split(xc)
        return self.Sf.join([self.Pv @ u for u in us], self.Pp @ p)

    def restrict(self, rf):
        """Transpose of prolong, on a residual whose boundary velocity rows are
        zero; coarse boundary velocity rows are set to zero and the pressure part
        is shifted to zero sum (compatibility with the null vector (0, 1))."""
        us, p = self.Sf.split(self.Sf.zero_boundary(rf))
        rc = self.Sc.join([self.Rv @ u for u in us], self.Rp @ p)
        rc = self.Sc.zero_boundary(rc)
        if self.Sc.lev.neumann:          # no null vector: nothing to be compatible with
            return rc
        uc, pc = self.Sc.split(rc)
        return self.Sc.join(uc, pc - pc.mean())
