"""Multicolour inexact Uzawa relaxation (oracle; test infrastructure).

Paper Sec. 3.2, eq. uzawa-iteration with the split steps eq. uzawa-velocity
(xi Gauss-Seidel iterations on A u = f - B^T p_k) and eq. uzawa-pressure
(p <- p - S_hat^{-1}(g - B u + C p_k)); A_f = forward Gauss-Seidel, A_s = one
forward and one backward sweep.

Orderings.  The paper relaxes in lexicographic order; here every Gauss-Seidel
sweep visits colour classes that have no coupling inside a class, so each
class can be updated at once.  P1 nodes (I,J,K): colour (I+J+K) mod 2.  P2
nodes on the doubled lattice (X,Y,Z): vertex nodes take ((X+Y+Z)/2) mod 2,
edge nodes take 2 + the index of their parity class in mesh.EDGE_DIRS.  Two
vertex classes suffice because the stiffness of a Kuhn tetrahedron couples
two vertex functions through grad(lambda_i) . grad(lambda_j) (P1 and the P2
vertex functions alike), which vanishes for every edge off the lattice axes
(face and body diagonals), so vertex nodes are coupled only to their six axis
neighbours.  A forward sweep visits colours in ascending order, a backward
sweep in descending order.  Inside a colour every update reads the state at
the start of that colour.

Pressure Schur approximation: S_hat = omega^{-1} D with a positive diagonal
D, so the pressure step is p <- p - omega D^{-1} (g - B u + C p), and
omega^{-1} is the largest eigenvalue of D^{-1}(C + B A_s^{-1} B^T) (eq.
omega-eigenvalue-problem, where D is the lumped P1 mass M_L), estimated by
power iteration.  Two choices of D:

* "ml": D = M_L, the matrix of the eigenproblem (default);
* "sd": D = diag(C + B diag(A)^{-1} B^T) over interior velocity DoFs, the
  diagonal of the Schur complement with A replaced by its diagonal; this
  weakens the pressure step less at boundary pressure nodes, where the
  Schur complement is much smaller than M_L.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import mesh


def colours(lev):
    """Colour of every velocity node (lattice order); a level that carries its
    own colouring (unstructured meshes, umesh.ULevel) gives it directly."""
    if hasattr(lev, "colour"):
        return lev.colour
    c = lev.vcoords
    if lev.vorder == 1:
        return (c.sum(axis=1)) % 2
    par = c % 2
    out = np.full(c.shape[0], -1, dtype=np.int64)
    isv = np.all(par == 0, axis=1)
    out[isv] = (c[isv].sum(axis=1) // 2) % 2
    for g, d in enumerate(mesh.EDGE_DIRS):
        sel = np.all(par == np.array(d), axis=1)
        out[sel] = 2 + g
    return out


def n_colours(vorder):
    return 2 if vorder == 1 else 9


def schur_diagonal(stokes, mode):
    """The diagonal D of S_hat = omega^{-1} D (see module docstring)."""
    lev = stokes.lev
    if mode == "ml":
        return lev.ML.copy()
    if mode == "sd":
        dinv = np.where(lev.vint, 1.0 / lev.Adiag, 0.0)
        d = lev.C.diagonal().copy()
        for b in lev.B:
            d += np.asarray(b.multiply(b) @ dinv).ravel()
        return d
    raise ValueError(mode)


class Uzawa:
    def __init__(self, stokes, schur="ml"):
        self.S = stokes
        self.D = schur_diagonal(stokes, schur)
        lev = stokes.lev
        col = colours(lev)
        self.ncol = getattr(lev, "ncolours", n_colours(lev.vorder))
        self.rows = []
        for c in range(self.ncol):
            idx = np.nonzero((col == c) & lev.vint)[0]
            self.rows.append((idx, lev.A[idx, :].tocsr(), [bt[idx, :].tocsr() for bt in stokes.BT]))
        self.invdiag = 1.0 / lev.Adiag

    def colour_update(self, c, us, f_us, p):
        """One colour of Gauss-Seidel on A u_d = f_d - (B^T p)_d, all d at once."""
        idx, Arows, BTrows = self.rows[c]
        if idx.size == 0:
            return
        for d in range(3):
            r = f_us[d][idx] - Arows @ us[d] - BTrows[d] @ p
            us[d][idx] = us[d][idx] + r * self.invdiag[idx]

    def sweep(self, us, f_us, p, forward=True):
        order = range(self.ncol) if forward else range(self.ncol - 1, -1, -1)
        for c in order:
            self.colour_update(c, us, f_us, p)

    def velocity_relax(self, us, f_us, p, gs, xi):
        for _ in range(xi):
            self.sweep(us, f_us, p, True)
            if gs == "s":
                self.sweep(us, f_us, p, False)

    def pressure_update(self, us, p, g, omega):
        rp = g - self.S.apply_B(us) + self.S.apply_C(p)
        return p - omega * rp / self.D

    def iterate(self, x, b, gs="f", xi=1, omega=1.0):
        """One inexact Uzawa iteration (eq. uzawa-iteration) on x; returns new x."""
        us, p = self.S.split(x.copy())
        us = [u.copy() for u in us]
        f_us, g = self.S.split(b)
        self.velocity_relax(us, f_us, p, gs, xi)
        p = self.pressure_update(us, p, g, omega)
        return self.S.join(us, p)

    def symmetric_sweep_solve(self, rhs_us):
        """A_s^{-1} v: one forward + one backward sweep on A z = v from z = 0."""
        zs = [np.zeros(self.S.nv) for _ in range(3)]
        zero_p = np.zeros(self.S.np_)
        self.sweep(zs, rhs_us, zero_p, True)
        self.sweep(zs, rhs_us, zero_p, False)
        return zs

    def estimate_omega_inv(self, v0, iters=100):
        """Power iteration on D^{-1}(C + B A_s^{-1} B^T) (eq. omega-eigenvalue-problem).

        v0: start vector on the pressure nodes (the caller draws it).  The
        start vector is projected to mean zero and normalised; each step maps
        v -> w, reports lambda = ||w|| / ||v|| and continues with w/||w||.
        """
        lev = self.S.lev
        m = lev.ML
        D = self.D
        v = v0 - (m @ v0) / m.sum() if not lev.neumann else np.array(v0, dtype=float)
        v = v / np.linalg.norm(v)
        lam = 0.0
        for _ in range(iters):
            bt = self.S.apply_BT(v)
            bt = [np.where(lev.vint, b, 0.0) for b in bt]
            z = self.symmetric_sweep_solve(bt)
            w = (self.S.apply_C(v) + self.S.apply_B(z)) / D
            lam = np.linalg.norm(w)
            v = w / lam
        return lam


class LexUzawa(Uzawa):
    """The paper's ordering (Sec. 5.2.1: lexicographic update inside each
    primitive, primitives in turn): pointwise Gauss-Seidel over the velocity
    unknowns in node order -- lattice order on the lattice levels, canonical
    order (vertices, edges, faces, cells of T_0; lexicographic inside) on
    unstructured levels.  A forward sweep is u <- u + (D + L)^{-1}(f - B^T p
    - A u) over the interior rows, D + L the lower triangle of A in that
    order (backward: the upper triangle), solved as a triangular system;
    for comparison with the multicolour order only."""

    def __init__(self, stokes, schur="ml"):
        super().__init__(stokes, schur)
        lev = stokes.lev
        self.vi = np.nonzero(lev.vint)[0]
        Aii = lev.A[self.vi][:, self.vi]
        self.lower = sp.tril(Aii, format="csr")
        self.upper = sp.triu(Aii, format="csr")
        self.Afull = lev.A

    def sweep(self, us, f_us, p, forward=True):
        T = self.lower if forward else self.upper
        bt = self.S.apply_BT(p)
        for d in range(3):
            r = (f_us[d] - self.Afull @ us[d] - bt[d])[self.vi]
            us[d][self.vi] = us[d][self.vi] + spla.spsolve_triangular(T, r, lower=forward)
