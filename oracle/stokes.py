"""Discrete Stokes saddle-point operator (oracle; test infrastructure).

Paper eq. stokes-discrete: calA = [[A, B^T], [B, -C]], A = diag(A, A, A).
Vectors hold every DoF of a level including the Dirichlet velocity DoFs, which
carry the boundary data w; the lifting terms of the right-hand side (the
boundary sums in the definition of f and g) then appear by applying the
operator to the full vector.  Operator rows exist for interior velocity DoFs
and for all pressure DoFs; boundary velocity rows of every output are zero.

Vector layout (oracle only): x = [u_1, u_2, u_3, p] with each velocity
component in the level's velocity lattice order and p in P1 lattice order.
"""
import numpy as np


class Stokes:
    def __init__(self, lev):
        self.lev = lev
        self.nv = lev.nv
        self.np_ = lev.np_
        self.n = 3 * lev.nv + lev.np_
        self.BT = [b.T.tocsr() for b in lev.B]

    # ---- vector helpers
    def split(self, x):
        nv = self.nv
        return [x[d * nv:(d + 1) * nv] for d in range(3)], x[3 * nv:]

    def join(self, us, p):
        return np.concatenate(list(us) + [p])

    def zeros(self):
        return np.zeros(self.n)

    # ---- blocks
    def apply_A(self, us):
        return [self.lev.A @ u for u in us]

    def apply_BT(self, p):
        return [bt @ p for bt in self.BT]

    def apply_B(self, us):
        return sum(b @ u for b, u in zip(self.lev.B, us))

    def apply_C(self, p):
        return self.lev.C @ p

    def apply(self, x):
        """y = calA x with zero boundary velocity rows."""
        us, p = self.split(x)
        Au = self.apply_A(us)
        Bp = self.apply_BT(p)
        vi = self.lev.vint
        yu = [np.where(vi, a + b, 0.0) for a, b in zip(Au, Bp)]
        yp = self.apply_B(us) - self.apply_C(p)
        return self.join(yu, yp)

    def apply_block(self, x, which):
        """Single blocks, laid out like apply(): A, BT, B, C, MASS."""
        us, p = self.split(x)
        vi = self.lev.vint
        z = np.zeros(self.nv)
        if which == "A":
            return self.join([np.where(vi, a, 0.0) for a in self.apply_A(us)], np.zeros(self.np_))
        if which == "BT":
            return self.join([np.where(vi, b, 0.0) for b in self.apply_BT(p)], np.zeros(self.np_))
        if which == "B":
            return self.join([z, z, z], self.apply_B(us))
        if which == "C":
            return self.join([z, z, z], self.apply_C(p))
        if which == "MASS":
            return self.join([self.lev.M @ u for u in us], self.lev.Mp @ p)
        raise ValueError(which)

    def residual(self, x, b):
        """r = b - calA x, boundary velocity rows zero."""
        r = b - self.apply(x)
        us, p = self.split(r)
        vi = self.lev.vint
        return self.join([np.where(vi, u, 0.0) for u in us], p)

    # ---- problem data
    def rhs(self, f_fn):
        """b = (M I(f) on interior velocity rows, 0): Sec. 2 right-hand side with
        the load integral taken as the mass matrix times the nodal interpolant."""
        pos = self.lev.vpos()
        fv = f_fn(pos[:, 0], pos[:, 1], pos[:, 2])
        vi = self.lev.vint
        us = [np.where(vi, self.lev.M @ fv[d], 0.0) for d in range(3)]
        return self.join(us, np.zeros(self.np_))

    def interpolate(self, u_fn, p_fn=None):
        """Nodal interpolant of a velocity (and pressure) field."""
        pos = self.lev.vpos()
        uv = u_fn(pos[:, 0], pos[:, 1], pos[:, 2])
        pp = self.lev.ppos()
        p = np.zeros(self.np_) if p_fn is None else p_fn(pp[:, 0], pp[:, 1], pp[:, 2]) * np.ones(self.np_)
        return self.join([np.asarray(uv[d], float) * np.ones(self.nv) for d in range(3)], p)

    def set_boundary(self, x, w):
        """Copy the boundary velocity values of w into x."""
        us, p = self.split(x)
        ws, _ = self.split(w)
        vb = self.lev.vbnd
        return self.join([np.where(vb, wd, ud) for ud, wd in zip(us, ws)], p)

    def zero_boundary(self, x):
        us, p = self.split(x)
        vi = self.lev.vint
        return self.join([np.where(vi, u, 0.0) for u in us], p)

    def mean_zero(self, x):
        """p <- p - (m^T p / m^T 1) 1 with m_k = int psi_k (Sec. 2, int p = 0).
        With an outflow boundary the pressure is determined and x is returned
        unchanged."""
        if self.lev.neumann:
            return x
        us, p = self.split(x)
        m = self.lev.ML
        return self.join(us, p - (m @ p) / m.sum())
