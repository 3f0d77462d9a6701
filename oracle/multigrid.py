"""Variable V-cycle and full multigrid (oracle; test infrastructure).

Paper Alg. fmg: exact solve on the coarsest level, then for each finer level
FMG interpolation followed by kappa variable V-cycles; the V-cycle on level l
inside a cycle with finest level l_fine does nu_pre + (l_fine - l) nu_inc
Uzawa iterations, restricts the defect, recurses with a zero initial guess,
prolongs and adds the correction, and does nu_post + (l_fine - l) nu_inc
post-smoothing iterations.  The paper's level 0 is the coarsest level of the
hierarchy here (Lmin).

Readings where the paper is silent: b_l is rediscretised on every level; after
FMG interpolation the boundary velocity values are reset to the interpolant of
the boundary data; the pressure is projected to mean zero after every cycle on
the finest level of the current FMG stage.

Error metrics: eq. error (M-norm of x*_{l+1} - I x~_l on level l+1, pressures
normalised to zero mean first), eq. gamma, eq. relative-error.
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fe
from .coarse import CoarseSolver
from .smoother import Uzawa
from .stokes import Stokes
from .transfer import Transfer


@dataclass
class Params:
    """FMG(nu_pre, nu_post, nu_inc, kappa, A_hat, xi) of Alg. fmg."""
    nu_pre: int = 1
    nu_post: int = 1
    nu_inc: int = 0
    kappa: int = 1
    gs: str = "f"      # "f": A_f (forward GS), "s": A_s (symmetric)
    xi: int = 1
    omega_inv: float = 0.5


@dataclass
class Problem:
    """Velocity / pressure fields and forcing as numpy callables of (x, y, z)."""
    u: object
    p: object
    f: object


class Hierarchy:
    def __init__(self, vorder, Lmin, Lmax, macro_refine=0, nu_fn=None, schur="ml", neumann=()):
        self.vorder = vorder
        self.Lmin, self.Lmax = Lmin, Lmax
        self.mr = macro_refine
        self.nu_fn = nu_fn
        self.neumann = tuple(neumann)
        self.S, self.U, self.T = {}, {}, {}
        for l in range(Lmin, Lmax + 1):
            self.S[l] = Stokes(self.make_level(l))
            self.U[l] = Uzawa(self.S[l], schur)
        for l in range(Lmin + 1, Lmax + 1):
            self.T[l] = Transfer(self.S[l - 1], self.S[l])
        self.coarse = CoarseSolver(self.S[Lmin])

    def N(self, l):
        return 2 ** (l + self.mr)

    def make_level(self, l):
        N = self.N(l)
        nu = None
        if self.nu_fn is not None:
            from . import mesh
            c = mesh.p1_coords(N) / float(N)
            nu = self.nu_fn(c[:, 0], c[:, 1], c[:, 2])
        return fe.Level(N, self.vorder, nu, self.neumann)

    # ------------------------------------------------------------ cycles
    def smooth(self, l, x, b, its, prm):
        for _ in range(its):
            x = self.U[l].iterate(x, b, prm.gs, prm.xi, 1.0 / prm.omega_inv)
        return x

    def vcycle(self, lf, l, x, b, prm):
        if l == self.Lmin:
            return self.coarse.solve(x, b)
        S = self.S[l]
        x = self.smooth(l, x, b, prm.nu_pre + (lf - l) * prm.nu_inc, prm)
        rc = self.T[l].restrict(S.residual(x, b))
        xc = self.vcycle(lf, l - 1, self.S[l - 1].zeros(), rc, prm)
        x = x + self.T[l].prolong(xc)
        x = self.smooth(l, x, b, prm.nu_post + (lf - l) * prm.nu_inc, prm)
        return x

    def boundary_data(self, l, prob):
        return self.S[l].interpolate(prob.u, prob.p)

    def rhs(self, l, prob):
        return self.S[l].rhs(prob.f)

    def initial(self, l, prob):
        """Boundary data in the velocity boundary DoFs, zero elsewhere."""
        S = self.S[l]
        return S.set_boundary(S.zeros(), self.boundary_data(l, prob))

    def fmg(self, prob, prm, b=None, cycles_on_finest=0):
        """Alg. fmg; returns x on Lmax (plus optional extra V-cycles on Lmax)."""
        bs = {l: (self.rhs(l, prob) if b is None else b[l]) for l in range(self.Lmin, self.Lmax + 1)}
        x = self.coarse.solve(self.initial(self.Lmin, prob), bs[self.Lmin])
        for l in range(self.Lmin + 1, self.Lmax + 1):
            S = self.S[l]
            x = S.set_boundary(self.T[l].prolong(x), self.boundary_data(l, prob))
            for _ in range(prm.kappa):
                x = S.mean_zero(self.vcycle(l, l, x, bs[l], prm))
        for _ in range(cycles_on_finest):
            x = self.S[self.Lmax].mean_zero(self.vcycle(self.Lmax, self.Lmax, x, bs[self.Lmax], prm))
        return x

    # ------------------------------------------------------- exact discrete
    def sparse_system(self, l):
        lev = self.S[l].lev
        A = lev.A
        Z = None
        blocks = [[A, Z, Z, lev.B[0].T], [Z, A, Z, lev.B[1].T], [Z, Z, A, lev.B[2].T],
                  [lev.B[0], lev.B[1], lev.B[2], -lev.C]]
        return sp.bmat(blocks, format="csr")

    def exact_discrete(self, l, prob, b=None):
        """Discrete solution by a sparse direct solve (scipy spsolve).

        The all-Dirichlet system is singular only along (0, 1_p); fixing the
        last pressure unknown to zero removes that direction, and the result
        is then shifted to zero pressure mean (int p = 0, Sec. 2).  With an
        outflow face the system is regular and solved on all unknowns."""
        from .coarse import unknown_index
        S = self.S[l]
        b = self.rhs(l, prob) if b is None else b
        x0 = self.initial(l, prob)
        idx = unknown_index(S)
        if not S.lev.neumann:
            idx = idx[:-1]
        K = self.sparse_system(l)[idx][:, idx].tocsc()
        r = S.residual(x0, b)[idx]
        sol = spla.spsolve(K, r)
        x = x0.copy()
        x[idx] += sol
        return S.mean_zero(x)

    # --------------------------------------------------------------- norms
    def residual_norms(self, l, x, b):
        r = self.S[l].residual(x, b)
        us, p = self.S[l].split(r)
        return float(np.sqrt(sum(u @ u for u in us))), float(np.linalg.norm(p))


def l2_errors(H_fine_stokes, T_up, x_l, prob):
    """eq. error: M-norm errors of (u, p) on level l+1 of the prolonged x_l.

    H_fine_stokes: Stokes object of level l+1; T_up: Transfer l -> l+1.
    """
    Sf = H_fine_stokes
    xf = T_up.prolong(x_l)
    xs = Sf.interpolate(prob.u, prob.p)
    us, p = Sf.split(xf)
    ws, ps = Sf.split(xs)
    m = Sf.lev.ML
    if not Sf.lev.neumann:          # pressure fixed only up to a constant
        p = p - (m @ p) / m.sum()
        ps = ps - (m @ ps) / m.sum()
    eu = np.sqrt(sum((w - u) @ (Sf.lev.M @ (w - u)) for u, w in zip(us, ws)))
    ep = np.sqrt((ps - p) @ (Sf.lev.Mp @ (ps - p)))
    return float(eu), float(ep)


def relative_error(S, x_tilde, x_ref):
    """eq. relative-error in the M-norm, separately for u and p."""
    us, p = S.split(x_tilde - x_ref)
    ur, pr = S.split(x_ref)
    M, Mp = S.lev.M, S.lev.Mp
    du = np.sqrt(sum(u @ (M @ u) for u in us)) / np.sqrt(sum(u @ (M @ u) for u in ur))
    dp = np.sqrt(p @ (Mp @ p)) / np.sqrt(pr @ (Mp @ pr))
    return float(du), float(dp)
