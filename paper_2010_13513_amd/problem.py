"""Host-side marshalling of problem data for one libhhg hierarchy.

Evaluates analytic fields (boundary data, forcing, viscosity) at the lattice
nodes of a level, hands them to the library in its layout, and builds the
right-hand sides of every level with the library's own kernels.  Nothing here
does any of the solver's arithmetic; the fields come from `workloads`.
"""
import numpy as np

from . import hhg


class Problem:
    """A hierarchy (levels lmin..lmax of one discretisation) on the given
    device plus the vectors of one problem instance."""

    def __init__(self, torch, ctx, disc, lmin, lmax, macro_refine=0, schur=hhg.HHG_SCHUR_SD, device="cuda:0"):
        self.torch = torch
        self.ctx = ctx
        self.disc = disc
        self.lmin, self.lmax, self.mr = lmin, lmax, macro_refine
        self.dev = torch.device(device)
        mesh = hhg.hhg_mesh_cube(ctx, macro_refine)
        try:
            self.h = hhg.hhg_hier_create(mesh, disc, lmin, lmax, schur)
        finally:
            hhg.hhg_mesh_destroy(mesh)
        self.has_nu = False

    def close(self):
        if self.h is not None:
            self.torch.cuda.synchronize()
            hhg.hhg_hier_destroy(self.h)
            self.h = None

    # ------------------------------------------------------------ lattices
    def N(self, level):
        return 2 ** (level + self.mr)

    def dofs(self, level):
        """All DoFs of a level, Dirichlet ones included."""
        N = self.N(level)
        m = N if self.disc == hhg.HHG_P1P1 else 2 * N
        return 3 * (m + 1) ** 3 + (N + 1) ** 3

    @staticmethod
    def _grid(M):
        t = np.arange(M + 1) / float(M)
        Z, Y, X = np.meshgrid(t, t, t, indexing="ij")
        return X.ravel(), Y.ravel(), Z.ravel()

    def p1_nodes(self, level):
        """Coordinates of the P1 nodes in lattice order (i fastest)."""
        return self._grid(self.N(level))

    def lattice(self, level, fn_u, fn_p=None):
        """Plain lattice-order vector: u1, u2, u3 over the velocity lattice, then p."""
        N = self.N(level)
        u = fn_u(*self._grid(N if self.disc == hhg.HHG_P1P1 else 2 * N))
        X, Y, Z = self.p1_nodes(level)
        p = np.zeros(X.size) if fn_p is None else fn_p(X, Y, Z)
        return np.concatenate([u[0], u[1], u[2], p])

    def upload(self, level, arr, prec=hhg.HHG_F64):
        _, _, vw, _ = hhg.hhg_vec_layout(self.h, level)
        dt = self.torch.float64 if prec == hhg.HHG_F64 else self.torch.float32
        dst = self.torch.zeros(vw, dtype=dt, device=self.dev)
        src = self.torch.from_numpy(np.ascontiguousarray(arr, dtype=np.float64)).to(self.dev)
        hhg.hhg_vec_from_lattice(self.h, level, src, dst, prec)
        return dst

    def download(self, level, x, prec=hhg.HHG_F64):
        _, _, _, lw = hhg.hhg_vec_layout(self.h, level)
        out = self.torch.empty(lw, dtype=self.torch.float64, device=self.dev)
        hhg.hhg_vec_to_lattice(self.h, level, x, out, prec)
        return out.cpu().numpy()

    def zeros(self, level, prec=hhg.HHG_F64):
        _, _, vw, _ = hhg.hhg_vec_layout(self.h, level)
        dt = self.torch.float64 if prec == hhg.HHG_F64 else self.torch.float32
        return self.torch.zeros(vw, dtype=dt, device=self.dev)

    # ------------------------------------------------------------ problem data
    def set_viscosity(self, nu_fn, levels=None):
        """nu at the P1 nodes of every level (or the given ones)."""
        for l in (range(self.lmin, self.lmax + 1) if levels is None else levels):
            nu = nu_fn(*self.p1_nodes(l))
            hhg.hhg_set_viscosity(self.h, l, self.torch.from_numpy(np.ascontiguousarray(nu)).to(self.dev))
        self.has_nu = True

    def rhs(self, prob, prec=hhg.HHG_F64):
        """b_l = (M I(f), 0) on every level (right-hand sides of Alg. fmg)."""
        bs = []
        for l in range(self.lmin, self.lmax + 1):
            f = self.upload(l, self.lattice(l, prob.f), prec)
            b = self.torch.zeros_like(f)
            hhg.hhg_rhs(self.h, l, f, b, prec)
            bs.append(b)
        return bs

    def boundary(self, prob, level=None, prec=hhg.HHG_F64):
        """Finest-level vector holding u at every velocity DoF (the library
        uses only the boundary values as Dirichlet data) and zero pressure."""
        level = self.lmax if level is None else level
        return self.upload(level, self.lattice(level, prob.u), prec)
