"""Helpers for the GPU parity tests: move oracle-ordered (lattice order)
float64 vectors through the library's layout on the device."""
import numpy as np

from paper_2010_13513_amd import hhg


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


class Lib:
    """One context + hierarchy on cuda:0, on torch's current stream."""

    def __init__(self, disc, lmin, lmax, macro_refine=0, schur=hhg.HHG_SCHUR_SD, outflow=0, mesh=None):
        """mesh: optional (xyz, tets) macro mesh for hhg_mesh_create instead
        of the Kuhn cube (a non-Kuhn mesh gives the unstructured path, whose
        plain vector order is the oracle's node order)."""
        torch = torch_cuda()
        self.torch = torch
        self.dev = torch.device("cuda:0")
        stream = torch.cuda.current_stream(self.dev).cuda_stream
        self.ctx = hhg.hhg_ctx_create(0, stream)
        if mesh is not None:
            mesh = hhg.hhg_mesh_create(self.ctx, mesh[0], mesh[1])
        else:
            mesh = hhg.hhg_mesh_cube(self.ctx, macro_refine)
        try:
            if outflow:
                hhg.hhg_mesh_set_outflow(mesh, outflow)
            self.h = hhg.hhg_hier_create(mesh, disc, lmin, lmax, schur)
        finally:
            hhg.hhg_mesh_destroy(mesh)
        self.disc = disc

    def close(self):
        self.torch.cuda.synchronize()
        hhg.hhg_hier_destroy(self.h)
        hhg.hhg_ctx_destroy(self.ctx)

    def layout(self, level):
        return hhg.hhg_vec_layout(self.h, level)

    def empty(self, level, dtype=None):
        torch = self.torch
        _, _, vw, _ = self.layout(level)
        return torch.zeros(vw, dtype=dtype or torch.float64, device=self.dev)

    def from_lattice(self, level, arr, prec=hhg.HHG_F64):
        torch = self.torch
        src = torch.from_numpy(np.ascontiguousarray(arr, dtype=np.float64)).to(self.dev)
        dst = self.empty(level, torch.float64 if prec == hhg.HHG_F64 else torch.float32)
        hhg.hhg_vec_from_lattice(self.h, level, src, dst, prec)
        torch.cuda.synchronize()
        return dst

    def to_lattice(self, level, vec, prec=hhg.HHG_F64):
        torch = self.torch
        _, _, _, lw = self.layout(level)
        out = torch.empty(lw, dtype=torch.float64, device=self.dev)
        hhg.hhg_vec_to_lattice(self.h, level, vec, out, prec)
        torch.cuda.synchronize()
        return out.cpu().numpy()


def rel_err(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def block_errors(lib, level, got, want):
    """Largest error of the velocity block and of the pressure block of two
    lattice-order vectors, each relative to the largest entry of that block of
    `want` (the pressure is often much smaller than the velocity, so one
    scale for both would check it loosely).  A block of `want` that is
    exactly zero must be exactly zero in `got` (error 0 or inf)."""
    _, nn, _, lw = lib.layout(level)
    nv = lw - nn
    out = []
    for sl in (slice(0, nv), slice(nv, lw)):
        a, b = np.asarray(got[sl]), np.asarray(want[sl])
        s = np.abs(b).max() if b.size else 0.0
        if s == 0.0:
            out.append(0.0 if not np.any(a) else float("inf"))
        else:
            out.append(float(np.abs(a - b).max() / s))
    return tuple(out)


def assert_blocks(lib, level, got, want, tol, what=""):
    eu, ep = block_errors(lib, level, got, want)
    print(f"[parity] {what} level {level}: velocity {eu:.2e}, pressure {ep:.2e} (tol {tol:.0e})", flush=True)
    assert eu <= tol and ep <= tol, (what, eu, ep, tol)
    return eu, ep


def coarse_tolerance(vorder, N, nu_nodes=None, neumann=()):
    """Parity tolerance for results that pass through the coarsest-level
    solve.  Both sides apply a pseudo-inverse of the same dense coarse
    operator, each computed independently by a backward-stable decomposition
    in float64; two such solutions differ by up to about kappa * u relative
    (kappa = largest / smallest nonzero singular value of the coarse operator,
    u = 2^-53), and the cycles above carry that difference along.  Taylor-Hood
    on N = 2 has kappa ~ 3e4, so its bound (2 kappa 2^-52 ~ 1.3e-11) is looser
    than the 1e-12 of every other step."""
    from oracle import coarse as ocoarse, fe
    from oracle.stokes import Stokes
    cs = ocoarse.CoarseSolver(Stokes(fe.Level(N, vorder, nu_nodes, neumann)))
    kappa = float(cs.sv[0] / cs.sv[cs.rank - 1])
    return max(1e-12, 2.0 * kappa * 2.0 ** -52), kappa
