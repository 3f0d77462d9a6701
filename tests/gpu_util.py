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

    def __init__(self, disc, lmin, lmax, macro_refine=0, schur=hhg.HHG_SCHUR_SD):
        torch = torch_cuda()
        self.torch = torch
        self.dev = torch.device("cuda:0")
        stream = torch.cuda.current_stream(self.dev).cuda_stream
        self.ctx = hhg.hhg_ctx_create(0, stream)
        self.h = hhg.hhg_hier_create(self.ctx, disc, macro_refine, lmin, lmax, schur)
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
