"""The one-workgroup small-level V-cycle against the launch-per-phase form:
same arithmetic (sums in another order), so FMG solves, V-cycles and the
float32 defect correction agree to rounding."""
import numpy as np
import pytest

from oracle import mesh, multigrid as mg
from paper_2010_13513_amd import hhg, workloads as W
from tests.gpu_util import Lib, rel_err

pytestmark = pytest.mark.gpu

P1, P2 = hhg.HHG_P1P1, hhg.HHG_P2P1
NU = W.gaussian_bump_viscosity(W.SEED_BASE + 4000, N_ref=32)


def _set_nu(lib, lmin, L):
    for l in range(lmin, L + 1):
        c = mesh.p1_coords(2 ** l) / float(2 ** l)
        hhg.hhg_set_viscosity(lib.h, l, lib.torch.from_numpy(NU(c[:, 0], c[:, 1], c[:, 2])).to(lib.dev))


@pytest.mark.parametrize("disc,lmin,L", [(P1, 0, 4), (P2, 1, 4)])
@pytest.mark.parametrize("varnu", [False, True])
def test_fused_fmg_matches_unfused(disc, lmin, L, varnu):
    lib = Lib(disc, lmin, L)
    try:
        if varnu:
            _set_nu(lib, lmin, L)
        H = mg.Hierarchy(1 if disc == P1 else 2, lmin, L, schur="sd")
        prob = W.fourier_forcing(W.SEED_BASE + 2000)
        bs = [lib.from_lattice(l, H.rhs(l, prob)) for l in range(lmin, L + 1)]
        x0 = lib.from_lattice(L, H.initial(L, prob))
        prm = hhg.solver_params(1, 2, 1, 1, hhg.HHG_GS_FWD, 2, 2.3, extra_cycles=2)
        out = {}
        for fused in (0, 10 ** 9, 5000):
            hhg.hhg_hier_set_fused_sites(lib.h, fused)
            for rep in range(2):                        # captured graph: first call captures, second replays
                x = x0.clone()
                hhg.hhg_fmg_solve(lib.h, x, bs, prm, want_stats=False)
            out[fused] = lib.to_lattice(L, x)
        assert rel_err(out[10 ** 9], out[0]) < 1e-11
        assert rel_err(out[5000], out[0]) < 1e-11
    finally:
        lib.close()


@pytest.mark.parametrize("disc,lmin,L", [(P1, 0, 3), (P2, 1, 3)])
def test_fused_vcycle_and_float32_dc_match_unfused(disc, lmin, L):
    lib = Lib(disc, lmin, L)
    try:
        H = mg.Hierarchy(1 if disc == P1 else 2, lmin, L, schur="sd")
        prob = W.fourier_forcing(W.SEED_BASE + 2001)
        b = lib.from_lattice(L, H.rhs(L, prob))
        x0 = lib.from_lattice(L, H.initial(L, prob))
        prm = hhg.solver_params(3, 3, 0, 1, hhg.HHG_GS_SYM, 1, 2.3)
        res = {}
        for fused in (0, 10 ** 9):
            hhg.hhg_hier_set_fused_sites(lib.h, fused)
            x = x0.clone()
            for _ in range(3):
                hhg.hhg_vcycle(lib.h, L, x, b, prm)
            xd = x0.clone()
            st = hhg.hhg_dc_solve(lib.h, xd, b, prm, hhg.HHG_F32, 1, 1e-12, 200)
            res[fused] = (lib.to_lattice(L, x), lib.to_lattice(L, xd), st.cycles)
        assert rel_err(res[10 ** 9][0], res[0][0]) < 1e-11
        assert rel_err(res[10 ** 9][1], res[0][1]) < 1e-9
        assert abs(res[10 ** 9][2] - res[0][2]) <= 1
    finally:
        lib.close()
