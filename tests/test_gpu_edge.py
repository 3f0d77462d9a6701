"""Edge cases through the C ABI: the size and argument limits of the
hierarchy and of the calls (status codes, no work done), the largest
hierarchy the library accepts (P1-P1 on 48 macro-tets at N = 512) checked on
sampled operator rows against the oracle, and the degenerate all-zero
problem (zero forcing, zero boundary data), whose FMG result is exactly 0."""
import numpy as np
import pytest

from paper_2010_13513_amd import hhg
from tests.gpu_util import Lib, torch_cuda
from tests.test_gpu_fullsize import check_rows, sampled_rows

pytestmark = pytest.mark.gpu

P1, P2 = hhg.HHG_P1P1, hhg.HHG_P2P1


def _status(fn, *args):
    try:
        fn(*args)
    except hhg.HHGError as e:
        return e.status
    return hhg.HHG_OK


def test_hierarchy_limits():
    torch = torch_cuda()
    ctx = hhg.hhg_ctx_create(0, torch.cuda.current_stream().cuda_stream)
    try:
        bad = [
            (P2, 0, 1, 9),        # N = 512 > 256 for P2-P1
            (P1, 0, 1, 10),       # N = 1024 > 512 for P1-P1
            (P2, 1, 1, 8),        # N = 512 with one macro refinement
            (P1, 0, 3, 3),        # lmin == lmax
            (P1, 0, -1, 2),       # negative level
            (P2, 0, 0, 3),        # Taylor-Hood with N(lmin) = 1
            (P1, 2, 0, 3),        # macro_refine outside {0, 1}
            (7, 0, 0, 3),         # unknown discretisation
        ]
        meshes = {0: hhg.hhg_mesh_cube(ctx, 0), 1: hhg.hhg_mesh_cube(ctx, 1)}
        for disc, mr, lmin, lmax in bad:
            if mr not in meshes:
                assert _status(hhg.hhg_mesh_cube, ctx, mr) == hhg.HHG_ERR_ARG
                continue
            assert _status(hhg.hhg_hier_create, meshes[mr], disc, lmin, lmax) == hhg.HHG_ERR_ARG, (disc, mr, lmin, lmax)
        assert _status(hhg.hhg_hier_create, meshes[0], P1, 0, 3, 9) == hhg.HHG_ERR_ARG      # unknown Schur option
        assert _status(hhg.hhg_hier_create, None, P1, 0, 3) == hhg.HHG_ERR_ARG              # no mesh
        # the smallest valid hierarchies
        for disc, lmin in ((P1, 0), (P2, 1)):
            h = hhg.hhg_hier_create(meshes[0], disc, lmin, lmin + 1)
            assert hhg.hhg_vec_layout(h, lmin)[0] == 2 ** lmin
            hhg.hhg_hier_destroy(h)
        for m in meshes.values():
            hhg.hhg_mesh_destroy(m)
    finally:
        torch.cuda.synchronize()
        hhg.hhg_ctx_destroy(ctx)


def test_call_arguments_are_checked():
    lib = Lib(P2, 1, 3)
    torch = lib.torch
    try:
        x, b = lib.empty(3), lib.empty(3)
        xc = lib.empty(1)
        prm = hhg.solver_params(1, 1, 0, 1, hhg.HHG_GS_FWD, 1, 2.3)
        E = hhg.HHG_ERR_ARG
        assert _status(hhg.hhg_restrict, lib.h, 1, lib.empty(1), xc) == E             # no level below lmin
        assert _status(hhg.hhg_prolong_add, lib.h, 3, x, x) == E                     # no level above lmax
        assert _status(hhg.hhg_smooth, lib.h, 3, x, b, -1, hhg.HHG_GS_FWD, 1, 2.3) == E
        assert _status(hhg.hhg_smooth, lib.h, 3, x, b, 1, hhg.HHG_GS_FWD, 0, 2.3) == E
        assert _status(hhg.hhg_smooth, lib.h, 3, x, b, 1, 5, 1, 2.3) == E            # unknown Gauss-Seidel variant
        assert _status(hhg.hhg_residual, lib.h, 3, x, b, x) == E                     # output aliases an input
        assert _status(hhg.hhg_hier_set_bf16_levels, lib.h, 4) == E                  # more levels than exist
        assert _status(hhg.hhg_hier_set_bf16_levels, lib.h, -1) == E
        assert _status(hhg.hhg_hier_set_fused_sites, lib.h, -5) == E
        assert _status(hhg.hhg_vcycle, lib.h, 3, x, b, prm, 7) == hhg.HHG_ERR_PREC
        assert _status(hhg.hhg_dc_solve, lib.h, x, b, prm, hhg.HHG_F32, 0) == E      # no inner cycle
        bad = hhg.solver_params(1, 1, 0, 1, hhg.HHG_GS_FWD, 1, 0.0)                  # omega_inv <= 0
        assert _status(hhg.hhg_vcycle, lib.h, 3, x, b, bad) == E
        # nothing above touched the vectors
        torch.cuda.synchronize()
        assert float(x.abs().max()) == 0.0 and float(b.abs().max()) == 0.0
    finally:
        lib.close()


@pytest.mark.parametrize("disc,lmin,L", [(P1, 0, 4), (P2, 1, 4)])
def test_zero_problem_gives_zero(disc, lmin, L):
    lib = Lib(disc, lmin, L)
    try:
        bs = [lib.empty(l) for l in range(lmin, L + 1)]
        x = lib.empty(L)
        st = hhg.hhg_fmg_solve(lib.h, x, bs, hhg.solver_params(1, 1, 1, 1, hhg.HHG_GS_FWD, 2, 2.3, extra_cycles=2))
        lib.torch.cuda.synchronize()
        assert float(x.abs().max()) == 0.0
        assert st.res_u == 0.0 and st.res_p == 0.0
        xd = lib.empty(L)
        hhg.hhg_dc_solve(lib.h, xd, bs[-1], hhg.solver_params(2, 2, 0, 1, hhg.HHG_GS_FWD, 2, 2.3),
                         hhg.HHG_F32, 1, 1e-12, 5)
        lib.torch.cuda.synchronize()
        assert float(xd.abs().max()) == 0.0
    finally:
        lib.close()


def test_apply_largest_p1_hierarchy_sampled_rows():
    """P1-P1 on 48 macro-tets at level 8: N = 512, the largest lattice the
    library accepts (1.35e8 nodes, 5.4e8 words per vector)."""
    lib = Lib(P1, 7, 8, macro_refine=1)
    torch = lib.torch
    try:
        N, nn, vw, lw = lib.layout(8)
        assert N == 512
        print(f"apply at the largest size: P1-P1, N {N}, {vw} words", flush=True)
        gen = torch.Generator(device=lib.dev).manual_seed(13513 + 3002)
        lat = torch.randn(lw, generator=gen, dtype=torch.float64, device=lib.dev)
        x = torch.zeros(vw, dtype=torch.float64, device=lib.dev)
        hhg.hhg_vec_from_lattice(lib.h, 8, lat, x)
        y = torch.empty_like(x)
        hhg.hhg_apply(lib.h, 8, hhg.HHG_OP_FULL, x, y)
        del x
        ylat = torch.empty_like(lat)
        hhg.hhg_vec_to_lattice(lib.h, 8, y, ylat)
        del y
        torch.cuda.synchronize()
        rows, bnd = sampled_rows(1, N, np.random.default_rng(9), per_class=4)
        got = ylat.index_select(0, torch.tensor([r[0] for r in rows] + bnd, device=lib.dev)).cpu().numpy()
        xi = sorted({t[0] for r in rows for t in r[1]})
        xv = dict(zip(xi, lat.index_select(0, torch.tensor(xi, device=lib.dev)).cpu().numpy()))
        check_rows(rows, bnd, xv, got)
    finally:
        lib.close()


def _kuhn_mesh(N, rng=None):
    """The Kuhn partition of the unit cube into N^3 sub-cubes (6 N^3
    tetrahedra), optionally with shuffled vertex numbering, tetrahedron order
    and vertex order inside each tetrahedron."""
    n1 = N + 1
    pts = np.array([(i, j, k) for k in range(n1) for j in range(n1) for i in range(n1)], float) / N
    idx = lambda c: int(c[0] + n1 * (c[1] + n1 * c[2]))
    tets = []
    for k in range(N):
        for j in range(N):
            for i in range(N):
                for perm in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
                    c = [i, j, k]
                    t = [idx(c)]
                    for a in perm:
                        c[a] += 1
                        t.append(idx(c))
                    tets.append(t)
    tets = np.array(tets)
    if rng is not None:
        relabel = rng.permutation(len(pts))
        inv = np.argsort(relabel)
        pts = pts[inv]                  # new vertex v is old vertex inv[v]
        tets = relabel[tets]
        tets = tets[rng.permutation(len(tets))]
        tets = np.array([rng.permutation(t) for t in tets])
    return pts, tets


def test_mesh_handle():
    """hhg_mesh_cube and hhg_mesh_create: the Kuhn cube meshes in any vertex
    and tetrahedron order give the hierarchy of hhg_mesh_cube (the same
    operator on the same lattice); other valid tetrahedral meshes become
    unstructured meshes; invalid ones are refused with HHG_ERR_ARG (no
    hierarchy is built from them)."""
    torch = torch_cuda()
    ctx = hhg.hhg_ctx_create(0, torch.cuda.current_stream().cuda_stream)
    rng = np.random.default_rng(2024)
    try:
        for N, mr in ((1, 0), (2, 1)):
            ref = hhg.hhg_mesh_cube(ctx, mr)
            assert hhg.hhg_mesh_info(ref) == ((N + 1) ** 3, 6 * N ** 3, mr)
            xyz, tet = _kuhn_mesh(N, rng)
            m = hhg.hhg_mesh_create(ctx, xyz, tet)
            assert hhg.hhg_mesh_info(m) == ((N + 1) ** 3, 6 * N ** 3, mr)
            outs = []
            for mesh in (ref, m):
                h = hhg.hhg_hier_create(mesh, P2, 1, 2)
                hhg.hhg_mesh_destroy(mesh)          # the hierarchy keeps what it needs
                _, _, vw, lw = hhg.hhg_vec_layout(h, 2)
                src = torch.from_numpy(np.random.default_rng(5).standard_normal(lw)).cuda()
                x = torch.zeros(vw, dtype=torch.float64, device="cuda")
                y = torch.zeros_like(x)
                hhg.hhg_vec_from_lattice(h, 2, src, x)
                hhg.hhg_apply(h, 2, hhg.HHG_OP_FULL, x, y)
                torch.cuda.synchronize()
                outs.append(y.cpu())
                hhg.hhg_hier_destroy(h)
            assert torch.equal(outs[0], outs[1])
        E = hhg.HHG_ERR_ARG
        xyz, tet = _kuhn_mesh(2)
        # meshes that are no Kuhn partition of the unit cube but valid
        # tetrahedral meshes: the unstructured path (macro_refine -1)
        general = {
            "47 tetrahedra": (xyz, tet[:47]),
            "vertex off the lattice": (xyz + np.array([[0.0, 0.0, 0.1]] * len(xyz)) * (np.arange(len(xyz)) == 13)[:, None], tet),
            "outside the unit cube": (xyz * 2.0, tet),
        }
        for why, (x_, t_) in general.items():
            m = hhg.hhg_mesh_create(ctx, x_, t_)
            assert hhg.hhg_mesh_info(m)[2] == -1, why
            hhg.hhg_mesh_destroy(m)
        bad = {
            "folded: a vertex moved through a face": (np.vstack([xyz[:-1], xyz[:1]]), tet),
            "degenerate tetrahedron": (xyz, np.vstack([tet[:-1], [[0, 1, 2, 26]]])),
            "tetrahedron twice": (xyz, np.vstack([tet[:-1], tet[:1]])),
            "vertex index out of range": (xyz, np.vstack([tet[:-1], [[0, 1, 4, 27]]])),
            "unused vertex": (np.vstack([xyz, [[0.5, 0.5, 0.5]]]), tet),
        }
        for why, (x_, t_) in bad.items():
            assert _status(hhg.hhg_mesh_create, ctx, x_, t_) == E, why
            print(f"[mesh] refused ({why}): {hhg.hhg_last_error()}")
        assert _status(hhg.hhg_mesh_cube, ctx, 2) == E
        assert _status(hhg.hhg_mesh_info, None) == E
    finally:
        torch.cuda.synchronize()
        hhg.hhg_ctx_destroy(ctx)
