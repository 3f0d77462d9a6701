"""GPU parity of the unstructured-mesh path (Sec. 2, 2.1: HHG on any T_0)
against oracle/umesh.py, element by element on the same seeded inputs.

Meshes: the 24-tetrahedron cube (the partition of the cube benchmark), a
jittered 48-tetrahedron cube (no Kuhn partition: every cell has its own
geometry) and a 2 x 1 x 1 box of two 24-tetrahedron cubes (a domain that is
not the unit cube).  Vectors cross the boundary in the oracle's node order
(canonical order, see include/hhg.h), so no permutation is involved.

Tolerance: 1e-12 relative per velocity and pressure block (both sides sum
the same few products per row in different orders); results through the
coarsest-level solve max(1e-12, 2 kappa 2^-52) with kappa the condition
number of the dense coarse operator, as on the lattice path.

Full size (the cube benchmark's level 6, 1.07e6 nodes, 62-point interior
rows, and level 7, 8.5e6 nodes, rows of two 64-point segments): properties
the oracle fixes at any size -- interior rows annihilate linear velocities,
B of a linear velocity is -div u times the lumped mass, prolongation
reproduces linear fields, restriction is the transpose of prolongation, and
the FMG solve on levels 0..7 contracts the residual at a multigrid rate.
"""
import numpy as np
import pytest

from oracle import coarse as ocoarse, multigrid as mg, smoother as osm, umesh
from oracle.stokes import Stokes
from paper_2010_13513_amd import hhg, workloads as W
from tests.gpu_util import Lib, assert_blocks

pytestmark = pytest.mark.gpu

MESHES = {
    "cube24": W.cube24,
    "jittered": lambda: W.jittered_cube(W.SEED_BASE + 7000),
    "box2": lambda: W.box_cube24(2, 1, 1),
}
CASES = [("cube24", 0, 2), ("cube24", 0, 3), ("jittered", 0, 2), ("box2", 0, 2)]   # (mesh, lmin, level)


@pytest.fixture(scope="module")
def oracle_levels():
    cache = {}

    def get(name, level):
        key = (name, level)
        if key not in cache:
            xyz, tets = MESHES[name]()
            cache[key] = Stokes(umesh.ULevel(xyz, tets, level))
        return cache[key]
    return get


@pytest.fixture(scope="module")
def libs():
    cache = {}

    def get(name, lmin, lmax, schur=hhg.HHG_SCHUR_SD):
        key = (name, lmin, lmax, schur)
        if key not in cache:
            print(f"[umesh] hierarchy {name} {lmin}..{lmax}", flush=True)
            cache[key] = Lib(hhg.HHG_P1P1, lmin, lmax, schur=schur, mesh=MESHES[name]())
        return cache[key]
    yield get
    for lib in cache.values():
        lib.close()


def _rand(S, seed, zero_bnd=False):
    x = W.normal_vector(seed, S.n)
    return S.zero_boundary(x) if zero_bnd else x


def _coarse_tol(S0):
    cs = ocoarse.CoarseSolver(S0)
    kappa = float(cs.sv[0] / cs.sv[cs.rank - 1])
    return max(1e-12, 2.0 * kappa * 2.0 ** -52), cs


@pytest.mark.parametrize("name,lmin,L", CASES)
@pytest.mark.parametrize("op", ["FULL", "A", "BT", "B", "C", "MASS"])
def test_apply(libs, oracle_levels, name, lmin, L, op):
    lib = libs(name, lmin, L)
    S = oracle_levels(name, L)
    x = _rand(S, 300 + L)
    dy = lib.empty(L)
    code = {"FULL": hhg.HHG_OP_FULL, "A": hhg.HHG_OP_A, "BT": hhg.HHG_OP_BT, "B": hhg.HHG_OP_B, "C": hhg.HHG_OP_C,
            "MASS": hhg.HHG_OP_MASS}[op]
    hhg.hhg_apply(lib.h, L, code, lib.from_lattice(L, x), dy)
    want = S.apply(x) if op == "FULL" else S.apply_block(x, op)
    assert_blocks(lib, L, lib.to_lattice(L, dy), want, 1e-12, f"{name} apply {op}")


@pytest.mark.parametrize("name,lmin,L", CASES)
def test_residual_rhs_dots(libs, oracle_levels, name, lmin, L):
    lib = libs(name, lmin, L)
    S = oracle_levels(name, L)
    prob = W.paper_cube()
    b = S.rhs(prob.f)
    db = lib.empty(L)
    hhg.hhg_rhs(lib.h, L, lib.from_lattice(L, S.interpolate(prob.f)), db)
    assert_blocks(lib, L, lib.to_lattice(L, db), b, 1e-12, f"{name} rhs")
    x = _rand(S, 7)
    dx = lib.from_lattice(L, x)
    dr = lib.empty(L)
    hhg.hhg_residual(lib.h, L, dx, db, dr)
    assert_blocks(lib, L, lib.to_lattice(L, dr), S.residual(x, b), 1e-12, f"{name} residual")
    us, p = S.split(x)
    du, dp = hhg.hhg_dots(lib.h, L, dx, dx)
    assert abs(du - sum(u @ u for u in us)) <= 1e-12 * du and abs(dp - p @ p) <= 1e-12 * dp
    nu, np_ = hhg.hhg_norms(lib.h, L, dx)
    assert abs(nu * nu - du) <= 1e-12 * du and abs(np_ * np_ - dp) <= 1e-12 * dp
    hhg.hhg_project_mean_zero(lib.h, L, dx)
    assert_blocks(lib, L, lib.to_lattice(L, dx), S.mean_zero(x), 1e-12, f"{name} mean zero")


@pytest.mark.parametrize("name,lmin,L", CASES)
@pytest.mark.parametrize("gs,xi", [("f", 1), ("f", 3), ("s", 1)])
def test_smooth(libs, oracle_levels, name, lmin, L, gs, xi):
    lib = libs(name, lmin, L)
    S = oracle_levels(name, L)
    U = osm.Uzawa(S, "sd")
    x = _rand(S, 11)
    b = _rand(S, 12, zero_bnd=True)
    omega_inv = 2.0
    want = x
    for _ in range(2):
        want = U.iterate(want, b, gs, xi, 1.0 / omega_inv)
    dx = lib.from_lattice(L, x)
    hhg.hhg_smooth(lib.h, L, dx, lib.from_lattice(L, b), 2, hhg.HHG_GS_FWD if gs == "f" else hhg.HHG_GS_SYM, xi,
                   omega_inv)
    assert_blocks(lib, L, lib.to_lattice(L, dx), want, 1e-12, f"{name} smooth {gs}{xi}")


@pytest.mark.parametrize("name,lmin,L", [("cube24", 0, 3), ("jittered", 0, 2), ("box2", 0, 2)])
def test_smooth_one_workgroup(oracle_levels, name, lmin, L):
    """A smoothing call run by one workgroup (hhg_hier_set_fused_sites above
    the level's slots) computes every value as the per-colour launches do:
    the two agree to rounding (the same per-node arithmetic), and both with
    the oracle."""
    lib = Lib(hhg.HHG_P1P1, lmin, L, mesh=MESHES[name]())     # own hierarchy: the bound is changed below
    try:
        S = oracle_levels(name, L)
        U = osm.Uzawa(S, "sd")
        x = _rand(S, 21)
        bl = _rand(S, 22, zero_bnd=True)
        b = lib.from_lattice(L, bl)
        for gs, xi in (("f", 1), ("s", 2)):
            mode = hhg.HHG_GS_FWD if gs == "f" else hhg.HHG_GS_SYM
            out = []
            for fused in (0, 10 ** 9):
                hhg.hhg_hier_set_fused_sites(lib.h, fused)
                dx = lib.from_lattice(L, x)
                hhg.hhg_smooth(lib.h, L, dx, b, 3, mode, xi, 2.0)
                out.append(dx)
            diff = float((out[0] - out[1]).abs().max() / out[0].abs().max())
            assert diff <= 1e-14, f"{name} {gs}{xi}: one workgroup vs launches {diff:.2e}"
            want = x
            for _ in range(3):
                want = U.iterate(want, bl, gs, xi, 0.5)
            assert_blocks(lib, L, lib.to_lattice(L, out[1]), want, 1e-12, f"{name} one-workgroup smooth {gs}{xi}")
    finally:
        lib.close()


def test_smooth_ml_schur(oracle_levels):
    lib = Lib(hhg.HHG_P1P1, 0, 2, schur=hhg.HHG_SCHUR_ML, mesh=MESHES["jittered"]())
    try:
        S = oracle_levels("jittered", 2)
        U = osm.Uzawa(S, "ml")
        x, b = _rand(S, 31), _rand(S, 32, zero_bnd=True)
        want = U.iterate(U.iterate(x, b, "f", 2, 0.5), b, "f", 2, 0.5)
        dx = lib.from_lattice(2, x)
        hhg.hhg_smooth(lib.h, 2, dx, lib.from_lattice(2, b), 2, hhg.HHG_GS_FWD, 2, 2.0)
        assert_blocks(lib, 2, lib.to_lattice(2, dx), want, 1e-12, "jittered smooth ML")
    finally:
        lib.close()


@pytest.mark.parametrize("name,lmin,L", CASES)
def test_transfers(libs, oracle_levels, name, lmin, L):
    lib = libs(name, lmin, L)
    Sc, Sf = oracle_levels(name, L - 1), oracle_levels(name, L)
    T = umesh.UTransfer(Sc, Sf)
    rf = _rand(Sf, 21)
    drc = lib.empty(L - 1)
    hhg.hhg_restrict(lib.h, L, lib.from_lattice(L, rf), drc)
    assert_blocks(lib, L - 1, lib.to_lattice(L - 1, drc), T.restrict(rf), 1e-12, f"{name} restrict")
    xc, xf = _rand(Sc, 22), _rand(Sf, 23)
    dxf = lib.from_lattice(L, xf)
    hhg.hhg_prolong_add(lib.h, L - 1, lib.from_lattice(L - 1, xc), dxf)
    assert_blocks(lib, L, lib.to_lattice(L, dxf), xf + T.prolong(xc), 1e-12, f"{name} prolong_add")


@pytest.mark.parametrize("name", ["cube24", "jittered", "box2"])
def test_coarse_solve(libs, oracle_levels, name):
    lib = libs(name, 0, 2)
    S0 = oracle_levels(name, 0)
    tol, cs = _coarse_tol(S0)
    x, b = _rand(S0, 41), _rand(S0, 42, zero_bnd=True)
    dx = lib.from_lattice(0, x)
    hhg.hhg_coarse_solve(lib.h, dx, lib.from_lattice(0, b))
    assert_blocks(lib, 0, lib.to_lattice(0, dx), cs.solve(x, b), tol, f"{name} coarse solve")


@pytest.mark.parametrize("name,L", [("cube24", 3), ("jittered", 2), ("box2", 2)])
def test_fmg_and_vcycle(libs, name, L):
    xyz, tets = MESHES[name]()
    H = umesh.hierarchy(xyz, tets, 0, L, schur="sd")
    tol, _ = _coarse_tol(H.S[0])
    lib = libs(name, 0, L)
    prob = W.sine_cube()
    prm = mg.Params(2, 2, 1, 1, "f", 2, 2.0)
    want = H.fmg(prob, prm, cycles_on_finest=1)
    bs = [lib.from_lattice(l, H.rhs(l, prob)) for l in range(0, L + 1)]
    dx = lib.from_lattice(L, H.initial(L, prob))
    st = hhg.hhg_fmg_solve(lib.h, dx, bs, hhg.solver_params(2, 2, 1, 1, hhg.HHG_GS_FWD, 2, 2.0, extra_cycles=1))
    assert st.cycles == 2
    assert_blocks(lib, L, lib.to_lattice(L, dx), want, tol, f"{name} FMG")
    # one more V-cycle from that iterate, then the pressure mean
    want2 = H.S[L].mean_zero(H.vcycle(L, L, want, H.rhs(L, prob), prm))
    hhg.hhg_vcycle(lib.h, L, dx, bs[L], hhg.solver_params(2, 2, 1, 1, hhg.HHG_GS_FWD, 2, 2.0))
    hhg.hhg_project_mean_zero(lib.h, L, dx)
    assert_blocks(lib, L, lib.to_lattice(L, dx), want2, tol, f"{name} V-cycle")


def test_fmg_reproduces_linear_solution(libs):
    """u = (y, z, x), p = 0 solves the discrete system exactly on any mesh."""
    lib = libs("jittered", 0, 2)
    xyz, tets = MESHES["jittered"]()
    prob = W.linear_exact()
    S = {l: Stokes(umesh.ULevel(xyz, tets, l)) for l in range(3)}
    bs = [lib.from_lattice(l, S[l].rhs(prob.f)) for l in range(3)]
    dx = lib.from_lattice(2, S[2].set_boundary(S[2].zeros(), S[2].interpolate(prob.u, prob.p)))
    hhg.hhg_fmg_solve(lib.h, dx, bs, hhg.solver_params(2, 2, 0, 1, hhg.HHG_GS_FWD, 1, 2.0, extra_cycles=30))
    got = lib.to_lattice(2, dx)
    want = S[2].interpolate(prob.u, prob.p)
    assert np.abs(got - want).max() < 1e-10


def test_estimate_omega(libs, oracle_levels):
    lib = libs("cube24", 0, 3)
    S = oracle_levels("cube24", 3)
    U = osm.Uzawa(S, "sd")
    v0 = W.normal_vector(51, S.np_)
    want = U.estimate_omega_inv(v0, iters=20)
    torch = lib.torch
    got = hhg.hhg_estimate_omega(lib.h, 3, torch.from_numpy(v0).to(lib.dev), 20)
    assert abs(got - want) <= 1e-12 * want, (got, want)


def test_refusals(libs):
    lib = libs("cube24", 0, 2)
    torch = lib.torch
    x32 = torch.zeros(lib.layout(2)[2], dtype=torch.float32, device=lib.dev)
    with pytest.raises(hhg.HHGError) as e:
        hhg.hhg_apply(lib.h, 2, hhg.HHG_OP_FULL, x32, torch.zeros_like(x32), hhg.HHG_F32)
    assert e.value.status == hhg.HHG_ERR_PREC
    with pytest.raises(hhg.HHGError) as e:
        hhg.hhg_hier_set_bf16_levels(lib.h, 1)
    assert e.value.status == hhg.HHG_ERR_STATE
    ctx = lib.ctx
    mesh = hhg.hhg_mesh_create(ctx, *W.cube24())
    try:
        assert hhg.hhg_mesh_info(mesh)[2] == -1
        with pytest.raises(hhg.HHGError):
            hhg.hhg_hier_create(mesh, hhg.HHG_P2P1, 0, 2)
        with pytest.raises(hhg.HHGError) as e:
            hhg.hhg_mesh_set_outflow(mesh, 63)                          # no Dirichlet face left
        assert e.value.status == hhg.HHG_ERR_ARG
        hhg.hhg_mesh_set_outflow(mesh, 1)                               # the x = 0 plane's triangles
        hhg.hhg_mesh_set_outflow(mesh, 0)
    finally:
        hhg.hhg_mesh_destroy(mesh)


# ------------------------------------------------------- k-marching rows
# One jittered tetrahedron (not a Kuhn simplex) at level 6: n = 64, so its
# interior rows run the k-marching kernel (levels with n >= 64), compared
# with the oracle on all 47,905 nodes (the oracle builds it in about 30 s).
ONE_TET = (np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.9, 1.1, 0.05], [1.05, 0.95, 1.2]]), np.array([[0, 1, 2, 3]]))


@pytest.fixture(scope="module")
def one_tet():
    print("[umesh] one tetrahedron, level 6: oracle operator", flush=True)
    S = Stokes(umesh.ULevel(*ONE_TET, 6))
    lib = Lib(hhg.HHG_P1P1, 5, 6, mesh=ONE_TET)
    yield lib, S
    lib.close()


@pytest.mark.parametrize("op", ["FULL", "A", "BT", "B", "C"])
def test_k_marching_rows(one_tet, op):
    lib, S = one_tet
    x = _rand(S, 900)
    dy = lib.empty(6)
    code = {"FULL": hhg.HHG_OP_FULL, "A": hhg.HHG_OP_A, "BT": hhg.HHG_OP_BT, "B": hhg.HHG_OP_B, "C": hhg.HHG_OP_C}[op]
    hhg.hhg_apply(lib.h, 6, code, lib.from_lattice(6, x), dy)
    want = S.apply(x) if op == "FULL" else S.apply_block(x, op)
    assert_blocks(lib, 6, lib.to_lattice(6, dy), want, 1e-12, f"one tet level 6 apply {op}")


def test_k_marching_residual(one_tet):
    lib, S = one_tet
    x = _rand(S, 901)
    b = _rand(S, 902, zero_bnd=True)
    dr = lib.empty(6)
    hhg.hhg_residual(lib.h, 6, lib.from_lattice(6, x), lib.from_lattice(6, b), dr)
    assert_blocks(lib, 6, lib.to_lattice(6, dr), S.residual(x, b), 1e-12, "one tet level 6 residual")


# ---------------------------------------------------------------- full size
@pytest.fixture(scope="module")
def big():
    """The cube benchmark's mesh at levels 0..7 (level 6: 1.07e6 nodes)."""
    print("[umesh] cube24 levels 0..7", flush=True)
    lib = Lib(hhg.HHG_P1P1, 0, 7, mesh=W.cube24())
    yield lib
    lib.close()


def _positions(L):
    return hhg.hhg_query_umesh(*W.cube24(), L)["pos"]


def test_full_size_linear_rows(big):
    """Level 6: interior velocity rows of A vanish on linear fields (Dirichlet
    rows are zero by definition), B u = -div(u) m with m = M 1 the lumped mass,
    C 1 = 0."""
    lib, L = big, 6
    pos = _positions(L)
    n = pos.shape[0]
    G = np.array([[0.3, -1.0, 0.7], [2.0, 0.1, -0.4], [-0.6, 0.9, 0.2]])   # u = G x + c
    u = pos @ G.T + np.array([0.1, -0.2, 0.3])
    x = np.concatenate([u[:, 0], u[:, 1], u[:, 2], np.ones(n)])
    dx = lib.from_lattice(L, x)
    dy = lib.empty(L)
    hhg.hhg_apply(lib.h, L, hhg.HHG_OP_A, dx, dy)
    ya = lib.to_lattice(L, dy)
    assert np.abs(ya[:3 * n]).max() <= 1e-12 * np.abs(u).max()
    hhg.hhg_apply(lib.h, L, hhg.HHG_OP_MASS, lib.from_lattice(L, np.ones(4 * n)), dy)
    m = lib.to_lattice(L, dy)[3 * n:]
    assert abs(m.sum() - 1.0) < 1e-12
    hhg.hhg_apply(lib.h, L, hhg.HHG_OP_B, dx, dy)
    yb = lib.to_lattice(L, dy)[3 * n:]
    assert np.abs(yb + np.trace(G) * m).max() <= 1e-12 * np.abs(np.trace(G) * m).max()
    hhg.hhg_apply(lib.h, L, hhg.HHG_OP_C, dx, dy)
    assert np.abs(lib.to_lattice(L, dy)[3 * n:]).max() <= 1e-12 * m.max()


def test_full_size_transfers(big):
    """Levels 6 -> 7: prolongation reproduces linear fields; restriction is
    its transpose on vectors with zero Dirichlet velocity rows (and coarse
    pressure of zero sum, which the compatibility shift leaves alone)."""
    lib = big
    torch = lib.torch
    pc = _positions(6)
    nc = pc.shape[0]
    w = np.array([0.4, -1.3, 2.2])
    xc = np.concatenate([pc @ w + 0.5] * 4)
    _, nnf, _, lwf = lib.layout(7)
    dxf = lib.empty(7)
    hhg.hhg_prolong_add(lib.h, 6, lib.from_lattice(6, xc), dxf)
    xf = lib.to_lattice(7, dxf)
    # fine positions from the prolongation of the coordinate fields
    fine_pos = []
    for d in range(3):
        dxf.zero_()
        hhg.hhg_prolong_add(lib.h, 6, lib.from_lattice(6, np.concatenate([pc[:, d]] * 4)), dxf)
        fine_pos.append(lib.to_lattice(7, dxf)[:nnf])
    fine_pos = np.stack(fine_pos, axis=1)
    assert np.abs(xf[:nnf] - (fine_pos @ w + 0.5)).max() <= 1e-13
    on_bnd = lambda P: np.any((np.abs(P) < 1e-12) | (np.abs(P - 1) < 1e-12), axis=1)
    bf, bc = on_bnd(fine_pos), on_bnd(pc)
    rf = W.normal_vector(61, lwf)
    for d in range(3):
        rf[d * nnf:(d + 1) * nnf][bf] = 0.0
    yc = W.normal_vector(62, 4 * nc)
    for d in range(3):
        yc[d * nc:(d + 1) * nc][bc] = 0.0
    yc[3 * nc:] -= yc[3 * nc:].mean()
    drc = lib.empty(6)
    hhg.hhg_restrict(lib.h, 7, lib.from_lattice(7, rf), drc)
    rc = lib.to_lattice(6, drc)
    dpf = lib.empty(7)
    hhg.hhg_prolong_add(lib.h, 6, lib.from_lattice(6, yc), dpf)
    pf = lib.to_lattice(7, dpf)
    lhs, rhs = rc @ yc, rf @ pf
    assert abs(lhs - rhs) <= 1e-11 * np.sqrt((rc @ rc) * (yc @ yc)), (lhs, rhs)
    del torch


def _fine_positions(lib, pc, lf):
    """Node positions of level lf from those of level lf - 1 (prolongation
    reproduces the coordinate fields, test_full_size_transfers)."""
    _, nnf, _, _ = lib.layout(lf)
    out = []
    d_f = lib.empty(lf)
    for d in range(3):
        d_f.zero_()
        hhg.hhg_prolong_add(lib.h, lf - 1, lib.from_lattice(lf - 1, np.concatenate([pc[:, d]] * 4)), d_f)
        out.append(lib.to_lattice(lf, d_f)[:nnf])
    return np.stack(out, axis=1)


def test_full_size_fmg_converges(big):
    """Levels 0..7 (level 7: 8.5e6 nodes, rows of two 64-point segments) on
    the paper's cube solution: FMG(3,3,0,1,A_s,1) followed by V-cycles to a
    relative residual of 1e-8, at a rate of at most 0.6 per cycle.  (The
    symmetric sweep: with one forward sweep the inexact Uzawa cycle on this
    mesh slows down from level 5 on -- rates 0.8 at level 5, 1.0 at level 6
    -- in the oracle and here alike up to level 4 where both were compared;
    the symmetric sweep gives A_hat >= A, the condition under which the
    inexact Uzawa iteration is known to converge.)"""
    lib = big
    torch = lib.torch
    prob = W.paper_cube()
    pos = {l: _positions(l) for l in range(7)}
    pos[7] = _fine_positions(lib, pos[6], 7)
    bs = []
    for l in range(8):
        P = pos[l]
        f = prob.f(P[:, 0], P[:, 1], P[:, 2])
        db = lib.empty(l)
        hhg.hhg_rhs(lib.h, l, lib.from_lattice(l, np.concatenate([f[0], f[1], f[2], np.zeros(P.shape[0])])), db)
        bs.append(db)
    P = pos[7]
    u = prob.u(P[:, 0], P[:, 1], P[:, 2])
    dx = lib.from_lattice(7, np.concatenate([u[0], u[1], u[2], np.zeros(P.shape[0])]))
    v0 = torch.from_numpy(W.normal_vector(71, pos[7].shape[0])).to(lib.dev)
    omega_inv = hhg.hhg_estimate_omega(lib.h, 7, v0, 100)
    print(f"[umesh] omega_inv (level 7, 100 power iterations) {omega_inv:.6f}", flush=True)
    st = hhg.hhg_fmg_solve(lib.h, dx, bs, hhg.solver_params(3, 3, 0, 1, hhg.HHG_GS_SYM, 1, omega_inv, rtol=1e-8,
                                                           max_cycles=60))
    rate = (st.rel_res / 1e-1) ** (1.0 / max(st.cycles - 1, 1))
    print(f"[umesh] level 7 FMG: {st.cycles} cycles, rel res {st.rel_res:.2e}, mean rate {rate:.3f}", flush=True)
    assert st.rel_res <= 1e-8 and rate <= 0.6


# ------------------------------------------------------------ outflow faces
@pytest.fixture(scope="module")
def outflow_case():
    """24-tetrahedron cube with the outflow face x = 1 (bit 1), levels 0..3,
    and the oracle hierarchy of the same problem."""
    xyz, tets = W.cube24()
    of = W.boundary_faces_on_planes(xyz, tets, (1,))
    lib = Lib(hhg.HHG_P1P1, 0, 3, mesh=(xyz, tets), outflow=2)
    H = umesh.hierarchy(xyz, tets, 0, 3, schur="sd", outflow=of)
    yield lib, H
    lib.close()


def test_outflow_operators(outflow_case):
    lib, H = outflow_case
    L = 3
    S = H.S[L]
    x = _rand(S, 81)
    dy = lib.empty(L)
    hhg.hhg_apply(lib.h, L, hhg.HHG_OP_FULL, lib.from_lattice(L, x), dy)
    assert_blocks(lib, L, lib.to_lattice(L, dy), S.apply(x), 1e-12, "outflow apply")
    b = _rand(S, 82, zero_bnd=True)
    want = H.U[L].iterate(H.U[L].iterate(x, b, "s", 1, 0.5), b, "s", 1, 0.5)
    dx = lib.from_lattice(L, x)
    hhg.hhg_smooth(lib.h, L, dx, lib.from_lattice(L, b), 2, hhg.HHG_GS_SYM, 1, 2.0)
    assert_blocks(lib, L, lib.to_lattice(L, dx), want, 1e-12, "outflow smooth")
    rf = _rand(S, 83)
    drc = lib.empty(L - 1)
    hhg.hhg_restrict(lib.h, L, lib.from_lattice(L, rf), drc)
    assert_blocks(lib, L - 1, lib.to_lattice(L - 1, drc), H.T[L].restrict(rf), 1e-12, "outflow restrict")
    tol, cs = _coarse_tol(H.S[0])
    x0, b0 = _rand(H.S[0], 84), _rand(H.S[0], 85, zero_bnd=True)
    dx0 = lib.from_lattice(0, x0)
    hhg.hhg_coarse_solve(lib.h, dx0, lib.from_lattice(0, b0))
    assert_blocks(lib, 0, lib.to_lattice(0, dx0), cs.solve(x0, b0), tol, "outflow coarse solve")


def test_outflow_fmg(outflow_case):
    """FMG on the smooth outflow solution matches the oracle; the P1 outflow
    polynomial u = (x, -y, 0), p = 1 is reproduced."""
    lib, H = outflow_case
    L = 3
    tol, _ = _coarse_tol(H.S[0])
    for prob, extra in ((W.outflow_cube(), 1), (W.outflow_polynomial(1), 30)):
        prm = mg.Params(2, 2, 0, 1, "s", 1, 2.3)
        want = H.fmg(prob, prm, cycles_on_finest=extra)
        bs = [lib.from_lattice(l, H.rhs(l, prob)) for l in range(0, L + 1)]
        dx = lib.from_lattice(L, H.initial(L, prob))
        hhg.hhg_fmg_solve(lib.h, dx, bs, hhg.solver_params(2, 2, 0, 1, hhg.HHG_GS_SYM, 1, 2.3, extra_cycles=extra))
        got = lib.to_lattice(L, dx)
        assert_blocks(lib, L, got, want, tol, f"outflow FMG {prob.name}")
        if prob.name.startswith("outflow_polynomial"):
            assert np.abs(got - H.S[L].interpolate(prob.u, prob.p)).max() < 1e-8


def test_outflow_face_refusals(libs):
    lib = libs("box2", 0, 2)
    ctx = lib.ctx
    xyz, tets = W.cube24()
    mesh = hhg.hhg_mesh_create(ctx, xyz, tets)
    try:
        with pytest.raises(hhg.HHGError):
            hhg.hhg_mesh_set_outflow_faces(mesh, [[0, 1, 14]])          # not a boundary face
        every = W.boundary_faces_on_planes(xyz, tets, range(6))
        with pytest.raises(hhg.HHGError):
            hhg.hhg_mesh_set_outflow_faces(mesh, every)                 # no Dirichlet face left
        hhg.hhg_mesh_set_outflow_faces(mesh, W.boundary_faces_on_planes(xyz, tets, (1,)))
    finally:
        hhg.hhg_mesh_destroy(mesh)
    cube = hhg.hhg_mesh_cube(ctx, 0)
    try:
        with pytest.raises(hhg.HHGError):
            hhg.hhg_mesh_set_outflow_faces(cube, [[0, 1, 3]])           # Kuhn meshes: hhg_mesh_set_outflow
    finally:
        hhg.hhg_mesh_destroy(cube)
