"""GPU parity: every library call against the float64 oracle on the same
seeded inputs (element by element).

Tolerance (float64): 1e-12 relative, velocity and pressure blocks each
scaled by their own largest entry, for single operator applications and
transfers (both sides sum the same O(10-100) products in a different order: a
few ulp of the largest term) and for multi-step results alike (smoothing,
cycles, whole solves: each step adds a few ulp and the iteration contracts
what earlier steps left).  Results that pass through the coarsest-level solve
are held to max(1e-12, 2 kappa 2^-52), kappa the condition number of the
dense coarse operator (tests.gpu_util.coarse_tolerance): two independently
computed float64 pseudo-inverses of it differ by that much.  Sizes span several 256-thread blocks with ragged
tails (nn = 9^3, 17^3, 33^3).  Both Schur diagonals of eq. uzawa-pressure are
covered: SD (the library default) and ML (the lumped mass of eq.
omega-eigenvalue-problem).
"""
import numpy as np
import pytest

from oracle import coarse as ocoarse, fe, multigrid as mg, smoother as osm
from oracle.stokes import Stokes
from oracle.transfer import Transfer
from paper_2010_13513_amd import hhg, workloads as W
from tests.gpu_util import Lib, assert_blocks, coarse_tolerance, rel_err

pytestmark = pytest.mark.gpu

P1, P2 = hhg.HHG_P1P1, hhg.HHG_P2P1
CASES = [(P1, 0, 3), (P1, 0, 4), (P2, 1, 3), (P2, 1, 4)]   # (disc, lmin, level)


def _vorder(disc):
    return 1 if disc == P1 else 2


def _rand(S, seed, zero_bnd=False):
    x = W.normal_vector(seed, S.n)
    return S.zero_boundary(x) if zero_bnd else x


@pytest.fixture(scope="module")
def libs():
    cache = {}

    def get(disc, lmin, lmax, mr=0, schur=hhg.HHG_SCHUR_SD):
        key = (disc, lmin, lmax, mr, schur)
        if key not in cache:
            cache[key] = Lib(disc, lmin, lmax, mr, schur)
        return cache[key]
    yield get
    for lib in cache.values():
        lib.close()


@pytest.mark.parametrize("disc,lmin,L", CASES)
@pytest.mark.parametrize("op", ["FULL", "A", "BT", "B", "C"])
def test_apply(libs, disc, lmin, L, op):
    lib = libs(disc, lmin, L)
    S = Stokes(fe.Level(2 ** L, _vorder(disc)))
    x = _rand(S, 100 + L)
    dx = lib.from_lattice(L, x)
    dy = lib.empty(L)
    code = {"FULL": hhg.HHG_OP_FULL, "A": hhg.HHG_OP_A, "BT": hhg.HHG_OP_BT, "B": hhg.HHG_OP_B, "C": hhg.HHG_OP_C}[op]
    hhg.hhg_apply(lib.h, L, code, dx, dy)
    got = lib.to_lattice(L, dy)
    want = S.apply(x) if op == "FULL" else S.apply_block(x, op)
    assert_blocks(lib, L, got, want, 1e-12, f"apply {op}")


@pytest.mark.parametrize("disc,lmin,L", CASES)
def test_residual_and_rhs(libs, disc, lmin, L):
    lib = libs(disc, lmin, L)
    S = Stokes(fe.Level(2 ** L, _vorder(disc)))
    prob = W.paper_cube()
    b = S.rhs(prob.f)
    fnod = S.interpolate(prob.f)         # nodal f in the velocity part
    db = lib.empty(L)
    hhg.hhg_rhs(lib.h, L, lib.from_lattice(L, fnod), db)
    assert_blocks(lib, L, lib.to_lattice(L, db), b, 1e-12, "rhs")
    x = _rand(S, 7)
    dr = lib.empty(L)
    hhg.hhg_residual(lib.h, L, lib.from_lattice(L, x), db, dr)
    assert_blocks(lib, L, lib.to_lattice(L, dr), S.residual(x, b), 1e-12, "residual")


@pytest.mark.parametrize("disc,lmin,L", CASES)
@pytest.mark.parametrize("gs,xi", [("f", 1), ("f", 3), ("s", 1)])
def test_smooth(libs, disc, lmin, L, gs, xi):
    lib = libs(disc, lmin, L)
    S = Stokes(fe.Level(2 ** L, _vorder(disc)))
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
    assert_blocks(lib, L, lib.to_lattice(L, dx), want, 1e-12, f"smooth {gs}{xi}")


@pytest.mark.parametrize("disc,lmin,L", CASES)
def test_transfers(libs, disc, lmin, L):
    lib = libs(disc, lmin, L)
    vo = _vorder(disc)
    Sc, Sf = Stokes(fe.Level(2 ** (L - 1), vo)), Stokes(fe.Level(2 ** L, vo))
    T = Transfer(Sc, Sf)
    rf = _rand(Sf, 21)
    drc = lib.empty(L - 1)
    hhg.hhg_restrict(lib.h, L, lib.from_lattice(L, rf), drc)
    assert_blocks(lib, L - 1, lib.to_lattice(L - 1, drc), T.restrict(rf), 1e-12, "restrict")
    xc = _rand(Sc, 22)
    xf = _rand(Sf, 23)
    dxf = lib.from_lattice(L, xf)
    hhg.hhg_prolong_add(lib.h, L - 1, lib.from_lattice(L - 1, xc), dxf)
    assert_blocks(lib, L, lib.to_lattice(L, dxf), xf + T.prolong(xc), 1e-12, "prolong_add")


@pytest.mark.parametrize("disc,lmin,L", [(P1, 0, 1), (P1, 2, 3), (P2, 1, 2)])
def test_coarse_solve(libs, disc, lmin, L):
    lib = libs(disc, lmin, L)
    S = Stokes(fe.Level(2 ** lmin, _vorder(disc)))
    cs = ocoarse.CoarseSolver(S)
    x = _rand(S, 31)
    b = _rand(S, 32, zero_bnd=True)
    us, p = S.split(b)
    b = S.join(us, p - p.mean())
    dx = lib.from_lattice(lmin, x)
    hhg.hhg_coarse_solve(lib.h, dx, lib.from_lattice(lmin, b))
    tol, kappa = coarse_tolerance(_vorder(disc), 2 ** lmin)
    assert_blocks(lib, lmin, lib.to_lattice(lmin, dx), cs.solve(x, b), tol, f"coarse solve (kappa {kappa:.1e})")


@pytest.mark.parametrize("disc,lmin,L", [(P1, 0, 3), (P2, 1, 3)])
def test_omega_estimate(libs, disc, lmin, L):
    lib = libs(disc, lmin, L)
    S = Stokes(fe.Level(2 ** L, _vorder(disc)))
    U = osm.Uzawa(S, "sd")
    v0 = W.normal_vector(41, S.np_)
    want = U.estimate_omega_inv(v0, 50)
    torch = lib.torch
    got = hhg.hhg_estimate_omega(lib.h, L, torch.from_numpy(v0).to(lib.dev), 50)
    print(f"[parity] SD omega_inv {got:.12f} oracle {want:.12f}")
    assert abs(got - want) <= 1e-12 * want


@pytest.mark.parametrize("disc,lmin,L", [(P1, 0, 3), (P2, 1, 3)])
def test_vcycle(libs, disc, lmin, L):
    lib = libs(disc, lmin, L)
    H = mg.Hierarchy(_vorder(disc), lmin, L, schur="sd")
    prob = W.sine_cube()
    b = H.rhs(L, prob)
    x = H.initial(L, prob)
    prm = mg.Params(2, 1, 1, 1, "f", 2, 2.3)
    want = H.vcycle(L, L, x, b, prm)
    dx = lib.from_lattice(L, x)
    hhg.hhg_vcycle(lib.h, L, dx, lib.from_lattice(L, b), hhg.solver_params(2, 1, 1, 1, hhg.HHG_GS_FWD, 2, 2.3))
    tol, kappa = coarse_tolerance(_vorder(disc), 2 ** lmin)
    assert_blocks(lib, L, lib.to_lattice(L, dx), want, tol, f"V-cycle (coarse kappa {kappa:.1e})")


def _fmg_gpu(lib, H, prob, L, prm_o, prm_c):
    bs = [lib.from_lattice(l, H.rhs(l, prob)) for l in range(H.Lmin, L + 1)]
    x0 = H.initial(L, prob)
    dx = lib.from_lattice(L, x0)
    st = hhg.hhg_fmg_solve(lib.h, dx, bs, prm_c)
    return lib.to_lattice(L, dx), st


@pytest.mark.parametrize("disc,lmin,L,s", [
    (P1, 0, 3, (3, 3, 0, 1, "f", 1)),        # V(3,3): the c1 workload
    (P1, 0, 4, (2, 3, 2, 1, "s", 1)),
    (P2, 1, 3, (0, 2, 1, 1, "f", 3)),
    (P2, 1, 4, (1, 3, 2, 1, "f", 3))])
def test_fmg(libs, disc, lmin, L, s):
    lib = libs(disc, lmin, L)
    H = mg.Hierarchy(_vorder(disc), lmin, L, schur="sd")
    prob = W.sine_cube() if disc == P1 else W.paper_cube()
    om = 2.3
    prm = mg.Params(*s, omega_inv=om)
    want = H.fmg(prob, prm, cycles_on_finest=1)
    got, st = _fmg_gpu(lib, H, prob, L, prm,
                       hhg.solver_params(s[0], s[1], s[2], s[3], hhg.HHG_GS_FWD if s[4] == "f" else hhg.HHG_GS_SYM,
                                         s[5], om, extra_cycles=1))
    tol, kappa = coarse_tolerance(_vorder(disc), 2 ** lmin)
    assert_blocks(lib, L, got, want, tol, f"FMG {s} (coarse kappa {kappa:.1e})")
    assert st.cycles == s[3] + 1


def test_fmg_c1_to_tolerance(libs):
    """c1 workload: P1-P1, 6 tets, L=3, sine solution, FMG with V(3,3), then
    V(3,3) cycles to relative residual 1e-10; result equals the oracle run with
    the same number of cycles."""
    lib = libs(P1, 0, 3)
    H = mg.Hierarchy(1, 0, 3, schur="sd")
    prob = W.sine_cube()
    om = 2.3
    got, st = _fmg_gpu(lib, H, prob, 3, None,
                       hhg.solver_params(3, 3, 0, 1, hhg.HHG_GS_FWD, 1, om, rtol=1e-10, max_cycles=60))
    assert st.rel_res <= 1e-10
    want = H.fmg(prob, mg.Params(3, 3, 0, 1, "f", 1, om), cycles_on_finest=st.cycles - 1)
    tol, kappa = coarse_tolerance(1, 1)
    assert_blocks(lib, 3, got, want, tol, f"FMG + V(3,3) to 1e-10 (coarse kappa {kappa:.1e})")
    b = H.rhs(3, prob)
    r = H.residual_norms(3, want, b)
    assert np.hypot(*r) <= 1.01e-10 * np.linalg.norm(b)


def test_exact_reproduction_gpu(libs):
    """Taylor-Hood reproduces quadratic velocity / linear pressure fields."""
    lib = libs(P2, 1, 3)
    H = mg.Hierarchy(2, 1, 3, schur="sd")
    prob = W.quadratic_exact()
    got, st = _fmg_gpu(lib, H, prob, 3, None,
                       hhg.solver_params(3, 3, 0, 1, hhg.HHG_GS_FWD, 3, 2.3, extra_cycles=3))
    xs = H.S[3].interpolate(prob.u, prob.p)
    assert np.abs(got - xs).max() < 1e-10


@pytest.mark.parametrize("disc,L", [(P1, 4), (P2, 3)])
def test_float32_apply_error(libs, disc, L):
    """float32 storage and accumulation: error against the float64 oracle
    bounded by a small multiple of the float32 unit roundoff times the row
    magnitude."""
    lib = libs(disc, 0 if disc == P1 else 1, L)
    S = Stokes(fe.Level(2 ** L, _vorder(disc)))
    x = _rand(S, 51)
    dx = lib.from_lattice(L, x, hhg.HHG_F32)
    dy = lib.empty(L, lib.torch.float32)
    hhg.hhg_apply(lib.h, L, hhg.HHG_OP_FULL, dx, dy, hhg.HHG_F32)
    got = lib.to_lattice(L, dy, hhg.HHG_F32)
    assert rel_err(got, S.apply(x)) < 2e-5


@pytest.mark.parametrize("disc,lmin,L", CASES)
def test_mass_and_dots(libs, disc, lmin, L):
    lib = libs(disc, lmin, L)
    S = Stokes(fe.Level(2 ** L, _vorder(disc)))
    x = _rand(S, 61)
    dx = lib.from_lattice(L, x)
    dy = lib.empty(L)
    hhg.hhg_apply(lib.h, L, hhg.HHG_OP_MASS, dx, dy)
    want = S.apply_block(x, "MASS")
    assert_blocks(lib, L, lib.to_lattice(L, dy), want, 1e-12, "mass")
    du, dp = hhg.hhg_dots(lib.h, L, dx, dy)
    us, p = S.split(x)
    wu, wp = S.split(want)
    assert abs(du - sum(a @ b for a, b in zip(us, wu))) < 1e-12 * abs(du)
    assert abs(dp - p @ wp) < 1e-12 * abs(dp)


def test_fmg_full_size_c2(libs):
    """The benchmark workload at full size: P2-P1, 6 tets, level 5 (859,812
    DoFs), paper cube solution, FMG(0,2,1,1,A_f,3) in the launch configuration
    bench.py times; every DoF against the oracle's FMG."""
    L = 5
    lib = libs(P2, 1, L)
    H = mg.Hierarchy(2, 1, L, schur="sd")
    prob = W.paper_cube()
    om = 2.3
    want = H.fmg(prob, mg.Params(0, 2, 1, 1, "f", 3, om))
    got, st = _fmg_gpu(lib, H, prob, L, None, hhg.solver_params(0, 2, 1, 1, hhg.HHG_GS_FWD, 3, om))
    assert got.size == 859812
    tol, kappa = coarse_tolerance(2, 2)
    assert_blocks(lib, L, got, want, tol, f"FMG c2 full size (coarse kappa {kappa:.1e})")


def test_fmg_graph_replay_matches_eager(libs):
    """Fixed-work FMG calls (no stats, no tolerance) replay a captured HIP
    graph; every replay, with eager library work and synchronisations in
    between, equals the eager solve bit for bit."""
    L = 4
    lib = libs(P2, 1, L)
    torch = lib.torch
    H = mg.Hierarchy(2, 1, L, schur="sd")
    prob = W.paper_cube()
    bs = [lib.from_lattice(l, H.rhs(l, prob)) for l in range(1, L + 1)]
    x0 = lib.from_lattice(L, H.initial(L, prob))
    prm = hhg.solver_params(0, 2, 1, 1, hhg.HHG_GS_FWD, 3, 2.3, extra_cycles=1)
    x = x0.clone()
    hhg.hhg_fmg_solve(lib.h, x, bs, prm, want_stats=True)          # eager
    want = lib.to_lattice(L, x)
    for rep in range(4):
        x.copy_(x0)
        hhg.hhg_fmg_solve(lib.h, x, bs, prm, want_stats=False)      # graph (captured on rep 0)
        torch.cuda.synchronize()
        got = lib.to_lattice(L, x)
        assert np.array_equal(got, want), rep
        y = lib.empty(L)
        hhg.hhg_apply(lib.h, L, hhg.HHG_OP_FULL, x, y)               # eager work between replays
        hhg.hhg_norms(lib.h, L, y)


def test_errors_are_reported(libs):
    lib = libs(P1, 0, 3)
    x = lib.empty(3)
    with pytest.raises(hhg.HHGError):
        hhg.hhg_apply(lib.h, 9, hhg.HHG_OP_FULL, x, lib.empty(3))
    with pytest.raises(hhg.HHGError):
        hhg.hhg_apply(lib.h, 3, hhg.HHG_OP_FULL, x, x)
    with pytest.raises(hhg.HHGError):
        hhg.hhg_coarse_solve(lib.h, x, lib.empty(3), hhg.HHG_F32)


# ------------------------------------------------- Schur diagonal M_L
# eq. omega-eigenvalue-problem normalises by the lumped P1 mass M_L; the
# HHG_SCHUR_ML hierarchy uses S_hat = omega^{-1} M_L in eq. uzawa-pressure.
ML_CASES = [(P1, 0, 3), (P2, 1, 3)]


@pytest.mark.parametrize("disc,lmin,L", ML_CASES)
def test_ml_omega_estimate(libs, disc, lmin, L):
    lib = libs(disc, lmin, L, 0, hhg.HHG_SCHUR_ML)
    S = Stokes(fe.Level(2 ** L, _vorder(disc)))
    v0 = W.normal_vector(43, S.np_)
    want = osm.Uzawa(S, "ml").estimate_omega_inv(v0, 100)
    got = hhg.hhg_estimate_omega(lib.h, L, lib.torch.from_numpy(v0).to(lib.dev), 100)
    print(f"[parity] ML omega_inv {got:.12f} oracle {want:.12f}")
    assert abs(got - want) <= 1e-12 * want


@pytest.mark.parametrize("disc,lmin,L", ML_CASES)
@pytest.mark.parametrize("gs,xi", [("f", 3), ("s", 1)])
def test_ml_smooth(libs, disc, lmin, L, gs, xi):
    lib = libs(disc, lmin, L, 0, hhg.HHG_SCHUR_ML)
    S = Stokes(fe.Level(2 ** L, _vorder(disc)))
    U = osm.Uzawa(S, "ml")
    x = _rand(S, 13)
    b = _rand(S, 14, zero_bnd=True)
    om = 0.45
    want = x
    for _ in range(2):
        want = U.iterate(want, b, gs, xi, 1.0 / om)
    dx = lib.from_lattice(L, x)
    hhg.hhg_smooth(lib.h, L, dx, lib.from_lattice(L, b), 2, hhg.HHG_GS_FWD if gs == "f" else hhg.HHG_GS_SYM, xi, om)
    assert_blocks(lib, L, lib.to_lattice(L, dx), want, 1e-12, f"ML smooth {gs}{xi}")


@pytest.mark.parametrize("disc,lmin,L", ML_CASES)
def test_ml_vcycle_and_fmg(libs, disc, lmin, L):
    lib = libs(disc, lmin, L, 0, hhg.HHG_SCHUR_ML)
    H = mg.Hierarchy(_vorder(disc), lmin, L, schur="ml")
    prob = W.sine_cube() if disc == P1 else W.paper_cube()
    om = 0.45
    s = (1, 2, 1, 1, "f", 1 if disc == P1 else 3)
    b = H.rhs(L, prob)
    x = H.initial(L, prob)
    want = H.vcycle(L, L, x, b, mg.Params(*s, omega_inv=om))
    dx = lib.from_lattice(L, x)
    cs = hhg.solver_params(s[0], s[1], s[2], s[3], hhg.HHG_GS_FWD, s[5], om)
    hhg.hhg_vcycle(lib.h, L, dx, lib.from_lattice(L, b), cs)
    tol, kappa = coarse_tolerance(_vorder(disc), 2 ** lmin)
    assert_blocks(lib, L, lib.to_lattice(L, dx), want, tol, f"ML V-cycle (coarse kappa {kappa:.1e})")
    want = H.fmg(prob, mg.Params(*s, omega_inv=om), cycles_on_finest=1)
    got, st = _fmg_gpu(lib, H, prob, L, None,
                       hhg.solver_params(s[0], s[1], s[2], s[3], hhg.HHG_GS_FWD, s[5], om, extra_cycles=1))
    assert_blocks(lib, L, got, want, tol, f"ML FMG (coarse kappa {kappa:.1e})")
