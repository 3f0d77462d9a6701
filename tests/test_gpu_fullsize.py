"""Operator apply at the benchmark's full size (48 macro-tets, level 7,
N = 256: 1.35e8 P2 sites for P2-P1, 1.7e7 nodes for P1-P1), in the launch
configuration the benchmark times, checked row by row on sampled outputs.

The oracle cannot assemble the operator at this size; a row of the
discrete operator depends only on the row type (velocity parity class and
the boundary class of its position) and scales with a power of h.  So each
sampled row's expected value is the oracle's assembled row at a
representative node of the same type on the N = 8 lattice, rescaled
(A: h, B and B^T: h^2, PSPG C: h^3) and applied to the same input words.
Samples: interior velocity rows of every parity class and component,
boundary velocity rows (zero), pressure rows of all 27 boundary classes.
The same check runs on the mixed-precision workload's variable-viscosity
operator (6 macro-tets, level 7, N = 128).  The row construction itself is
checked on the CPU against the oracle's assembled operator at N = 16."""
import numpy as np
import pytest

from oracle import fe
from oracle.stokes import Stokes
from paper_2010_13513_amd import hhg, workloads as W
from tests.gpu_util import Lib

NS = 8          # oracle lattice of the representative rows
PARITIES = [(a, b, c) for c in (0, 1) for b in (0, 1) for a in (0, 1)]


def sampled_rows(vo, N, rng, per_class=6, nu=None):
    """Rows of calA on the N lattice, as (lattice index of the output,
    [(lattice index of an input word, weight)]), plus lattice indices of
    boundary velocity rows (whose output is zero).  Plain lattice order:
    [u1 | u2 | u3 | p], velocity on the (vo N + 1)^3 lattice.

    nu: viscosity at the P1 nodes of the N lattice ((N+1)^3, lattice order)
    for the variable-viscosity A.  A velocity row then comes from an N = 8
    oracle level whose vertex viscosities are those of the same window of the
    big lattice (shifted by the P1 offset between the sampled site and its
    representative); only the vertices of the row's own elements enter it."""
    lev = fe.Level(NS, vo)
    A = lev.A.tocsr()
    BT = [b.tocsc() for b in lev.B]
    Bc = [b.tocsr() for b in lev.B]
    C = lev.C.tocsr()
    vc, pc = lev.vcoords, lev.pcoords
    ms = vo * NS + 1
    n1, M = N + 1, vo * N
    m1 = M + 1
    f = NS / float(N)
    fA, fB, fC = f, f * f, f ** 3

    def vlat(d, X, Y, Z):
        return int(d * m1 ** 3 + X + m1 * (Y + m1 * Z))

    def plat(i, j, k):
        return int(3 * m1 ** 3 + i + n1 * (j + n1 * k))

    rows = []
    for par in PARITIES:
        n = 0
        while n < per_class:
            S = np.array([rng.integers(1, M) for _ in range(3)])
            S = S - (S & 1) + np.array(par)
            if S.min() < 1 or S.max() > M - 1:
                continue
            n += 1
            d = int(rng.integers(0, 3))
            rep = np.array([vo * NS // 2 + (s & 1) for s in S])
            r = int(rep[0] + ms * (rep[1] + ms * rep[2]))
            terms = []
            if nu is not None:
                delta = (S - rep) // vo
                q = np.arange(NS + 1)
                I, J, K = np.meshgrid(q, q, q, indexing="ij")
                idx = [np.clip(a + o, 0, N) for a, o in zip((I, J, K), delta)]
                nu_s = nu.reshape(N + 1, N + 1, N + 1)[idx[2], idx[1], idx[0]]
                A = fe.Level(NS, vo, np.transpose(nu_s, (2, 1, 0)).ravel()).A.tocsr()
            row = A.getrow(r)
            for c, w in zip(row.indices, row.data):
                terms.append((vlat(d, *(S + vc[c] - rep)), fA * w))
            col = BT[d][:, r]
            for kk, w in zip(col.indices, col.data):
                terms.append((plat(*((S + vo * pc[kk] - rep) // vo)), fB * w))
            rows.append((vlat(d, *S), terms))
    bnd = []
    for _ in range(16):
        S = [int(rng.integers(0, M + 1)) for _ in range(3)]
        S[int(rng.integers(0, 3))] = int(rng.choice([0, M]))
        bnd.append(vlat(int(rng.integers(0, 3)), *S))
    for cls in range(27):
        cc = [cls % 3, (cls // 3) % 3, cls // 9]
        for _ in range(2):
            P = np.array([0 if c == 0 else (N if c == 2 else int(rng.integers(1, N))) for c in cc])
            rep = np.array([0 if c == 0 else (NS if c == 2 else NS // 2) for c in cc])
            k = int(rep[0] + (NS + 1) * (rep[1] + (NS + 1) * rep[2]))
            terms = []
            for d in range(3):
                row = Bc[d].getrow(k)
                for c, w in zip(row.indices, row.data):
                    terms.append((vlat(d, *(vo * P + vc[c] - vo * rep)), fB * w))
            row = C.getrow(k)
            for c, w in zip(row.indices, row.data):
                terms.append((plat(*(P + pc[c] - rep)), -fC * w))
            rows.append((plat(*P), terms))
    return rows, bnd


def check_rows(rows, bnd, xval, got, rtol=1e-12, bval=None):
    """Compare gathered outputs with the rows; xval maps input index -> value.
    bval (residual): the right-hand side at each row's output, expected b -
    row . x, error relative to |b| + sum |w x|."""
    for q, ((yl, terms), g) in enumerate(zip(rows, got[:len(rows)])):
        want = sum(w * xval[i] for i, w in terms)
        scale = sum(abs(w * xval[i]) for i, w in terms)
        if bval is not None:
            want, scale = bval[q] - want, scale + abs(bval[q])
        assert abs(g - want) <= rtol * scale, (yl, g, want)
    assert np.all(got[len(rows):] == 0.0)


def _nu_nodes(N):
    """The variable-viscosity workload's field at the P1 nodes of the N
    lattice (lattice order)."""
    from oracle import mesh
    c = mesh.p1_coords(N) / float(N)
    return W.gaussian_bump_viscosity(W.SEED_BASE + 4000, N_ref=N)(c[:, 0], c[:, 1], c[:, 2])


@pytest.mark.parametrize("vo", [2, 1])
@pytest.mark.parametrize("varnu", [False, True])
def test_sampled_rows_reproduce_assembled_operator(vo, varnu):
    """CPU: the representative-row construction at N = 16 against the
    oracle's operator assembled at N = 16 (constant and variable viscosity)."""
    N = 16
    nu = _nu_nodes(N) if varnu else None
    rows, bnd = sampled_rows(vo, N, np.random.default_rng(11), per_class=3, nu=nu)
    S = Stokes(fe.Level(N, vo, nu))
    x = np.random.default_rng(12).standard_normal(S.n)
    y = S.apply(x)
    got = y[[r[0] for r in rows] + bnd]
    check_rows(rows, bnd, x, got)


@pytest.mark.gpu
@pytest.mark.parametrize("disc,prec", [(hhg.HHG_P2P1, hhg.HHG_F64), (hhg.HHG_P1P1, hhg.HHG_F64),
                                       (hhg.HHG_P2P1, hhg.HHG_F32)])
def test_apply_full_size_sampled_rows(disc, prec):
    """float32: the input is the float32 rounding of the float64 lattice
    vector, which the expected rows use as well; arithmetic in float32.
    Tolerance 3e-5 of the sum of |weight x input| of the row: a float32 sum
    of n terms errs by at most about n u of that sum (u = 6e-8), and the
    longest row (a P2-P1 pressure row) has ~200 terms plus a few rounded
    scalings, so 500 u bounds every row."""
    lib = Lib(disc, 6, 7, macro_refine=1)
    torch = lib.torch
    try:
        vo = 2 if disc == hhg.HHG_P2P1 else 1
        dt = torch.float64 if prec == hhg.HHG_F64 else torch.float32
        N, nn, vw, lw = lib.layout(7)
        assert N == 256
        print(f"apply full size: disc {disc}, prec {prec}, N {N}, {vw} words", flush=True)
        gen = torch.Generator(device=lib.dev).manual_seed(13513 + 3000)
        lat = torch.randn(lw, generator=gen, dtype=torch.float64, device=lib.dev)
        if prec == hhg.HHG_F32:
            lat = lat.float().double()
        x = torch.zeros(vw, dtype=dt, device=lib.dev)
        hhg.hhg_vec_from_lattice(lib.h, 7, lat, x, prec)
        y = torch.empty_like(x)
        hhg.hhg_apply(lib.h, 7, hhg.HHG_OP_FULL, x, y, prec)
        del x
        ylat = torch.empty_like(lat)
        hhg.hhg_vec_to_lattice(lib.h, 7, y, ylat, prec)
        del y
        torch.cuda.synchronize()

        rows, bnd = sampled_rows(vo, N, np.random.default_rng(7))
        assert len(rows) > 100
        got = ylat.index_select(0, torch.tensor([r[0] for r in rows] + bnd, device=lib.dev)).cpu().numpy()
        xi = sorted({t[0] for r in rows for t in r[1]})
        xv = dict(zip(xi, lat.index_select(0, torch.tensor(xi, device=lib.dev)).cpu().numpy()))
        check_rows(rows, bnd, xv, got, rtol=1e-12 if prec == hhg.HHG_F64 else 3e-5)
    finally:
        lib.close()


@pytest.mark.gpu
@pytest.mark.parametrize("disc,prec", [(hhg.HHG_P2P1, hhg.HHG_F64), (hhg.HHG_P2P1, hhg.HHG_F32),
                                       (hhg.HHG_P1P1, hhg.HHG_F32)])
def test_residual_full_size_sampled_rows(disc, prec):
    """r = b - calA x in the same launch configuration (the residual form of
    the k-marching kernel, which loads b ahead of each plane's arithmetic):
    sampled interior rows against b - (rescaled oracle row) . x, Dirichlet
    velocity rows zero.  Tolerances as for the apply, relative to |b| +
    sum |w x|."""
    lib = Lib(disc, 6, 7, macro_refine=1)
    torch = lib.torch
    try:
        vo = 2 if disc == hhg.HHG_P2P1 else 1
        dt = torch.float64 if prec == hhg.HHG_F64 else torch.float32
        N, nn, vw, lw = lib.layout(7)
        print(f"residual full size: disc {disc}, prec {prec}, N {N}, {vw} words", flush=True)
        gen = torch.Generator(device=lib.dev).manual_seed(13513 + 3002)
        lat = torch.randn(lw, generator=gen, dtype=torch.float64, device=lib.dev)
        blat = torch.randn(lw, generator=gen, dtype=torch.float64, device=lib.dev)
        if prec == hhg.HHG_F32:
            lat, blat = lat.float().double(), blat.float().double()
        x = torch.zeros(vw, dtype=dt, device=lib.dev)
        b = torch.zeros(vw, dtype=dt, device=lib.dev)
        hhg.hhg_vec_from_lattice(lib.h, 7, lat, x, prec)
        hhg.hhg_vec_from_lattice(lib.h, 7, blat, b, prec)
        r = torch.empty_like(x)
        hhg.hhg_residual(lib.h, 7, x, b, r, prec)
        del x, b
        rlat = torch.empty_like(lat)
        hhg.hhg_vec_to_lattice(lib.h, 7, r, rlat, prec)
        del r
        torch.cuda.synchronize()

        rows, bnd = sampled_rows(vo, N, np.random.default_rng(9))
        out = torch.tensor([q[0] for q in rows] + bnd, device=lib.dev)
        got = rlat.index_select(0, out).cpu().numpy()
        bval = blat.index_select(0, out).cpu().numpy()[:len(rows)]
        xi = sorted({t[0] for q in rows for t in q[1]})
        xv = dict(zip(xi, lat.index_select(0, torch.tensor(xi, device=lib.dev)).cpu().numpy()))
        check_rows(rows, bnd, xv, got, rtol=1e-12 if prec == hhg.HHG_F64 else 3e-5, bval=bval)
    finally:
        lib.close()


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [hhg.HHG_F64, hhg.HHG_F32])
def test_restriction_adjoint_full_size(prec):
    """The restriction at the throughput size (48 tets, level 7 -> 6, the
    k-marching velocity form) is the transpose of the interpolation (Sec.
    3.3): <R r, x_c>_u = <r, P x_c>_u for random r and a coarse x_c with zero
    boundary velocity (x_c = R r2), velocity parts.  Tolerance: 1e-12
    (float64) / 1e-5 (float32) of sum |terms|, bounded by |r| |P x_c|."""
    lib = Lib(hhg.HHG_P2P1, 6, 7, macro_refine=1)
    torch = lib.torch
    try:
        dt = torch.float64 if prec == hhg.HHG_F64 else torch.float32
        _, _, vwf, _ = lib.layout(7)
        _, _, vwc, _ = lib.layout(6)
        print(f"restriction adjoint full size: prec {prec}, {vwf} fine words", flush=True)
        gen = torch.Generator(device=lib.dev).manual_seed(13513 + 3003)
        r = torch.randn(vwf, generator=gen, dtype=torch.float64, device=lib.dev).to(dt)
        r2 = torch.randn(vwf, generator=gen, dtype=torch.float64, device=lib.dev).to(dt)
        rc = torch.zeros(vwc, dtype=dt, device=lib.dev)
        xc = torch.zeros(vwc, dtype=dt, device=lib.dev)
        hhg.hhg_restrict(lib.h, 7, r, rc, prec)
        hhg.hhg_restrict(lib.h, 7, r2, xc, prec)
        pxc = torch.zeros(vwf, dtype=dt, device=lib.dev)
        hhg.hhg_prolong_add(lib.h, 6, xc, pxc, prec)
        lhs, _ = hhg.hhg_dots(lib.h, 6, rc, xc, prec)
        rhs, _ = hhg.hhg_dots(lib.h, 7, r, pxc, prec)
        un, _ = hhg.hhg_dots(lib.h, 7, r, r, prec)
        pn, _ = hhg.hhg_dots(lib.h, 7, pxc, pxc, prec)
        scale = float(np.sqrt(un * pn))
        tol = 1e-12 if prec == hhg.HHG_F64 else 1e-5
        assert abs(lhs - rhs) <= tol * scale, (lhs, rhs, scale)
    finally:
        lib.close()


@pytest.mark.gpu
@pytest.mark.parametrize("disc", [hhg.HHG_P2P1, hhg.HHG_P1P1])
def test_variable_viscosity_apply_full_size_sampled_rows(disc):
    """The mixed-precision workload's operator: 6 macro-tets, level 7
    (N = 128), Gaussian-bump viscosity 1:100, float64, sampled rows against
    oracle rows assembled with the same vertex viscosities."""
    lib = Lib(disc, 6, 7)
    torch = lib.torch
    try:
        vo = 2 if disc == hhg.HHG_P2P1 else 1
        N, nn, vw, lw = lib.layout(7)
        assert N == 128
        nu = _nu_nodes(N)
        hhg.hhg_set_viscosity(lib.h, 7, torch.from_numpy(nu).to(lib.dev))
        print(f"variable-viscosity apply full size: disc {disc}, N {N}, {vw} words", flush=True)
        gen = torch.Generator(device=lib.dev).manual_seed(13513 + 3001)
        lat = torch.randn(lw, generator=gen, dtype=torch.float64, device=lib.dev)
        x = torch.zeros(vw, dtype=torch.float64, device=lib.dev)
        hhg.hhg_vec_from_lattice(lib.h, 7, lat, x)
        y = torch.empty_like(x)
        hhg.hhg_apply(lib.h, 7, hhg.HHG_OP_FULL, x, y)
        ylat = torch.empty_like(lat)
        hhg.hhg_vec_to_lattice(lib.h, 7, y, ylat)
        torch.cuda.synchronize()

        rows, bnd = sampled_rows(vo, N, np.random.default_rng(8), per_class=4, nu=nu)
        got = ylat.index_select(0, torch.tensor([r[0] for r in rows] + bnd, device=lib.dev)).cpu().numpy()
        xi = sorted({t[0] for r in rows for t in r[1]})
        xv = dict(zip(xi, lat.index_select(0, torch.tensor(xi, device=lib.dev)).cpu().numpy()))
        check_rows(rows, bnd, xv, got)
    finally:
        lib.close()


def _lattice_xyz(torch, dev, M):
    """Coordinates of the (M+1)^3 lattice in plain order X + (M+1)(Y + (M+1) Z)."""
    g = torch.arange(M + 1, dtype=torch.float64, device=dev) / M
    z, y, x = torch.meshgrid(g, g, g, indexing="ij")
    return x.reshape(-1), y.reshape(-1), z.reshape(-1)


@pytest.mark.gpu
@pytest.mark.parametrize("disc,prec,lmin,L,refine", [
    (hhg.HHG_P2P1, hhg.HHG_F64, 6, 7, 1), (hhg.HHG_P2P1, hhg.HHG_F32, 6, 7, 1),
    (hhg.HHG_P1P1, hhg.HHG_F64, 6, 7, 1), (hhg.HHG_P2P1, hhg.HHG_F64, 5, 6, 0)])
def test_prolongation_reproduces_polynomials_full_size(disc, prec, lmin, L, refine):
    """Prolong-add at the throughput size (48 tets, level 6 -> 7, the
    coarse-cube form; and 6 tets, level 5 -> 6, its smallest lattice): the
    interpolation is the embedding of the coarse element spaces (Sec. 3.3), so
    coarse nodal values of a quadratic velocity (P2; linear for P1) and a
    linear pressure arrive as the fine nodal values of the same polynomials,
    added to a random fine vector at every site (boundary sites included, as
    this call adds there).  Tolerance: 1e-13 (float64) / 2e-6 (float32) of
    the largest polynomial value plus the random word."""
    lib = Lib(disc, lmin, L, macro_refine=refine)
    torch = lib.torch
    try:
        dev = lib.dev
        vo = 2 if disc == hhg.HHG_P2P1 else 1
        dt = torch.float64 if prec == hhg.HHG_F64 else torch.float32
        Nf, _, vwf, lwf = lib.layout(L)
        Nc, _, vwc, lwc = lib.layout(L - 1)
        assert Nf == 2 * Nc and Nf >= 64
        print(f"prolongation polynomials: disc {disc} prec {prec} N {Nc} -> {Nf}", flush=True)

        def fields(N):
            x, y, z = _lattice_xyz(torch, dev, vo * N)
            if vo == 2:
                u = [0.3 + x - 2 * y + 0.5 * z + 3 * x * y - y * z + 2 * z * z - x * x,
                     -1 + 0.25 * x + y * y - 2 * x * z + 1.5 * y * z,
                     2 - x + 0.75 * y - z + x * z - 3 * y * y + 0.5 * x * y]
            else:
                u = [0.3 + x - 2 * y + 0.5 * z, -1 + 0.25 * x + 1.5 * z, 2 - x + 0.75 * y - z]
            del x, y, z
            px, py, pz = _lattice_xyz(torch, dev, N)
            p = 0.5 - px + 2 * py + 0.25 * pz
            return u, p

        u, p = fields(Nc)
        src = torch.cat(u + [p])
        del u, p
        assert src.numel() == lwc
        xc = torch.zeros(vwc, dtype=dt, device=dev)
        hhg.hhg_vec_from_lattice(lib.h, L - 1, src, xc, prec)
        del src
        gen = torch.Generator(device=dev).manual_seed(13513 + 3004)
        rnd = torch.randn(lwf, generator=gen, dtype=torch.float64, device=dev)
        xf = torch.zeros(vwf, dtype=dt, device=dev)
        hhg.hhg_vec_from_lattice(lib.h, L, rnd, xf, prec)
        before = torch.empty(lwf, dtype=torch.float64, device=dev)
        hhg.hhg_vec_to_lattice(lib.h, L, xf, before, prec)  # the random words as stored
        del rnd
        hhg.hhg_prolong_add(lib.h, L - 1, xc, xf, prec)
        got = torch.empty(lwf, dtype=torch.float64, device=dev)
        hhg.hhg_vec_to_lattice(lib.h, L, xf, got, prec)
        torch.cuda.synchronize()
        u, p = fields(Nf)
        m3 = (vo * Nf + 1) ** 3
        tol = (1e-13 if prec == hhg.HHG_F64 else 2e-6) * (max(float(t.abs().max()) for t in u + [p]) +
                                                         float(before.abs().max()))
        for d in range(3):
            err = float((got[d * m3:(d + 1) * m3] - before[d * m3:(d + 1) * m3] - u[d]).abs().max())
            assert err <= tol, (d, err, tol)
        err = float((got[3 * m3:] - before[3 * m3:] - p).abs().max())
        assert err <= tol, ("p", err, tol)
    finally:
        lib.close()
