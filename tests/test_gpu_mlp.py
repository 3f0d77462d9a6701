"""GPU tests of the learned coarse solve: the MFMA network against the float64
MLP oracle (same bf16 storage points), training, training pairs against the
oracle's exact coarse correction, and the fallback monitor.

Tolerances.  (i) Exact-arithmetic networks: small-integer inputs, sparse
+-1 weights and integer biases keep every pre-activation a small integer, and
a batch of B x n_out a power of two makes the loss gradient's scale 2 / (B
n_out) exact, so every product, bf16 rounding and float32 sum is exact on
both sides and outputs and gradients must agree entry by entry, bit for bit
-- at ragged sizes (n_in = 331, tails of every 16-wide tile) and the hidden
width of the learned coarse solve (512), so a dropped or misplaced tile
cannot hide.  (ii) Random real-valued networks: weights and layer inputs are
bf16 on both sides, so the products agree up to float32-vs-float64
accumulation; where that difference crosses a bf16 rounding boundary of a
hidden activation the two sides round one entry differently (one bf16 ulp),
which moves the outputs by about 1e-3 relative, so these are compared in
norm at 1e-2 and the bulk of entries at 2e-3.
"""
import numpy as np
import pytest

from oracle import coarse as ocoarse, fe, mesh, mlp as omlp, multigrid as mg
from oracle.stokes import Stokes
from paper_2010_13513_amd import hhg, workloads as W
from tests.gpu_util import Lib, rel_err, torch_cuda

pytestmark = pytest.mark.gpu


def _flat(ps):
    return np.concatenate([p.reshape(-1) for p in ps]).astype(np.float32)


def _split(v, shapes):
    out, q = [], 0
    for s in shapes:
        n = int(np.prod(s))
        out.append(v[q:q + n].reshape(s))
        q += n
    return out


@pytest.fixture(scope="module")
def ctx():
    torch = torch_cuda()
    c = hhg.hhg_ctx_create(0, torch.cuda.current_stream().cuda_stream)
    yield torch, c
    torch.cuda.synchronize()
    hhg.hhg_ctx_destroy(c)


@pytest.mark.parametrize("n_in,H,n_out,B", [(37, 32, 21, 20), (331, 64, 206, 48)])
def test_forward_and_gradients_match_oracle(ctx, n_in, H, n_out, B):
    torch, c = ctx
    rng = np.random.default_rng(n_in)
    ps = omlp.init_params(rng, n_in, H, n_out)
    for k in range(1, 8, 2):
        ps[k] = rng.standard_normal(ps[k].shape) * 0.1
    ps = [p.astype(np.float32).astype(np.float64) for p in ps]     # float32 masters on both sides
    X = rng.standard_normal((B, n_in))
    Y = rng.standard_normal((B, n_out))
    m = hhg.hhg_mlp_create(c, n_in, H, n_out, 64)
    try:
        hhg.hhg_mlp_set_params(m, _flat(ps))
        assert np.array_equal(hhg.hhg_mlp_get_params(m), _flat(ps))
        dx = torch.from_numpy(X.astype(np.float32)).cuda()
        dy = torch.from_numpy(Y.astype(np.float32)).cuda()
        out = torch.empty(B, n_out, dtype=torch.float32, device="cuda")
        hhg.hhg_mlp_forward(m, dx, B, out)
        torch.cuda.synchronize()
        net = omlp.MLP(ps, quantize=True)
        want, _ = net.forward(X.astype(np.float32).astype(np.float64))
        got = out.cpu().numpy().astype(np.float64)
        assert np.linalg.norm(got - want) < 1e-2 * np.linalg.norm(want)
        assert np.median(np.abs(got - want)) < 2e-3 * np.abs(want).max()
        loss, g = hhg.hhg_mlp_loss_grad(m, dx, dy, B)
        wl, wg = net.loss_and_grads(X.astype(np.float32).astype(np.float64), Y.astype(np.float32).astype(np.float64))
        assert abs(loss - wl) < 1e-2 * wl
        shapes = [p.shape for p in ps]
        for k, (a, b) in enumerate(zip(_split(g.astype(np.float64), shapes), wg)):
            assert np.linalg.norm(a - b) < 2e-2 * np.linalg.norm(b) + 1e-12, k
    finally:
        hhg.hhg_mlp_destroy(m)


def _exact_net(rng, n_in, H, n_out, per_row=4):
    """Sparse +-1 weights (per_row nonzeros per row), biases in {-1, 0, 1}."""
    dims = [n_in, H, H, H, n_out]
    ps = []
    for l in range(4):
        W = np.zeros((dims[l + 1], dims[l]))
        for r in range(dims[l + 1]):
            cols = rng.choice(dims[l], size=min(per_row, dims[l]), replace=False)
            W[r, cols] = rng.choice([-1.0, 1.0], size=cols.size)
        ps += [W, rng.integers(-1, 2, size=dims[l + 1]).astype(np.float64)]
    return ps


@pytest.mark.parametrize("n_in,H,n_out,B", [(331, 512, 64, 32), (37, 48, 16, 16), (331, 64, 206, 64)])
def test_exact_arithmetic_network_matches_oracle_entrywise(ctx, n_in, H, n_out, B):
    torch, c = ctx
    rng = np.random.default_rng(1000 + n_in + H)
    ps = _exact_net(rng, n_in, H, n_out)
    X = rng.integers(-2, 3, size=(B, n_in)).astype(np.float64)
    Y = rng.integers(-3, 4, size=(B, n_out)).astype(np.float64)
    net = omlp.MLP(ps, quantize=True)
    want, cache = net.forward(X)
    assert max(np.abs(z).max() for _, z in cache) < 128        # every value exact in bf16
    assert np.all(want == np.round(want))
    m = hhg.hhg_mlp_create(c, n_in, H, n_out, B)
    try:
        hhg.hhg_mlp_set_params(m, _flat(ps))
        dx = torch.from_numpy(X.astype(np.float32)).cuda()
        dy = torch.from_numpy(Y.astype(np.float32)).cuda()
        out = torch.empty(B, n_out, dtype=torch.float32, device="cuda")
        hhg.hhg_mlp_forward(m, dx, B, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().astype(np.float64)
        assert np.array_equal(got, want), np.argwhere(got != want)[:5]
        scale = 2.0 / (B * n_out)
        if scale != 2.0 ** round(np.log2(scale)):
            return             # loss-gradient scale not exact (n_out = 206): forward only
        loss, g = hhg.hhg_mlp_loss_grad(m, dx, dy, B)
        wl, wg = net.loss_and_grads(X, Y)
        assert abs(loss - wl) <= 1e-12 * abs(wl)
        for k, (a, b) in enumerate(zip(_split(g.astype(np.float64), [p.shape for p in ps]), wg)):
            assert np.array_equal(a, b), (k, np.argwhere(a != b)[:5])
    finally:
        hhg.hhg_mlp_destroy(m)


def test_training_reduces_loss(ctx):
    """Fit a smooth map on the GPU with Adam; the held-out loss drops by 10x."""
    torch, c = ctx
    rng = np.random.default_rng(11)
    n_in, H, n_out, n = 16, 64, 8, 1024
    A = rng.standard_normal((n_out, n_in)) / 4.0
    X = rng.standard_normal((n + 256, n_in))
    Y = np.tanh(X @ A.T)
    m = hhg.hhg_mlp_create(c, n_in, H, n_out, 256)
    try:
        hhg.hhg_mlp_set_params(m, _flat(omlp.init_params(rng, n_in, H, n_out)))
        dx = torch.from_numpy(X.astype(np.float32)).cuda()
        dy = torch.from_numpy(Y.astype(np.float32)).cuda()
        l0, _ = hhg.hhg_mlp_loss_grad(m, dx[n:], dy[n:], 256)
        order = np.concatenate([rng.permutation(n) for _ in range(40)])
        hhg.hhg_mlp_train(m, dx, dy, n, 64, 40, 2e-3, order)
        l1, _ = hhg.hhg_mlp_loss_grad(m, dx[n:], dy[n:], 256)
        assert l1 < 0.1 * l0, (l0, l1)
    finally:
        hhg.hhg_mlp_destroy(m)


NU = W.lognormal_viscosity(W.SEED_BASE + 5000)


def _nu_nodes(N, fn=NU):
    cc = mesh.p1_coords(N) / float(N)
    return fn(cc[:, 0], cc[:, 1], cc[:, 2])


def test_training_pairs_match_oracle():
    """Features and exact-correction targets of the coarsest level (P1-P1, N=4,
    206 unknowns) against the oracle's pseudo-inverse solve with the same nu."""
    lib = Lib(hhg.HHG_P1P1, 2, 3)
    torch = lib.torch
    try:
        for l in (2, 3):
            hhg.hhg_set_viscosity(lib.h, l, torch.from_numpy(_nu_nodes(2 ** l)).cuda())
        n_in, n_out = hhg.hhg_mlp_dims(lib.h)
        assert (n_in, n_out) == (206 + 125, 206)
        S = Stokes(fe.Level(4, 1, _nu_nodes(4)))
        cs = ocoarse.CoarseSolver(S)
        r = S.zero_boundary(W.normal_vector(77, S.n))
        us, p = S.split(r)
        r = S.join(us, p - p.mean())
        feat = torch.empty(n_in, dtype=torch.float32, device="cuda")
        targ = torch.empty(n_out, dtype=torch.float32, device="cuda")
        hhg.hhg_coarse_pair(lib.h, lib.from_lattice(2, r), feat, targ)
        torch.cuda.synchronize()
        idx = ocoarse.unknown_index(S)
        nr = np.linalg.norm(r[idx])
        want_f = np.concatenate([r[idx] / nr, np.log(_nu_nodes(4))])
        corr = cs.solve(S.zeros(), r)
        want_t = corr[idx] / nr
        assert np.abs(feat.cpu().numpy() - want_f).max() < 1e-6 * np.abs(want_f).max()
        assert np.abs(targ.cpu().numpy() - want_t).max() < 1e-5 * np.abs(want_t).max()
    finally:
        lib.close()


def _solve_with(lib, H, prob, L, prm, torch):
    bs = [lib.from_lattice(l, H.rhs(l, prob)) for l in range(H.Lmin, L + 1)]
    dx = lib.from_lattice(L, H.initial(L, prob))
    st = hhg.hhg_fmg_solve(lib.h, dx, bs, prm)
    return lib.to_lattice(L, dx), st


def test_fallback_fires_on_bad_network_and_solve_converges():
    """A network with zero weights (no coarse correction) or NaN weights makes
    the finest-level residual ratio exceed the plain rate; the monitor undoes
    the cycle, switches to the exact coarse solve, and the solve reaches the
    tolerance with the same answer as the plain solver."""
    L = 4
    lib = Lib(hhg.HHG_P1P1, 2, L)
    torch = lib.torch
    try:
        nu_fn = W.lognormal_viscosity(W.SEED_BASE + 5001)
        for l in range(2, L + 1):
            hhg.hhg_set_viscosity(lib.h, l, torch.from_numpy(_nu_nodes(2 ** l, nu_fn)).cuda())
        H = mg.Hierarchy(1, 2, L, nu_fn=nu_fn, schur="sd")
        prob = W.fourier_forcing(W.SEED_BASE + 2001)
        prm = hhg.solver_params(3, 3, 0, 1, hhg.HHG_GS_FWD, 1, 2.3, rtol=1e-10, max_cycles=80)
        x_plain, st_plain = _solve_with(lib, H, prob, L, prm, torch)
        assert st_plain.fallbacks == 0
        n_in, n_out = hhg.hhg_mlp_dims(lib.h)
        m = hhg.hhg_mlp_create(lib.ctx, n_in, 64, n_out, 16)
        try:
            for bad in ("zero", "nan"):
                npar = hhg.hhg_mlp_num_params(m)
                w = np.zeros(npar, np.float32) if bad == "zero" else np.full(npar, np.nan, np.float32)
                hhg.hhg_mlp_set_params(m, w)
                hhg.hhg_hier_set_mlp(lib.h, m, rho_plain=0.3, tau=0.2)
                x, st = _solve_with(lib, H, prob, L, prm, torch)
                assert st.fallbacks >= 1, bad
                assert st.rel_res <= 1e-10
                assert rel_err(x, x_plain) < 1e-7, bad
            hhg.hhg_hier_set_mlp(lib.h, None)
        finally:
            hhg.hhg_mlp_destroy(m)
    finally:
        lib.close()
