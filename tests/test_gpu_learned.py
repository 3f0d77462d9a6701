"""GPU tests of the learned coarse-solve pipeline: pairs recorded at the
coarse-grid visits of plain solves (checked against the oracle's
pseudo-inverse), smoothing-only coarse treatment, and a network trained on
the GPU that (i) beats the solver without a coarse solve, (ii) needs no
pseudo-inverse rebuild for a new viscosity, and (iii) with the fallback
monitor reaches the plain solver's answer.

Sizes: P1-P1 PSPG, coarsest N = 4 (206 unknowns, 331 features), finest N = 16;
a few hundred training seeds (a reduced form of the 20k-pair workload)."""
import numpy as np
import pytest

from oracle import coarse as ocoarse, fe, mesh
from oracle.stokes import Stokes
from paper_2010_13513_amd import hhg, learned, workloads as W
from paper_2010_13513_amd.problem import Problem
from tests.gpu_util import torch_cuda

pytestmark = pytest.mark.gpu


def _nu_nodes(N, fn):
    c = mesh.p1_coords(N) / float(N)
    return fn(c[:, 0], c[:, 1], c[:, 2])


@pytest.fixture(scope="module")
def env():
    torch = torch_cuda()
    ctx = hhg.hhg_ctx_create(0, torch.cuda.current_stream().cuda_stream)
    yield torch, ctx
    torch.cuda.synchronize()
    hhg.hhg_ctx_destroy(ctx)


def _prm(rtol=1e-10, coarse_smooth=0, max_cycles=60):
    return hhg.solver_params(2, 2, 1, 1, hhg.HHG_GS_FWD, 1, 2.3, rtol=rtol, max_cycles=max_cycles,
                             coarse_smooth=coarse_smooth)


def test_recorded_pairs_match_oracle(env):
    """Every pair recorded during a plain FMG solve: target = oracle
    pseudo-inverse solve of the recorded residual (pressure at zero mean)."""
    torch, ctx = env
    P = Problem(torch, ctx, hhg.HHG_P1P1, 2, 3)
    try:
        seed = learned.TRAIN_BASE + 7
        F, T, used = learned.collect_pairs(P, [seed], _prm(), 64)
        n_in, n_out = hhg.hhg_mlp_dims(P.h)
        assert used == 1 and F.shape[0] >= 3          # initial FMG solve + one per cycle
        nu = W.lognormal_viscosity(seed)
        S = Stokes(fe.Level(4, 1, _nu_nodes(4, nu)))
        cs = ocoarse.CoarseSolver(S)
        idx = ocoarse.unknown_index(S)
        Fh, Th = F.cpu().numpy().astype(np.float64), T.cpu().numpy().astype(np.float64)
        assert np.allclose(Fh[:, n_out:], np.log(_nu_nodes(4, nu))[None, :], rtol=1e-6, atol=1e-6)
        for k in range(F.shape[0]):
            assert abs(np.linalg.norm(Fh[k, :n_out]) - 1.0) < 1e-5
            r = S.zeros()
            r[idx] = Fh[k, :n_out]
            want = cs.solve(S.zeros(), r)[idx]
            assert np.linalg.norm(Th[k] - want) < 1e-4 * np.linalg.norm(want), k
    finally:
        P.close()


V33 = (3, 3, 0, 1, hhg.HHG_GS_FWD, 1)     # V(3,3): no extra coarse-level smoothing


def _v33(rtol=0.0, coarse_smooth=0):
    return hhg.solver_params(*V33, 2.3, rtol=rtol, max_cycles=60, coarse_smooth=coarse_smooth)


def test_smoothing_only_coarse_treatment_converges_slower(env):
    torch, ctx = env
    P = Problem(torch, ctx, hhg.HHG_P1P1, 2, 4)
    try:
        seed = learned.TEST_BASE + 1
        exact = learned.cycle_rates(P, seed, _v33(), cycles=8)
        smooth = learned.cycle_rates(P, seed, _v33(coarse_smooth=2), cycles=8)
        print(f"exact {np.round(exact, 3)}, smoothing only {np.round(smooth, 3)}")
        assert max(exact[2:]) < 0.45
        assert np.mean(smooth[2:]) > 1.2 * np.mean(exact[2:])
    finally:
        P.close()


def test_trained_network_gain(env):
    torch, ctx = env
    P = Problem(torch, ctx, hhg.HHG_P1P1, 2, 4)
    m = None
    try:
        seeds = [learned.TRAIN_BASE + s for s in range(700)]
        F, T, used = learned.collect_pairs(P, seeds, _prm(rtol=1e-8), 16000)
        assert F.shape[0] == 16000
        m, hist = learned.train(ctx, F, T, hidden=256, batch=256, epochs=60, lr=2e-3, lr_final=2e-4, stages=4)
        assert hist[-1] < 0.5 * hist[0]
        # held-out fields
        Fh, Th, _ = learned.collect_pairs(P, [learned.TEST_BASE + s for s in range(40)], _prm(rtol=1e-8), 400)
        err_test = learned.pair_errors(P, m, Fh, Th)
        err_train = learned.pair_errors(P, m, F[:1000], T[:1000])
        print(f"pair rel. error: train median {np.median(err_train):.3f}, held-out median {np.median(err_test):.3f}")
        assert np.median(err_test) < 0.6
        # V(3,3) rates on held-out fields: the network beats no coarse solve
        rates = {"exact": [], "mlp": [], "smooth": []}
        for s in range(3):
            seed = learned.TEST_BASE + 500 + s
            rates["exact"].append(np.mean(learned.cycle_rates(P, seed, _v33(), 8)[2:]))
            rates["smooth"].append(np.mean(learned.cycle_rates(P, seed, _v33(coarse_smooth=2), 8)[2:]))
            hhg.hhg_hier_set_mlp(P.h, m, 1.0, 0.0)
            rates["mlp"].append(np.mean(learned.cycle_rates(P, seed, _v33(), 8)[2:]))
            hhg.hhg_hier_set_mlp(P.h, None)
        print({k: np.round(v, 3).tolist() for k, v in rates.items()})
        assert np.mean(rates["mlp"]) < np.mean(rates["smooth"])
        # a new viscosity: the network path skips the pseudo-inverse rebuild,
        # and with the monitor reaches the plain solver's answer
        seed = learned.TEST_BASE + 900
        x_plain, st_plain, _ = learned.solve_instance(P, seed, _v33(rtol=1e-10))
        rho = st_plain.rel_res ** (1.0 / st_plain.cycles)
        hhg.hhg_hier_set_mlp(P.h, m, rho_plain=rho, tau=0.5)
        x_mlp, st_mlp, _ = learned.solve_instance(P, seed, _v33(rtol=1e-10))
        hhg.hhg_hier_set_mlp(P.h, None)
        print(f"plain cycles {st_plain.cycles}, network cycles {st_mlp.cycles}, fallbacks {st_mlp.fallbacks}")
        assert st_mlp.rel_res <= 1e-10
        d = (x_mlp - x_plain).abs().max().item() / x_plain.abs().max().item()
        assert d < 1e-7
    finally:
        if m is not None:
            hhg.hhg_hier_set_mlp(P.h, None)
            hhg.hhg_mlp_destroy(m)
        P.close()
