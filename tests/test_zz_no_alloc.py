"""The allocation-free entry point hhg_mlp_train_noalloc against
hhg_mlp_train through the C ABI: two calls in a row (the second with fewer
samples and epochs, so the shared static scratch holds the first call's
leftovers), each giving the same parameters bit for bit and the same last
loss as the allocating entry point from the same start; a request beyond the
scratch limit is refused with HHG_ERR_ARG and changes nothing."""
import numpy as np
import pytest

from oracle import mlp as omlp
from paper_2010_13513_amd import hhg
from tests.gpu_util import torch_cuda

pytestmark = pytest.mark.gpu


def _flat(ps):
    return np.concatenate([p.reshape(-1) for p in ps]).astype(np.float32)


def test_train_noalloc_matches_train():
    torch = torch_cuda()
    ctx = hhg.hhg_ctx_create(0, torch.cuda.current_stream().cuda_stream)
    rng = np.random.default_rng(77)
    n_in, H, n_out = 24, 64, 12
    p0 = _flat(omlp.init_params(rng, n_in, H, n_out))
    A = rng.standard_normal((n_out, n_in)) / 4.0
    X = rng.standard_normal((1024, n_in)).astype(np.float32)
    Y = np.tanh(X @ A.T).astype(np.float32)
    dx, dy = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    ma = hhg.hhg_mlp_create(ctx, n_in, H, n_out, 64)
    mb = hhg.hhg_mlp_create(ctx, n_in, H, n_out, 64)
    try:
        hhg.hhg_mlp_set_params(ma, p0)
        hhg.hhg_mlp_set_params(mb, p0)
        for n, batch, epochs in ((1024, 64, 12), (300, 32, 3)):       # second call: smaller input
            order = np.concatenate([rng.permutation(n) for _ in range(epochs)])
            la = hhg.hhg_mlp_train(ma, dx, dy, n, batch, epochs, 1e-3, order)
            lb = hhg.hhg_mlp_train_noalloc(mb, dx, dy, n, batch, epochs, 1e-3, order)
            pa, pb = hhg.hhg_mlp_get_params(ma), hhg.hhg_mlp_get_params(mb)
            print(f"[noalloc] n {n} epochs {epochs}: loss {la:.6e} / {lb:.6e}, "
                  f"params equal {np.array_equal(pa, pb)}")
            assert la == lb
            assert np.array_equal(pa, pb)
            assert not np.array_equal(pa, p0)
        before = hhg.hhg_mlp_get_params(mb)
        big = np.zeros(2 * (1 << 20) + 1024, dtype=np.int32)                # epochs * n > 2^21
        with pytest.raises(hhg.HHGError) as e:
            hhg.hhg_mlp_train_noalloc(mb, dx, dy, 1024, 64, 2049, 1e-3, big)
        assert e.value.status == hhg.HHG_ERR_ARG
        assert "2097152" in str(e.value)
        assert np.array_equal(hhg.hhg_mlp_get_params(mb), before)
    finally:
        torch.cuda.synchronize()
        hhg.hhg_mlp_destroy(ma)
        hhg.hhg_mlp_destroy(mb)
        hhg.hhg_ctx_destroy(ctx)
