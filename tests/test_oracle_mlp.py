"""Pins of the MLP oracle: bfloat16 rounding vs torch, backward vs central
finite differences, Adam vs torch.optim.Adam, a hand-computed tiny network."""
import numpy as np
import pytest
import torch

from oracle import mlp


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-20, 20, 5000),
                        [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0, -0.0, 3.0e38]])
    want = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x), want)
    assert mlp.bf16(np.array([1.0 + 2 ** -8]))[0] == 1.0            # tie to even
    assert mlp.bf16(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6


def test_tiny_network_by_hand():
    # 1 -> 1 -> 1 -> 1 -> 1 with known weights
    ps = [np.array([[2.0]]), np.array([-1.0]), np.array([[3.0]]), np.array([0.5]),
          np.array([[1.0]]), np.array([-4.0]), np.array([[-2.0]]), np.array([1.0])]
    net = mlp.MLP(ps, quantize=False)
    out, _ = net.forward(np.array([[1.5]]))
    # z1 = 2, a1 = 2; z2 = 6.5, a2 = 6.5; z3 = 2.5, a3 = 2.5; z4 = -4
    assert out[0, 0] == -4.0
    out, _ = net.forward(np.array([[0.25]]))
    # z1 = -0.5 -> 0; z2 = 0.5; z3 = -3.5 -> 0; z4 = 1
    assert out[0, 0] == 1.0


@pytest.mark.parametrize("seed", [1, 2])
def test_gradients_central_differences(seed):
    rng = np.random.default_rng(seed)
    ps = mlp.init_params(rng, 7, 9, 5)
    for k in range(1, 8, 2):
        ps[k] = rng.standard_normal(ps[k].shape) * 0.1
    X = rng.standard_normal((6, 7))
    Y = rng.standard_normal((6, 5))
    net = mlp.MLP(ps, quantize=False)
    loss, grads = net.loss_and_grads(X, Y)
    h = 1e-6
    for k in range(len(ps)):
        flat = ps[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            pp = [p.copy() for p in ps]
            pm = [p.copy() for p in ps]
            pp[k].reshape(-1)[idx] += h
            pm[k].reshape(-1)[idx] -= h
            fd = (mlp.MLP(pp, False).loss_and_grads(X, Y)[0] - mlp.MLP(pm, False).loss_and_grads(X, Y)[0]) / (2 * h)
            assert abs(fd - grads[k].reshape(-1)[idx]) < 1e-6 * max(1.0, abs(fd)), (k, idx)


def test_adam_matches_torch():
    rng = np.random.default_rng(3)
    ps = [rng.standard_normal((4, 3)), rng.standard_normal(4)]
    gs_seq = [[rng.standard_normal((4, 3)), rng.standard_normal(4)] for _ in range(5)]
    tp = [torch.tensor(p, requires_grad=True) for p in ps]
    opt = torch.optim.Adam(tp, lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m = [np.zeros_like(p) for p in ps]
    v = [np.zeros_like(p) for p in ps]
    cur = ps
    for t, gs in enumerate(gs_seq, start=1):
        for p, g in zip(tp, gs):
            p.grad = torch.tensor(g)
        opt.step()
        cur = mlp.adam_step(cur, gs, m, v, t, 1e-2)
    for a, b in zip(cur, tp):
        assert np.allclose(a, b.detach().numpy(), rtol=0, atol=1e-12)
