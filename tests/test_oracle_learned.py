"""Pins of the learned-scorer oracle (CPU only).

  * bfloat16 rounding equals torch's float32 -> bfloat16 conversion (round to nearest even);
  * MLP gradients equal central finite differences (float64, unrounded) and torch float64 autograd, with and
    without the bfloat16 rounding (straight-through for the rounded values);
  * one Adam step equals torch.optim.Adam;
  * features: one-hot type, the move's bits, demand and return window, costs and setup distances.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import learned as L
from paper_1704_05132_amd.instances import draw_instance


def test_bf16_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 3, 5000), rng.normal(0, 1e-3, 1000), [0.0, -0.0, 1.0, 65504.0, 3.1415926]])
    x = x.astype(np.float32)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert (L.bf16(x).view(np.uint32) == ref.view(np.uint32)).all()


def _torch_loss(X, y, params, quantize):
    tp = [torch.tensor(p.astype(np.float64), requires_grad=True) for p in params]

    def q(t):
        if not quantize:
            return t
        r = torch.tensor(L.bf16(t.detach().numpy().astype(np.float32)).astype(np.float64))
        return t + (r - t).detach()

    W1, b1, W2, b2, W3, b3 = tp
    a0 = q(torch.tensor(X.astype(np.float64)))
    h1 = torch.relu(a0 @ q(W1) + b1)
    h2 = torch.relu(q(h1) @ q(W2) + b2)
    s = (q(h2) @ q(W3) + b3)[:, 0]
    loss = ((s - torch.tensor(y.astype(np.float64))) ** 2).mean()
    loss.backward()
    return float(loss), [t.grad.numpy() for t in tp]


@pytest.mark.parametrize("quantize", [False, True])
def test_gradients_match_torch_autograd(quantize):
    rng = np.random.default_rng(2)
    X = rng.normal(0, 1, (37, 16)).astype(np.float32)
    y = rng.normal(0, 1, 37)
    params = L.init_params(3)
    params[1] = rng.normal(0, 0.1, 64).astype(np.float32)
    loss, grads = L.loss_and_grads(X, y, params, quantize)
    tl, tg = _torch_loss(X, y, params, quantize)
    assert abs(loss - tl) < 1e-9 * max(1, abs(tl))
    for g, t in zip(grads, tg):
        assert np.allclose(np.reshape(g, t.shape), t, rtol=1e-9, atol=1e-12)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(4)
    X = rng.normal(0, 1, (9, 16)).astype(np.float32)
    y = rng.normal(0, 1, 9)
    params = [p.astype(np.float64) for p in L.init_params(5)]
    params[1] = rng.normal(0, 0.1, 64)
    _, grads = L.loss_and_grads(X, y, [p.astype(np.float32) for p in params], quantize=False)
    f32 = lambda ps: [p.astype(np.float32) for p in ps]
    for pi in range(6):
        flat = params[pi].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            h = 1e-2
            up = [p.copy() for p in params]
            dn = [p.copy() for p in params]
            up[pi].reshape(-1)[idx] += h
            dn[pi].reshape(-1)[idx] -= h
            lu, _ = L.loss_and_grads(X, y, f32(up), quantize=False)
            ld, _ = L.loss_and_grads(X, y, f32(dn), quantize=False)
            fd = (lu - ld) / (2 * h)
            g = np.reshape(grads[pi], -1)[idx]
            assert abs(fd - g) <= 2e-3 * max(1.0, abs(g)), (pi, idx, fd, g)


def test_adam_matches_torch():
    rng = np.random.default_rng(6)
    params = L.init_params(7)
    grads = [rng.normal(0, 1, p.shape) for p in params]
    m = [np.zeros(p.shape) for p in params]
    v = [np.zeros(p.shape) for p in params]
    p1, m1, v1 = L.adam_step(params, grads, m, v, 1, lr=1e-2)
    p2, _, _ = L.adam_step(p1, grads, m1, v1, 2, lr=1e-2)
    tp = [torch.tensor(p.astype(np.float64), requires_grad=True) for p in params]
    opt = torch.optim.Adam(tp, lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for _ in range(2):
        opt.zero_grad()
        for t, g in zip(tp, grads):
            t.grad = torch.tensor(g)
        opt.step()
    for a, t in zip(p2, tp):
        assert np.allclose(a, t.detach().numpy().astype(np.float32), rtol=1e-6, atol=1e-7)


def test_features_of_a_hand_example():
    inst = draw_instance(np.random.default_rng(8), 1, 5)
    inst.D[0] = [10, 20, 0, 30, 5]
    inst.R[0] = [5, 5, 5, 5, 0]
    inst.kM[0], inst.kR[0], inst.hM[0], inst.hR[0] = 100, 50, 2, 1
    zM = np.array([1, 0, 0, 0, 0], np.uint8)
    zR = np.array([0, 0, 0, 1, 0], np.uint8)
    f = L.move_features(inst, 0, zM, zR, 5 + 3)        # flip zR at t = 3
    assert list(f[:4]) == [0, 1, 0, 0]
    assert f[4] == 0 and f[5] == 1
    assert f[6] == np.float32(30) / np.float32(200) and f[7] == np.float32(5) / np.float32(200)
    assert f[8] == 0.0 and f[9] == np.float32(5) / np.float32(200)
    assert f[10] == np.float32(0.05) and f[12] == np.float32(0.25)
    assert f[14] == 0.0                                 # setup at t itself
    assert f[15] == np.float32(2) / np.float32(5)      # no later setup: T - t
    g = L.move_features(inst, 0, zM, zR, 3 * 5 - 3)    # swap zM at t = 2
    assert list(g[:4]) == [0, 0, 1, 0]
    assert g[14] == np.float32(2) / np.float32(5) and g[15] == np.float32(1) / np.float32(5)
    assert L.move_features(inst, 0, zM, zR, 0)[8] == 0.0   # no D(t-1) at t = 0
    z0 = np.zeros(5, np.uint8)
    h = L.move_features(inst, 0, z0, z0, 1)
    assert h[14] == 1.0 and h[15] == 0.8                # no setup at all
