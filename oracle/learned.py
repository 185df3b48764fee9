"""Oracle of the learned move scorer — TEST INFRASTRUCTURE ONLY (tests, smoke, benchmark baseline).

Move features (16 float32 values per move, computed from integers with float32 arithmetic so that any
implementation following the same recipe gets identical bits):
   0-3  one-hot move type: flip zM, flip zR, swap zM, swap zR
   4,5  current setup bits zM(t), zR(t) at the move's period t
   6,7  D(t) / 200, R(t) / 200
   8,9  D(t-1) / 200, D(t+1) / 200 (0 outside the horizon)
  10-13 kM / 2000, kR / 2000, hM / 8, hR / 8
  14    (t - p) / T, p the last period <= t with a setup of either type in the current pattern (1 if none)
  15    (n - t) / T, n the first period > t with a setup of either type (T if none)
Features 14 and 15 place the move inside its setup interval; unlike the interval's inventories they need
no pass over the horizon, so a lane gets them from its own bit rows in a few operations.

Scorer: an MLP 16 -> 64 -> 64 -> 1 with ReLU, weights rounded to bfloat16 (round to nearest even) and the
inputs of every layer rounded to bfloat16, products accumulated in float64 here (float32 on the device).
Training target: the move's cost change divided by TARGET_SCALE; lower scores rank first.  Loss: mean
squared error.  Everything here is float64 numpy; its gradients are pinned by finite differences and by
torch's float64 autograd (tests/test_oracle_learned.py).
"""
from __future__ import annotations

import numpy as np


N_FEAT = 16
H = 64
TARGET_SCALE = 1000.0
LAYERS = ((N_FEAT, H), (H, H), (H, 1))


# ------------------------------------------------------------------------------------------------------
# features
# ------------------------------------------------------------------------------------------------------
def _f32(x):
    return np.float32(x)


def move_type(T, l):
    return 0 if l < T else 1 if l < 2 * T else 2 if l < 3 * T else 3


def move_features(inst, k, zM_row, zR_row, l):
    """Features of local slot l of product k for the given current rows (float32[16])."""
    T = inst.T
    ty = move_type(T, l)
    t = l - ty * T
    D, R = inst.D[k], inst.R[k]
    setup = [bool(zM_row[u]) or bool(zR_row[u]) for u in range(T)]
    prev = next((u for u in range(t, -1, -1) if setup[u]), None)
    nxt = next((u for u in range(t + 1, T) if setup[u]), T)
    f = np.zeros(N_FEAT, np.float32)
    f[ty] = 1.0
    f[4] = _f32(zM_row[t])
    f[5] = _f32(zR_row[t])
    f[6] = _f32(D[t]) / _f32(200)
    f[7] = _f32(R[t]) / _f32(200)
    f[8] = _f32(D[t - 1]) / _f32(200) if t > 0 else _f32(0)
    f[9] = _f32(D[t + 1]) / _f32(200) if t + 1 < T else _f32(0)
    f[10] = _f32(inst.kM[k]) / _f32(2000)
    f[11] = _f32(inst.kR[k]) / _f32(2000)
    f[12] = _f32(inst.hM[k]) / _f32(8)
    f[13] = _f32(inst.hR[k]) / _f32(8)
    f[14] = _f32(t - prev) / _f32(T) if prev is not None else _f32(1)
    f[15] = _f32(nxt - t) / _f32(T)
    return f


# ------------------------------------------------------------------------------------------------------
# bfloat16 rounding (round to nearest, ties to even) of float32 values
# ------------------------------------------------------------------------------------------------------
def bf16(x):
    a = np.ascontiguousarray(np.asarray(x, np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    return np.where(np.isnan(a), a, out).astype(np.float32)


# ------------------------------------------------------------------------------------------------------
# MLP
# ------------------------------------------------------------------------------------------------------
def _q(quantize):
    """Rounding applied to weights and layer inputs: bfloat16 (as float64 values) or none."""
    if quantize:
        return lambda a: bf16(np.asarray(a, np.float32)).astype(np.float64)
    return lambda a: np.asarray(a, np.float64)


def init_params(seed):
    """He-uniform weights, zero biases: [W1 (16x64), b1, W2 (64x64), b2, W3 (64x1), b3] as float32."""
    rng = np.random.default_rng(seed)
    ps = []
    for fan_in, fan_out in LAYERS:
        lim = np.sqrt(6.0 / fan_in)
        ps.append(rng.uniform(-lim, lim, (fan_in, fan_out)).astype(np.float32))
        ps.append(np.zeros(fan_out, np.float32))
    return ps


def forward(X, params, quantize=True):
    """Scores of feature rows X [N,16] and the cache for backward.  With `quantize`, weights and layer
    inputs are rounded to bfloat16 first (the device arithmetic); sums are float64."""
    q = _q(quantize)
    W1, b1, W2, b2, W3, b3 = params
    a0 = q(X)
    z1 = a0 @ q(W1) + b1.astype(np.float64)
    h1 = np.maximum(z1, 0.0)
    a1 = q(h1)
    z2 = a1 @ q(W2) + b2.astype(np.float64)
    h2 = np.maximum(z2, 0.0)
    a2 = q(h2)
    out = a2 @ q(W3) + b3.astype(np.float64)
    return out[:, 0], (a0, z1, a1, z2, a2)


def loss_and_grads(X, y, params, quantize=True):
    """Mean squared error of the scores against y, and its gradients with respect to every parameter
    (the rounded weights and activations are treated as their float values: straight-through)."""
    q = _q(quantize)
    W1, b1, W2, b2, W3, b3 = params
    s, (a0, z1, a1, z2, a2) = forward(X, params, quantize)
    N = len(y)
    d = (s - np.asarray(y, np.float64)) / N
    loss = float(np.mean((s - np.asarray(y, np.float64)) ** 2))
    ds = 2.0 * d                                  # dL/ds  [N]
    gW3 = a2.T @ ds[:, None]
    gb3 = np.array([ds.sum()])
    dz2 = (ds[:, None] @ q(W3).T) * (z2 > 0)
    gW2 = a1.T @ dz2
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ q(W2).T) * (z1 > 0)
    gW1 = a0.T @ dz1
    gb1 = dz1.sum(0)
    return loss, [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_step(params, grads, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) in float64, returning float32 parameters and the new moments."""
    out_p, out_m, out_v = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = b1 * mm + (1 - b1) * g
        vv = b2 * vv + (1 - b2) * g * g
        mh = mm / (1 - b1 ** step)
        vh = vv / (1 - b2 ** step)
        out_p.append((p.astype(np.float64) - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32))
        out_m.append(mm)
        out_v.append(vv)
    return out_p, out_m, out_v
