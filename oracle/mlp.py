"""Reference of the learned preconditioner's network (TEST ONLY).

The network: g = w3 . relu(W2 relu(W1 x + b1) + b2) + b3 with x in R^4,
hidden width 128; correction factor exp(clamp(g, -4, 4)); training loss over
rows  L = sum_r w_r (exp(clamp(g_r)) tj_r - e_r)^2  (no gradient through the
clamp where it is active). Plain NumPy in FP64; with `bf16=True` the operands
that the GPU feeds to its BF16 matrix cores (h1, W2 and dL/dz2) are rounded
to BF16 (round to nearest even) at the same points, so the GPU's FP32 result
can be compared to it closely. The weight blob layout: W1[128][4], b1[128],
W2[128][128], b2[128], w3[128], b3.
"""
from __future__ import annotations

import numpy as np

H = 128
NIN = 4
N_PARAMS = H * NIN + H + H * H + H + H + 1
CLAMP = 4.0


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    o = 0
    W1 = w[o:o + H * NIN].reshape(H, NIN); o += H * NIN
    b1 = w[o:o + H]; o += H
    W2 = w[o:o + H * H].reshape(H, H); o += H * H
    b2 = w[o:o + H]; o += H
    w3 = w[o:o + H]; o += H
    b3 = w[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, [b3]])


def bf16_round(a):
    """Round to BF16 (nearest even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(w, X, bf16=False):
    W1, b1, W2, b2, w3, b3 = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    h1m = bf16_round(h1) if bf16 else h1
    W2m = bf16_round(W2) if bf16 else W2
    z2 = h1m @ W2m.T + b2
    h2 = np.maximum(z2, 0.0)
    g = h2 @ w3 + b3
    return g, (X, z1, h1m, W2m, z2, h2)


def loss_grad(w, X, tj, e, wr, bf16=False):
    """Loss and gradient (same layout as the weight blob)."""
    W1, b1, W2, b2, w3, b3 = unpack(w)
    g, (X, z1, h1m, W2m, z2, h2) = forward(w, X, bf16)
    tj = np.asarray(tj, np.float64); e = np.asarray(e, np.float64); wr = np.asarray(wr, np.float64)
    gc = np.clip(g, -CLAMP, CLAMP)
    y = np.exp(gc) * tj
    d = y - e
    loss = np.sum(wr * d * d)
    dg = np.where((g > -CLAMP) & (g < CLAMP), 2.0 * wr * d * y, 0.0)
    gw3 = h2.T @ dg
    gb3 = dg.sum()
    dz2 = np.where(z2 > 0, dg[:, None] * w3[None, :], 0.0)
    gb2 = dz2.sum(0)
    dz2m = bf16_round(dz2) if bf16 else dz2
    gW2 = dz2m.T @ h1m
    dh1 = dz2m @ W2m
    dz1 = np.where(h1m > 0, dh1, 0.0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(0)
    return loss, pack(gW1, gb1, gW2, gb2, gw3, gb3)
