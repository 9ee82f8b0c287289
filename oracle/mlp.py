"""FP64 oracle of the warm-start network: a per-node MLP and its training.

TEST INFRASTRUCTURE ONLY (see the package header).

Network (the learned warm start of the Fredholm solve; not in the paper,
whose warm start is the previous stage's density, Sec. 5):
    h0 = x (13 features), z_l = W_l h_{l-1} + b_l, h_l = silu(z_l) (l = 1..3),
    y = W_4 h_3 + b_4  (3 outputs),  silu(z) = z / (1 + exp(-z)),
loss = mean over samples and outputs of (y - t)^2, minimised by Adam
(Kingma & Ba 2015: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
w -= lr (m / (1 - b1^k)) / (sqrt(v / (1 - b2^k)) + eps)).

``bf16=True`` rounds to bfloat16 (round to nearest even) exactly the values
the device kernels store in bfloat16: the input, the weights used in
products, every pre-activation z_l (from which silu' is taken) and
activation h_l, the output gradient dL/dy and every back-propagated dL/dz_l.
Products and sums stay in high precision, so the two differ only by the
accumulation order of FP32 sums (and rare rounding-boundary flips).
"""
from __future__ import annotations

import numpy as np

SIZES = (13, 128, 128, 128, 3)


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_params(seed, sizes=SIZES):
    """He-uniform weights, zero biases: W_l ~ U(-a, a), a = sqrt(6 / fan_in)
    (drawn with numpy's default_rng(seed), layer by layer, W as (out, in))."""
    rng = np.random.default_rng(seed)
    params = []
    for i in range(len(sizes) - 1):
        a = np.sqrt(6.0 / sizes[i])
        params.append([rng.uniform(-a, a, size=(sizes[i + 1], sizes[i])), np.zeros(sizes[i + 1])])
    return params


def _identity(a):
    return a


def forward(params, x, bf16=False):
    """Returns (y, cache) for inputs x (n, 13)."""
    rnd = bf16_round if bf16 else _identity
    h = rnd(x)
    hs, zs = [h], []
    for li, (W, b) in enumerate(params):
        z = h @ rnd(W).T + b
        if li == len(params) - 1:
            return z, (hs, zs)
        zs.append(rnd(z))
        h = rnd(silu(z))
        hs.append(h)
    raise AssertionError


def loss_and_grads(params, x, t, bf16=False):
    """Mean squared error and its gradients (list of [dW, db])."""
    rnd = bf16_round if bf16 else _identity
    y, (hs, zs) = forward(params, x, bf16)
    diff = y - t
    loss = np.mean(diff ** 2)
    dz = rnd(2.0 * diff / diff.size)
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W = rnd(params[li][0])
        grads[li] = [dz.T @ hs[li], dz.sum(axis=0)]
        if li > 0:
            dz = rnd((dz @ W) * silu_grad(zs[li - 1]))
    return loss, grads


def adam_step(params, grads, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place; state = {"k": steps so far, "m": [...], "v": [...]}."""
    if not state:
        state.update(k=0, m=[[np.zeros_like(p) for p in l] for l in params],
                     v=[[np.zeros_like(p) for p in l] for l in params])
    state["k"] += 1
    k = state["k"]
    for l, (pl, gl) in enumerate(zip(params, grads)):
        for j in range(2):
            m = state["m"][l][j] = b1 * state["m"][l][j] + (1 - b1) * gl[j]
            v = state["v"][l][j] = b2 * state["v"][l][j] + (1 - b2) * gl[j] ** 2
            pl[j] -= lr * (m / (1 - b1 ** k)) / (np.sqrt(v / (1 - b2 ** k)) + eps)
    return params


def node_features(nodes, normals, lap, q_prev, dq_prev, nodes_per_drop, scales):
    """(n, 13) inputs: position relative to the drop's centroid (mean of its
    nodes), normal, curvature term -(Lap x . n), previous density and its last
    change; each column multiplied by scales[k]."""
    n = nodes.shape[0]
    cen = nodes.reshape(n // nodes_per_drop, nodes_per_drop, 3).mean(axis=1)
    rel = nodes - np.repeat(cen, nodes_per_drop, axis=0)
    c = -np.einsum("ij,ij->i", lap, normals)
    f = np.concatenate([rel, normals, c[:, None], q_prev, dq_prev], axis=1)
    return f * np.asarray(scales, dtype=np.float64)[None, :]
