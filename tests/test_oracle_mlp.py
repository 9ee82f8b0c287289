"""Pins of the warm-start network oracle (CPU).

Gradients against central finite differences of the loss (FP64), Adam's
first step against its closed form (a step of -lr sign(g) up to eps), the
bfloat16 rounding against exactly representable values and ties, and a
short training run that must lower the loss on a smooth target.
"""
import numpy as np

from oracle import mlp as M


def test_bf16_rounding():
    exact = np.array([1.0, -2.5, 0.0, 3.0 * 2 ** -20, 65280.0])
    assert np.array_equal(M.bf16_round(exact), exact)
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties go to even (1.0)
    assert M.bf16_round(np.array([1 + 2 ** -8]))[0] == 1.0
    assert M.bf16_round(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6
    assert M.bf16_round(np.array([1 + 2 ** -8 + 2 ** -12]))[0] == 1 + 2 ** -7
    x = np.random.default_rng(0).standard_normal(1000)
    assert np.abs(M.bf16_round(x) / x - 1).max() <= 2 ** -8   # half an ulp of 8 bits


def test_gradients_match_finite_differences(rng):
    sizes = (13, 6, 5, 4, 3)
    params = M.init_params(1, sizes)
    for l in params:
        l[1] += 0.1 * rng.standard_normal(l[1].shape)
    x = rng.standard_normal((7, 13))
    t = rng.standard_normal((7, 3))
    _, grads = M.loss_and_grads(params, x, t)
    h = 1e-6
    for li in range(4):
        for j in range(2):
            p = params[li][j]
            it = np.nditer(p, flags=["multi_index"])
            for _ in it:
                idx = it.multi_index
                old = p[idx]
                p[idx] = old + h
                lp, _ = M.loss_and_grads(params, x, t)
                p[idx] = old - h
                lm, _ = M.loss_and_grads(params, x, t)
                p[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - grads[li][j][idx]) < 1e-7 * max(1.0, abs(fd)), (li, j, idx)


def test_adam_first_step_and_training(rng):
    sizes = (13, 16, 16, 16, 3)
    params = M.init_params(2, sizes)
    x = rng.standard_normal((256, 13))
    t = np.stack([np.sin(x[:, 0]), x[:, 1] * x[:, 2], 0.5 * x[:, 3]], axis=1)
    l0, g = M.loss_and_grads(params, x, t)
    before = [[p.copy() for p in l] for l in params]
    state = {}
    M.adam_step(params, g, state, lr=1e-3)
    for l in range(4):
        for j in range(2):
            step = params[l][j] - before[l][j]
            gg = g[l][j]
            # first step: m/(1-b1) = g, v/(1-b2) = g^2 -> -lr g/(|g| + eps)
            assert np.allclose(step, -1e-3 * gg / (np.abs(gg) + 1e-8), rtol=1e-12, atol=1e-18)
    for _ in range(300):
        _, g = M.loss_and_grads(params, x, t)
        M.adam_step(params, g, state, lr=3e-3)
    l1, _ = M.loss_and_grads(params, x, t)
    assert l1 < 0.2 * l0
