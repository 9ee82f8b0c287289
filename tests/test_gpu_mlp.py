"""The warm-start network's kernels against the FP64 oracle (oracle.mlp).

Forward outputs and loss gradients are compared with the oracle run with the
same bfloat16 roundings (the kernels' storage points), so what remains is
FP32 accumulation order; the plain FP64 network is checked at the looser
bfloat16 level.  Adam's arithmetic is checked on the kernels' own gradients.
The guided GMRES start takes the least-squares step along a proposed
correction: 1 along the exact correction, 0 against it.
"""
import numpy as np
import pytest

from oracle import mlp as M

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_1109_6587_amd as G  # noqa: E402

DEV = torch.device("cuda:0")


def pack(params):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params]).astype(np.float32)


def unpack(v):
    out, o = [], 0
    for i in range(4):
        a, b = M.SIZES[i], M.SIZES[i + 1]
        W = v[o:o + a * b].reshape(b, a).astype(np.float64)
        o += a * b
        out.append([W, v[o:o + b].astype(np.float64)])
        o += b
    assert o == v.size
    return out


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def net():
    rng = np.random.default_rng(11)
    params = M.init_params(5)
    for l in params:
        l[1] += 0.1 * rng.standard_normal(l[1].shape)
    v = pack(params)
    return unpack(v), v, rng


def test_packed_size():
    assert pack(M.init_params(0)).size == G.MLP_PARAMS


@pytest.mark.parametrize("n", [1, 63, 300, 2500])
def test_forward(net, n):
    params, v, rng = net
    print(f"mlp forward n={n}", flush=True)
    x = rng.standard_normal((n, 13)).astype(np.float32)
    mlp = G.MLP(4096, torch.as_tensor(v, device=DEV))
    y = mlp.forward(torch.as_tensor(x, device=DEV)).cpu().numpy()
    ref, _ = M.forward(params, x.astype(np.float64), bf16=True)
    assert rel(y, ref) < 2e-4
    exact, _ = M.forward(params, x.astype(np.float64))
    assert rel(y, exact) < 3e-2
    dq = mlp.predict(torch.as_tensor(x, device=DEV), 0.5).cpu().numpy()
    assert np.array_equal(dq, 0.5 * y.astype(np.float64))


@pytest.mark.parametrize("n", [300, 2500])
def test_gradients(net, n):
    params, v, rng = net
    print(f"mlp gradients n={n}", flush=True)
    x = rng.standard_normal((n, 13)).astype(np.float32)
    t = (0.3 * rng.standard_normal((n, 3))).astype(np.float32)
    mlp = G.MLP(4096, torch.as_tensor(v, device=DEV))
    loss, g = mlp.gradients(torch.as_tensor(x, device=DEV), torch.as_tensor(t, device=DEV))
    gl = unpack(g.cpu().numpy())
    rloss, rg = M.loss_and_grads(params, x.astype(np.float64), t.astype(np.float64), bf16=True)
    assert abs(loss - rloss) < 1e-5 * rloss
    for l in range(4):
        for j in range(2):
            assert rel(gl[l][j], rg[l][j]) < 2e-3, (l, j)
    _, eg = M.loss_and_grads(params, x.astype(np.float64), t.astype(np.float64))
    for l in range(4):
        assert rel(gl[l][0], eg[l][0]) < 5e-2, l


def test_adam_steps(net):
    """Three steps: the oracle's Adam, fed the kernels' own gradients and
    starting from the kernels' parameters, lands on the same parameters."""
    params, v, rng = net
    print("mlp adam", flush=True)
    n = 700
    x = torch.as_tensor(rng.standard_normal((n, 13)).astype(np.float32), device=DEV)
    t = torch.as_tensor((0.3 * rng.standard_normal((n, 3))).astype(np.float32), device=DEV)
    mlp = G.MLP(1024, torch.as_tensor(v, device=DEV))
    state = {}
    for k in range(3):
        _, g = mlp.gradients(x, t)
        ref = unpack(mlp.get_params().cpu().numpy())
        mlp.train_step(x, t, 1e-3)
        M.adam_step(ref, unpack(g.cpu().numpy()), state, lr=1e-3)
        assert np.abs(pack(ref) - mlp.get_params().cpu().numpy()).max() < 1e-6, k


def test_training_lowers_loss():
    print("mlp training", flush=True)
    rng = np.random.default_rng(3)
    n = 4096
    x = rng.standard_normal((n, 13)).astype(np.float32)
    t = np.stack([np.sin(x[:, 0]), x[:, 1] * x[:, 2], 0.5 * x[:, 3] - x[:, 9]], 1).astype(np.float32)
    X, T = torch.as_tensor(x, device=DEV), torch.as_tensor(t, device=DEV)
    mlp = G.MLP(n, torch.as_tensor(pack(M.init_params(2)), device=DEV))
    l0 = mlp.gradients(X, T)[0]
    for _ in range(300):
        mlp.train_step(X, T, 2e-3)
    l1 = mlp.gradients(X, T)[0]
    assert l1 < 0.05 * l0


def test_features():
    print("mlp features", flush=True)
    rng = np.random.default_rng(4)
    npd, nd = 50, 3
    nodes = rng.standard_normal((npd * nd, 3)) + 5
    nrm = rng.standard_normal(nodes.shape)
    lap = rng.standard_normal(nodes.shape)
    qp = rng.standard_normal(nodes.shape)
    dqp = rng.standard_normal(nodes.shape)
    sc = [1, 1, 1, 1, 1, 1, 0.5, 10, 10, 10, 3, 3, 3]
    t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=DEV)  # noqa: E731
    mlp = G.MLP(1024)
    X = mlp.features(t(nodes), t(nrm), t(lap), t(qp), t(dqp), npd, sc).cpu().numpy()
    ref = M.node_features(nodes, nrm, lap, qp, dqp, npd, sc)
    assert np.abs(X - ref).max() <= 1e-6 * np.abs(ref).max()
