"""Pins of the FP64 reference of the surrogate perceptron (oracle/mlp.py):
backward against central finite differences, GELU derivative against finite
differences, BF16 rounding against torch's conversion."""
import numpy as np
import torch

from oracle import mlp

K = [16, 256, 256, 256, 256]
N = [256, 256, 256, 256, 16]


def _net(rng, scale=1.0):
    Ws = [rng.standard_normal((n, k)) * np.sqrt(2.0 / k) * scale for k, n in zip(K, N)]
    bs = [rng.standard_normal(n) * 0.1 for n in N]
    return Ws, bs


def test_gelu_grad_fd():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(z), fd, atol=1e-8)


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(1000) * 10.0 ** rng.integers(-8, 8, 1000), [0.0, -0.0, 1.0, 3.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16_round(x), ref)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    Ws, bs = _net(rng)
    X = rng.uniform(-1, 1, (8, 16))
    label = rng.uniform(-2, 0, 8)
    lam = 0.3
    out, cache = mlp.forward(Ws, bs, X)
    loss, dout = mlp.loss_and_grad(out, label, lam)
    dWs, dbs, dX = mlp.backward(Ws, bs, cache, dout)

    def L(Ws_, bs_, X_):
        o, _ = mlp.forward(Ws_, bs_, X_)
        # second target held fixed at its value for the unperturbed output
        res = o[:, 0] - label
        tgt = np.log10(np.abs(out[:, 0] - label) + 1e-6)
        return np.mean(res ** 2 + lam * (o[:, 1] - tgt) ** 2)

    h = 1e-6
    for l in (0, 2, 4):
        for (i, j) in [(0, 0), (3, 5), (N[l] - 1, K[l] - 1), (1, 7)]:
            Wp = [w.copy() for w in Ws]; Wp[l][i, j] += h
            Wm = [w.copy() for w in Ws]; Wm[l][i, j] -= h
            fd = (L(Wp, bs, X) - L(Wm, bs, X)) / (2 * h)
            assert abs(fd - dWs[l][i, j]) <= 1e-6 * max(1.0, abs(fd)), (l, i, j, fd, dWs[l][i, j])
        for i in (0, N[l] // 2, N[l] - 1):
            bp = [b.copy() for b in bs]; bp[l][i] += h
            bm = [b.copy() for b in bs]; bm[l][i] -= h
            fd = (L(Ws, bp, X) - L(Ws, bm, X)) / (2 * h)
            assert abs(fd - dbs[l][i]) <= 1e-6 * max(1.0, abs(fd))
    for (r, c) in [(0, 0), (5, 11)]:
        Xp = X.copy(); Xp[r, c] += h
        Xm = X.copy(); Xm[r, c] -= h
        fd = (L(Ws, bs, Xp) - L(Ws, bs, Xm)) / (2 * h)
        assert abs(fd - dX[r, c]) <= 1e-6 * max(1.0, abs(fd))
