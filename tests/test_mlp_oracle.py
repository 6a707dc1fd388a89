"""CPU pins of the network reference: its analytic gradient against central
finite differences (FP64, no BF16 rounding), and the BF16 rounding helper
against exactly representable cases."""
import numpy as np

from oracle import mlp


def _data(n=37, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 4))
    tj = rng.standard_normal(n)
    e = rng.standard_normal(n) * 0.5
    wr = rng.random(n)
    w = rng.standard_normal(mlp.N_PARAMS) * 0.1
    return w, X, tj, e, wr


def test_gradient_matches_finite_differences():
    w, X, tj, e, wr = _data()
    L, G = mlp.loss_grad(w, X, tj, e, wr)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.integers(0, 512, 5), rng.integers(512, 640, 3),
                          rng.integers(640, 640 + 16384, 8), rng.integers(17024, 17281, 5), [17280]])
    h = 1e-6
    for i in idx:
        wp = w.copy(); wp[i] += h
        wm = w.copy(); wm[i] -= h
        fd = (mlp.loss_grad(wp, X, tj, e, wr)[0] - mlp.loss_grad(wm, X, tj, e, wr)[0]) / (2 * h)
        assert abs(fd - G[i]) <= 1e-6 * max(1.0, abs(G[i])), (i, fd, G[i])


def test_clamp_blocks_gradient():
    w, X, tj, e, wr = _data(5)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(w)
    w = mlp.pack(W1, b1, W2, b2, w3, 10.0)          # g > 4 for every row
    g, _ = mlp.forward(w, X)
    assert np.all(g > mlp.CLAMP)
    _, G = mlp.loss_grad(w, X, tj, e, wr)
    assert np.all(G == 0)


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 0.0])
    r = mlp.bf16_round(x)
    # 1 + 2^-8 is a tie -> even (1.0); 1 + 3*2^-8 is a tie -> even (1 + 2^-6)
    np.testing.assert_array_equal(r, [1.0, 1.0 + 2 ** -7, 1.0, 1.0 + 2 ** -6, -2.5, 0.0])
