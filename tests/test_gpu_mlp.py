"""Learned preconditioner: the GPU network's forward pass and gradient against
the NumPy reference with the same BF16 rounding points (oracle/mlp.py, itself
pinned by finite differences), training on the device reduces the loss, and
MLP-preconditioned Davidson reaches the same eigenpairs as the Jacobi form."""
import numpy as np
import pytest

import oracle
import synth
from oracle import mlp as ref

pytestmark = pytest.mark.gpu


def _net(seed=3, scale=0.15):
    import paper_1709_03005_amd as cc
    net = cc.Mlp(seed=seed)
    rng = np.random.default_rng(seed)
    w = (rng.standard_normal(net.n_params) * scale).astype(np.float32)
    net.set_weights(w)
    return net, w.astype(np.float64)


def _rows(n, seed=4):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 4)).astype(np.float32)
    tj = rng.standard_normal(n).astype(np.float32)
    e = (tj * np.exp(0.5 * np.sin(X[:, 0]))).astype(np.float32)
    wr = rng.random(n).astype(np.float32)
    return X, tj, e, wr


def test_forward_matches_reference():
    net, w = _net()
    X, *_ = _rows(1000)                       # 15 full tiles of 64 and a ragged one
    g = net.forward(X)
    gr, _ = ref.forward(w, X.astype(np.float64), bf16=True)
    assert np.abs(g - gr).max() <= 1e-3 * max(1.0, np.abs(gr).max())
    net.close()


def test_gradient_matches_reference():
    net, w = _net()
    X, tj, e, wr = _rows(3000)
    loss, G = net.grad(X, tj, e, wr)
    Lr, Gr = ref.loss_grad(w, X, tj, e, wr, bf16=True)
    assert abs(loss - Lr) <= 1e-4 * abs(Lr)
    blocks = [(0, 512), (512, 640), (640, 17024), (17024, 17152), (17152, 17280), (17280, 17281)]
    for a, b in blocks:
        rel = np.linalg.norm(G[a:b] - Gr[a:b]) / max(np.linalg.norm(Gr[a:b]), 1e-12)
        assert rel <= 5e-3, (a, b, rel)
    # determinism of the reduction
    loss2, G2 = net.grad(X, tj, e, wr)
    assert loss2 == loss and np.array_equal(G2, G)
    net.close()


def test_training_reduces_loss():
    net, _ = _net(scale=0.05)
    X, tj, e, wr = _rows(20000, seed=9)
    l0 = net.train_step(X, tj, e, wr, lr=1e-3)
    for _ in range(150):
        l = net.train_step(X, tj, e, wr, lr=1e-3)
    print(f"[mlp] loss {l0:.4f} -> {l:.4f}")
    assert l < 0.5 * l0
    net.close()


@pytest.mark.parametrize("name", ["tiny", "small"])
def test_mlp_davidson_converges(name):
    import paper_1709_03005_amd as cc
    inst = synth.CONFIGS[name]()
    H = oracle.Oracle(inst).build()
    w = np.linalg.eigvalsh(H)[:5]
    net = cc.Mlp(seed=1)                       # untrained: starts close to the Jacobi step
    with cc.from_instance(inst) as ctx:
        ctx.build()
        ctx.set_mlp(net)
        ev, vec, info, rc = ctx.davidson(5, tol=1e-9, precond=cc.CCH_PRECOND_MLP)
        ev_j, _, info_j, _ = ctx.davidson(5, tol=1e-9)
        X = ctx.mlp_features(float(ev[0]))
    assert rc == cc.CCH_OK
    assert np.all(np.abs(ev - w) <= 1e-10 * np.abs(w).max())
    print(f"[{name}] iterations MLP {info.iterations} Jacobi {info_j.iterations}, fallbacks {info.fallbacks}")
    assert X.shape == (inst.dim(), 4) and np.isfinite(X).all()
    assert set(np.unique(X[:, 3])) <= {0.0, 1.0}
    net.close()
