"""Learned preconditioner against the Jacobi form, with the committed trained
weights: on held-out instances drawn like the training set and on the
60000-dimensional test instance (40 target orbitals, N = 12, 8000
determinants, 50 states, 400 continuum orbitals, 40000 L2 functions), both
forms reach the same lowest 10 eigenpairs to residual 1e-8 on a matrix whose
sampled elements match the oracle. The measured outcome is asserted against
the committed expectation: the trained network gains nothing over the
Jacobi step on these inputs (iteration ratios between 0.8 and 1.25 were
measured), so the test requires the learned solve to stay within 25% of the
Jacobi iterations -- a regression guard, not a claim of gain. Non-finite
weights fall back to the Jacobi step on every row and the solve still
converges."""
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1709_03005_amd",
                       "mlp_weights.npy")


def _trained(cc):
    net = cc.Mlp(seed=0)
    net.set_weights(np.load(WEIGHTS))
    return net


def _sample_parity(inst, G, n=24, seed=5):
    D, Dc = inst.dim(), inst.n_cont_rows()
    rng = np.random.default_rng(seed)
    rows = np.concatenate([rng.integers(0, Dc, n), rng.integers(Dc, D, n), rng.integers(Dc, D, n)])
    cols = np.concatenate([rng.integers(0, Dc, n), rng.integers(0, Dc, n), rng.integers(Dc, D, n)])
    v, a, k = oracle.Oracle(inst).elements(rows, cols)
    g = G[rows, cols]
    ok, _ = oracle.tolerance_ok(g, v, a, k)
    assert ok.all(), [(int(r), int(c), g[i], v[i]) for i, (r, c) in enumerate(zip(rows, cols)) if not ok[i]][:5]


def _ab(cc, ctx, net, name, k=10, tol=1e-8):
    ev_j, x_j, inf_j, rc_j = ctx.davidson(k, tol=tol, max_iter=400)
    ctx.set_mlp(net)
    ev_m, x_m, inf_m, rc_m = ctx.davidson(k, tol=tol, max_iter=400, precond=cc.CCH_PRECOND_MLP)
    ctx.set_mlp(None)
    assert rc_j == cc.CCH_OK and rc_m == cc.CCH_OK
    print(f"[{name}] Jacobi {inf_j.iterations} it {1e3 * inf_j.seconds:.1f} ms | MLP {inf_m.iterations} it "
          f"{1e3 * inf_m.seconds:.1f} ms (fallbacks {inf_m.fallbacks}) | iteration gain "
          f"{inf_j.iterations / inf_m.iterations:.3f}x, time gain {inf_j.seconds / inf_m.seconds:.3f}x", flush=True)
    # the committed expectation: no gain, and no loss beyond 25% in iterations
    assert inf_m.iterations <= 1.25 * inf_j.iterations, (inf_m.iterations, inf_j.iterations)
    return (ev_j, x_j), (ev_m, x_m)


def _certify(G, ev, x, scale):
    r = G @ x.T - x.T * ev[None, :]
    assert np.linalg.norm(r, axis=0).max() < 2e-8
    assert np.all(np.diff(ev) >= -1e-12 * scale)


@pytest.mark.parametrize("i", [1000, 1001])
def test_ab_held_out(i):
    import paper_1709_03005_amd as cc
    inst = synth.learned_train(i)                 # seeds disjoint from the training draws
    print(f"[held-out {i}] D={inst.dim()}", flush=True)
    net = _trained(cc)
    with cc.from_instance(inst) as ctx:
        ctx.build()
        G = ctx.get_matrix()
        (ev_j, x_j), (ev_m, x_m) = _ab(cc, ctx, net, f"held-out {i}")
    net.close()
    _sample_parity(inst, G)
    scale = np.abs(ev_j).max()
    assert np.abs(ev_j - ev_m).max() <= 1e-10 * scale
    _certify(G, ev_j, x_j, scale)
    _certify(G, ev_m, x_m, scale)


def test_ab_learned_test_instance():
    import torch
    import paper_1709_03005_amd as cc
    inst = synth.learned_test()
    print(f"[learned-test] generated D={inst.dim()}", flush=True)
    net = _trained(cc)
    with cc.from_instance(inst, stream=torch.cuda.current_stream().cuda_stream) as ctx:
        ctx.build()
        print("[learned-test] built", flush=True)
        (ev_j, x_j), (ev_m, x_m) = _ab(cc, ctx, net, "learned-test")
        G = ctx.get_matrix()
    net.close()
    print("[learned-test] matrix on host", flush=True)
    _sample_parity(inst, G)
    scale = np.abs(ev_j).max()
    assert np.abs(ev_j - ev_m).max() <= 1e-10 * scale
    _certify(G, ev_j, x_j, scale)
    _certify(G, ev_m, x_m, scale)


def test_nonfinite_weights_fall_back():
    import paper_1709_03005_amd as cc
    inst = synth.small()
    w = np.linalg.eigvalsh(oracle.Oracle(inst).build())[:5]
    net = cc.Mlp(seed=0)
    net.set_weights(np.full(net.n_params, np.nan, np.float32))
    with cc.from_instance(inst) as ctx:
        ctx.build()
        ctx.set_mlp(net)
        ev, _, info, rc = ctx.davidson(5, tol=1e-9, precond=cc.CCH_PRECOND_MLP)
    net.close()
    assert rc == cc.CCH_OK
    assert info.fallbacks > 0
    assert np.all(np.abs(ev - w) <= 1e-10 * np.abs(w).max())
