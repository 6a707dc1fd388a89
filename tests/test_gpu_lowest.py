"""The Davidson pairs are the lowest ones, on the large-matrix solver path
(from D = 20000 on: basis limit 96, the seeded first block, and restarts
that keep the previous iteration's Ritz vectors). The
half-size precision shape (D = 20000, two-word determinants) is built on the
GPU, its sampled elements of every block class are checked against the
oracle, and k + 1 = 11 pairs are asked for. Each returned pair has a
residual below 2e-8 on the host copy of the matrix; Sylvester's law of
inertia then decides the rest: an LDL^T factorisation (LAPACK dsytrf,
Bunch-Kaufman pivoting) of H - sigma I with sigma halfway between theta_10
and theta_11 must show exactly 10 negative eigenvalues in its block-diagonal
factor. With the residual bound this proves that theta_1..theta_10
approximate the 10 lowest eigenvalues of H (Sec. 3.2: the solve is for the
lowest eigenpairs)."""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import negative_inertia


def test_negative_inertia_small():
    """The counting rule itself, against eigvalsh on random symmetric
    matrices with 2x2 pivots forced by a zero diagonal."""
    rng = np.random.default_rng(3)
    for n in (1, 2, 7, 64, 300):
        A = rng.standard_normal((n, n))
        A = A + A.T
        np.fill_diagonal(A, 0.0)
        want = int((np.linalg.eigvalsh(A) < 0).sum())
        assert negative_inertia(A.copy()) == want


@pytest.mark.gpu
def test_lowest_k_by_inertia():
    import torch
    import time
    import paper_1709_03005_amd as cc
    inst = synth.mid()
    D, Dc = inst.dim(), inst.n_cont_rows()
    k = 10
    print(f"[lowest] generated D={D}", flush=True)
    with cc.from_instance(inst, stream=torch.cuda.current_stream().cuda_stream) as ctx:
        ctx.build()
        G = ctx.get_matrix()
        ev, vec, info, rc = ctx.davidson(k + 1, tol=1e-8)
    print(f"[lowest] davidson rc={rc} iters={info.iterations} restarts={info.restarts} "
          f"previous-vector directions kept={info.prev_kept}", flush=True)
    assert rc == cc.CCH_OK
    assert info.restarts == 0 or info.prev_kept > 0   # the default from a basis of 96: previous Ritz vectors kept
    assert np.abs(G).max() > 0
    rng = np.random.default_rng(7)
    rows = np.concatenate([rng.integers(0, Dc, 16), rng.integers(Dc, D, 16), rng.integers(Dc, D, 16)])
    cols = np.concatenate([rng.integers(0, Dc, 16), rng.integers(0, Dc, 16), rng.integers(Dc, D, 16)])
    v, a, kk = oracle.Oracle(inst).elements(rows, cols)
    ok, _ = oracle.tolerance_ok(G[rows, cols], v, a, kk)
    assert ok.all()
    r = np.linalg.norm(G @ vec.T - vec.T * ev[None, :], axis=0)
    assert r.max() < 2e-8, r
    assert np.abs(vec @ vec.T - np.eye(k + 1)).max() < 1e-10
    gap = ev[k] - ev[k - 1]
    assert gap > 1e-6, gap        # sigma sits well clear of both Ritz values
    sigma = 0.5 * (ev[k - 1] + ev[k])
    G[np.diag_indices(D)] -= sigma
    t0 = time.time()
    neg = negative_inertia(G)
    print(f"[lowest] theta_{k} = {ev[k - 1]:.12f}, theta_{k + 1} = {ev[k]:.12f}, "
          f"eigenvalues below sigma: {neg} (LDL^T {time.time() - t0:.1f} s)", flush=True)
    assert neg == k
