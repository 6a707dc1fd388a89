"""Every eigenpair of a dense symmetric matrix (cch_eig_all; Sec. 3.2 notes
that often all eigenvectors are required): eigenvalues against LAPACK
(numpy eigh / eigvalsh) within 1e-10 of the spectral radius, eigenvectors by
residual ||A v - lambda v|| and orthonormality within 1e-10 (scaled by the
spectral radius), and by overlap with LAPACK's where the eigenvalue is well
separated. Random matrices of sizes 1 to 1000 (one to many 32-reflector
panels and 128-reflector back-transformation blocks, ragged tails: 66 gives
a block of 65, 130 a last block of one) and of sizes 4500 (the tiled product of the trailing
block, then the row pass) and 8300 (on the device), a diagonal matrix of
size 3300 (every column already reduced, through both passes), matrices with exactly repeated and tightly clustered
eigenvalues, a diagonal and a zero matrix, the built contracted matrices of
the tiny and small instances and of the medium one (D = 8000), and device
arrays."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _check(M, w, V, tol=1e-10, lapack_vectors=True):
    n = M.shape[0]
    wl, vl = np.linalg.eigh(M)
    scale = max(np.abs(wl).max(), 1e-300)
    assert np.all(np.diff(w) >= 0)
    assert np.abs(w - wl).max() <= tol * scale, np.abs(w - wl).max() / scale
    if V is not None:
        assert np.abs(V @ V.T - np.eye(n)).max() <= tol * max(1.0, n / 100)
        R = M @ V.T - V.T * w[None, :]
        assert np.abs(R).max() <= tol * scale
        if lapack_vectors:
            gaps = np.minimum(np.diff(wl, prepend=-np.inf), np.diff(wl, append=np.inf))
            sep = gaps > 1e-6 * scale
            ov = np.abs(np.sum(V.T * vl, axis=0))
            assert np.all(np.abs(ov[sep] - 1.0) < 1e-8)


@pytest.mark.parametrize("n", [1, 2, 3, 31, 32, 33, 64, 66, 100, 129, 130, 257, 1000])
def test_random_symmetric(n):
    import paper_1709_03005_amd as cc
    rng = np.random.default_rng(n)
    M = rng.standard_normal((n, n))
    M = M + M.T
    with cc.Context(0) as ctx:
        w, V, info = ctx.eig_all(M)
        w2, V2, _ = ctx.eig_all(M, vectors=False)
    assert V2 is None and np.array_equal(w, w2)
    _check(M, w, V)


def test_random_symmetric_tiled_pass():
    # from 3072 trailing rows on, the reduction multiplies the trailing block
    # from its lower triangle in 128 x 128 tiles: n = 4500 switches from that
    # to the row pass after 1428 columns, and its first tiles' last tile row
    # holds 19 rows
    import paper_1709_03005_amd as cc
    n = 4500
    rng = np.random.default_rng(n)
    M = rng.standard_normal((n, n))
    M = M + M.T
    print(f"[eig_all] tiled pass n = {n}", flush=True)
    with cc.Context(0) as ctx:
        w, V, info = ctx.eig_all(M)
        w2, V2, _ = ctx.eig_all(M)
    # every sum runs in a fixed order: a second call repeats the first bit for bit
    assert np.array_equal(w, w2) and np.array_equal(V, V2)
    _check(M, w, V)


def test_large_diagonal_tiled_pass():
    # every column is already reduced (sigma = 0, tau = 0), through the tiled
    # product (n - 1 >= 3072 trailing rows) and then the row pass; T splits
    # into 1 x 1 blocks
    import paper_1709_03005_amd as cc
    n = 3300
    rng = np.random.default_rng(7)
    d = rng.uniform(-5.0, 5.0, n)
    d[100:110] = 1.25                     # a repeated value
    M = np.diag(d)
    with cc.Context(0) as ctx:
        w, V, info = ctx.eig_all(M)
    ds = np.sort(d)
    assert np.abs(w - ds).max() <= 1e-14 * np.abs(d).max()
    assert np.abs(V @ V.T - np.eye(n)).max() <= 1e-12
    # each eigenvector is a unit vector on a row holding its eigenvalue
    piv = np.abs(V).argmax(axis=1)
    assert np.allclose(np.abs(V[np.arange(n), piv]), 1.0)
    assert np.abs(d[piv] - w).max() <= 1e-14 * np.abs(d).max()


def test_repeated_and_clustered():
    import paper_1709_03005_amd as cc
    rng = np.random.default_rng(5)
    n = 120
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.sort(rng.uniform(-3, 3, n))
    ev[10:14] = ev[10]              # exactly repeated
    ev[40:45] = ev[40] + 1e-9 * np.arange(5)   # a tight cluster
    M = (Q * ev) @ Q.T
    M = 0.5 * (M + M.T)
    with cc.Context(0) as ctx:
        w, V, info = ctx.eig_all(M)
    print(f"[eig_all] clusters {info.clusters} holding {info.clustered} eigenvalues", flush=True)
    assert info.clusters >= 2
    _check(M, w, V, tol=1e-9, lapack_vectors=False)


@pytest.mark.parametrize("kind", ["diagonal", "zero", "tridiagonal"])
def test_special_matrices(kind):
    import paper_1709_03005_amd as cc
    rng = np.random.default_rng(9)
    n = 70
    if kind == "diagonal":
        M = np.diag(rng.uniform(-5, 5, n))
    elif kind == "zero":
        M = np.zeros((n, n))
    else:
        M = np.diag(rng.uniform(-1, 1, n)) + np.diag(rng.uniform(-1, 1, n - 1), 1)
        M = M + np.triu(M, 1).T
    with cc.Context(0) as ctx:
        w, V, _ = ctx.eig_all(M)
    wl = np.linalg.eigvalsh(M)
    assert np.abs(w - wl).max() <= 1e-12 * max(1.0, np.abs(wl).max())
    assert np.abs(V @ V.T - np.eye(n)).max() <= 1e-10
    assert np.abs(M @ V.T - V.T * w[None, :]).max() <= 1e-10 * max(1.0, np.abs(wl).max())


@pytest.mark.parametrize("name", ["tiny", "small"])
def test_built_matrix(name):
    import paper_1709_03005_amd as cc
    inst = synth.CONFIGS[name]()
    H = oracle.Oracle(inst).build()
    with cc.from_instance(inst) as ctx:
        ctx.build()
        G = ctx.get_matrix()
        w, V, info = ctx.eig_all()
        ev, _, _, rc = ctx.davidson(5, tol=1e-10, want_vectors=False)
    _check(G, w, V)
    wl = np.linalg.eigvalsh(H)             # the oracle's matrix
    assert np.abs(w - wl).max() <= 1e-10 * np.abs(wl).max()
    assert np.abs(w[:5] - ev).max() <= 1e-10 * np.abs(wl).max()


def test_medium_all_eigenpairs():
    import torch
    import time
    import paper_1709_03005_amd as cc
    inst = synth.medium()
    with cc.from_instance(inst, stream=torch.cuda.current_stream().cuda_stream) as ctx:
        ctx.build()
        G = ctx.get_matrix()
        t0 = time.time()
        w, V, info = ctx.eig_all()
        dt = time.time() - t0
    n = G.shape[0]
    print(f"[eig_all] D = {n}: {dt:.2f} s (tridiagonalisation {info.tridiag_ms:.0f} ms, "
          f"{info.tridiag_bytes / (info.tridiag_ms * 1e-3) / 1e9:.0f} GB/s of trailing-block traffic; "
          f"eigenvalues {info.eigenvalues_ms:.0f} ms; vectors + back-transformation {info.vectors_ms:.0f} ms); "
          f"clusters {info.clusters}", flush=True)
    t0 = time.time()
    wl = np.linalg.eigvalsh(G)
    print(f"[eig_all] LAPACK eigvalsh on the host: {time.time() - t0:.1f} s", flush=True)
    scale = np.abs(wl).max()
    assert np.abs(w - wl).max() <= 1e-10 * scale
    rng = np.random.default_rng(1)
    pick = np.concatenate([np.arange(10), rng.choice(n, 190, replace=False)])
    R = G @ V[pick].T - V[pick].T * w[pick][None, :]
    assert np.abs(R).max() <= 1e-10 * scale
    O = V[pick] @ V.T
    O[np.arange(len(pick)), pick] -= 1.0
    assert np.abs(O).max() <= 1e-10


def test_random_symmetric_large():
    # n = 8300: more than 32 column-kernel workgroups and more than 64 tiles a
    # side at the start of the reduction; matrix and vectors stay on the GPU
    import torch
    import paper_1709_03005_amd as cc
    n = 8300
    rng = np.random.default_rng(n)
    M = rng.standard_normal((n, n))
    M = M + M.T
    print(f"[eig_all] random n = {n}", flush=True)
    with cc.Context(0, torch.cuda.current_stream().cuda_stream) as ctx:
        w_t, V_t, info = ctx.eig_all(torch.from_numpy(M), device=True)
        w = w_t.cpu().numpy()
        pick = np.concatenate([np.arange(8), n - 8 + np.arange(8), rng.choice(n, 84, replace=False)])
        Vp = V_t[torch.from_numpy(pick).cuda()].cpu().numpy()
        O = (V_t[torch.from_numpy(pick).cuda()] @ V_t.T).cpu().numpy()
    wl = np.linalg.eigvalsh(M)
    scale = np.abs(wl).max()
    assert np.all(np.diff(w) >= 0)
    assert np.abs(w - wl).max() <= 1e-10 * scale
    R = M @ Vp.T - Vp.T * w[pick][None, :]
    assert np.abs(R).max() <= 1e-10 * scale
    O[np.arange(len(pick)), pick] -= 1.0
    assert np.abs(O).max() <= 1e-10


def test_device_arrays_and_refusals():
    import torch
    import ctypes as C
    import paper_1709_03005_amd as cc
    rng = np.random.default_rng(2)
    n = 50
    M = rng.standard_normal((n, n))
    M = M + M.T
    with cc.Context(0, torch.cuda.current_stream().cuda_stream) as ctx:
        w_h, V_h, _ = ctx.eig_all(M)
        tA = torch.from_numpy(M).cuda()
        tw = torch.zeros(n, dtype=torch.float64, device="cuda")
        tV = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        rc = cc.lib.cch_eig_all(ctx.h, C.c_void_p(tA.data_ptr()), n, n, C.c_void_p(tw.data_ptr()),
                                C.c_void_p(tV.data_ptr()), n, cc.CCH_MEM_DEVICE, None)
        assert rc == cc.CCH_OK
        assert np.array_equal(tw.cpu().numpy(), w_h) and np.array_equal(tV.cpu().numpy(), V_h)
        # the binding's device form: tensors in and out
        w_t, V_t, _ = ctx.eig_all(tA, device=True)
        assert w_t.is_cuda and V_t.is_cuda
        assert np.array_equal(w_t.cpu().numpy(), w_h) and np.array_equal(V_t.cpu().numpy(), V_h)
        bad = M.copy()
        bad[3, 4] = bad[4, 3] = np.nan
        with pytest.raises(cc.CchError) as e:
            ctx.eig_all(bad)
        assert e.value.code == cc.CCH_E_INPUT
        with pytest.raises(cc.CchError) as e:
            ctx.eig_all()                  # nothing built
        assert e.value.code == cc.CCH_E_STATE
    with cc.from_instance(synth.tiny(), sparse_l2=True) as sp:
        sp.build()
        with pytest.raises(cc.CchError) as e:
            sp.eig_all()
        assert e.value.code == cc.CCH_E_STATE
