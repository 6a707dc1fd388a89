"""Parity at the precision-configuration size (40 target orbitals, N = 12,
8000 determinants in one symmetry, 40 states, 300 continuum orbitals, 28000
L2 functions: D = 40000, two-word determinants): sampled elements of every
block class against the oracle computed one by one, exact symmetry of sampled
pairs, and the Davidson residual certificate ||H x - theta x|| on the
verified matrix, and Sylvester's inertia (LDL^T of H - sigma I, sigma halfway
between theta_10 and theta_11) proving that the ten pairs are the lowest ten.
Then the reduced-precision expansion products (FP32, split
BF16 with 3 and 7 slices) are built at the same size and the same sampled
elements are compared with the same oracle values: the max-abs element error
against the FP64 oracle is printed and bounded per mode (FP32 and 3 slices:
1e-5 of the largest element, about 2^-17; 7 slices: 1e-12), and each mode's
lowest eigenvalues are compared with the FP64 build's."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

_state = {}


def _fp64():
    """The FP64 build, its Davidson pairs and the oracle's sampled elements."""
    if not _state:
        import torch
        import paper_1709_03005_amd as cc
        inst = synth.precision()
        print("[precision] generated", flush=True)
        D, Dc = inst.dim(), inst.n_cont_rows()
        with cc.from_instance(inst, stream=torch.cuda.current_stream().cuda_stream) as ctx:
            ctx.build()
            print("[precision] built", flush=True)
            G = ctx.get_matrix()
            ev, vec, info, rc = ctx.davidson(11, tol=1e-8)   # one pair more for the inertia check
        print(f"[precision] davidson rc={rc} iters={info.iterations}", flush=True)
        rng = np.random.default_rng(5)
        rows = np.concatenate([rng.integers(0, Dc, 24), rng.integers(Dc, D, 24), rng.integers(Dc, D, 24),
                               rng.integers(0, D, 8)])
        cols = np.concatenate([rng.integers(0, Dc, 24), rng.integers(0, Dc, 24), rng.integers(Dc, D, 24),
                               rows[-8:]])
        v, a, k = oracle.Oracle(inst).elements(rows, cols)
        _state.update(inst=inst, G=G, ev=ev[:10], vec=vec[:10], ev11=ev, vec11=vec, rc=rc, rows=rows, cols=cols,
                      v=v, a=a, k=k, scale=float(np.abs(G).max()))
    return _state


def test_precision_size_parity():
    import paper_1709_03005_amd as cc
    s = _fp64()
    G, rows, cols, v = s["G"], s["rows"], s["cols"], s["v"]
    assert s["scale"] > 0
    g = G[rows, cols]
    ok, _ = oracle.tolerance_ok(g, v, s["a"], s["k"])
    assert ok.all(), [(int(r), int(c), g[i], v[i]) for i, (r, c) in enumerate(zip(rows, cols)) if not ok[i]][:5]
    assert np.count_nonzero(v) > len(v) // 3
    assert np.array_equal(G[rows, cols], G[cols, rows])
    assert s["rc"] == cc.CCH_OK
    ev, vec = s["ev"], s["vec"]
    r = G @ vec.T - vec.T * ev[None, :]
    assert np.linalg.norm(r, axis=0).max() < 2e-8
    assert np.all(np.diff(ev) >= -1e-12)


@pytest.mark.parametrize("mode,slices,bound", [("fp32", 0, 1e-5), ("bf16", 3, 1e-5), ("bf16", 7, 1e-12)])
def test_precision_modes_at_size(mode, slices, bound):
    import torch
    import paper_1709_03005_amd as cc
    s = _fp64()
    inst, rows, cols, v = s["inst"], s["rows"], s["cols"], s["v"]
    prec = cc.CCH_PREC_FP32 if mode == "fp32" else cc.CCH_PREC_SPLIT_BF16
    print(f"[precision {mode}{slices or ''}] build", flush=True)
    with cc.from_instance(inst, stream=torch.cuda.current_stream().cuda_stream, precision=prec,
                          split_slices=slices) as ctx:
        ctx.build()
        g = ctx.get_elements(rows, cols)
        gt = ctx.get_elements(cols, rows)
        diag = ctx.get_diagonal()
        ev, _, info, rc = ctx.davidson(10, tol=1e-8, want_vectors=False)
    assert np.abs(diag).max() > 0
    assert np.array_equal(g, gt)
    err = np.abs(g - v).max()
    eerr = np.abs(ev - s["ev"]).max()
    scale = s["scale"]
    print(f"[precision {mode}{slices or ''}] max-abs element error against the FP64 oracle {err:.3e} "
          f"(relative to max|H| = {scale:.3f}: {err / scale:.3e}); eigenvalue error against the FP64 build "
          f"{eerr:.3e}; Davidson {info.iterations} iterations", flush=True)
    assert err <= bound * scale
    assert rc == cc.CCH_OK
    assert eerr <= max(10 * bound * scale, 1e-10 * np.abs(s["ev"]).max())


def test_precision_lowest_k_by_inertia():
    """Runs last: it factorises the host copy of the matrix in place."""
    import time
    from tests.helpers import negative_inertia
    s = _fp64()
    G, ev, vec = s["G"], s["ev11"], s["vec11"]
    k = 10
    r = np.linalg.norm(G @ vec.T - vec.T * ev[None, :], axis=0)
    assert r.max() < 2e-8, r
    assert ev[k] - ev[k - 1] > 1e-6
    sigma = 0.5 * (ev[k - 1] + ev[k])
    G[np.diag_indices(G.shape[0])] -= sigma
    t0 = time.time()
    neg = negative_inertia(G)
    print(f"[precision] eigenvalues below sigma = {sigma:.12f}: {neg} (LDL^T of D = {G.shape[0]} in "
          f"{time.time() - t0:.1f} s)", flush=True)
    _state.clear()
    assert neg == k
