"""Parity at the size of the paper's L2-heavy case (phosphoric acid: 712
contracted rows + 122103 L2 functions, D = 122815, a dense matrix of 121 GB
on the device): sampled elements of every block class read back with
cch_get_elements and compared with the oracle one by one, exact symmetry of
the sampled pairs, and the Davidson residual certificate ||H x - theta x||
computed by the library on the device matrix, with the dense mat-vec and
with the L2 block as CSR (the same eigenvalues). Also cch_get_elements itself
against the full read-out on a small instance, and its index check."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def test_get_elements_matches_full_matrix():
    import paper_1709_03005_amd as cc
    inst = synth.tiny()
    D = inst.dim()
    rng = np.random.default_rng(1)
    rows, cols = rng.integers(0, D, 300), rng.integers(0, D, 300)
    with cc.from_instance(inst) as ctx:
        ctx.build()
        G = ctx.get_matrix()
        assert np.array_equal(ctx.get_elements(rows, cols), G[rows, cols])
        with pytest.raises(cc.CchError) as e:
            ctx.get_elements([0, D], [0, 0])
        assert e.value.code == cc.CCH_E_INVALID_ARG


def test_l2heavy_size_parity():
    import paper_1709_03005_amd as cc
    inst = synth.l2heavy()
    D, Dc = inst.dim(), inst.n_cont_rows()
    assert (D, Dc) == (122815, 712)
    print(f"[l2heavy] generated D = {D}", flush=True)
    rng = np.random.default_rng(9)
    l2 = lambda n: rng.integers(Dc, D, n)
    ct = lambda n: rng.integers(0, Dc, n)
    near = l2(24)
    rows = np.concatenate([ct(16), l2(24), l2(40), near, l2(8)])
    cols = np.concatenate([ct(16), ct(24), l2(40), np.minimum(near + rng.integers(1, 6, 24), D - 1), rows[-8:]])
    with cc.from_instance(inst) as ctx:
        ctx.build()
        print("[l2heavy] built", flush=True)
        g = ctx.get_elements(rows, cols)
        gt = ctx.get_elements(cols, rows)
        ev, vr, info, rc = ctx.davidson(5, tol=1e-8, residuals=True)
        print(f"[l2heavy] davidson rc={rc} iterations={info.iterations}", flush=True)
        ev_s, vs, info_s, rc_s = ctx.davidson(5, tol=1e-8, residuals=True, sparse_l2=True)
    print(f"[l2heavy] sparse-L2 davidson rc={rc_s} iterations={info_s.iterations}", flush=True)
    assert rc_s == cc.CCH_OK
    assert np.all(np.abs(ev_s - ev) <= 1e-10 * np.abs(ev).max())
    assert np.linalg.norm(vs[5:], axis=1).max() < 2e-8
    v, a, k = oracle.Oracle(inst).elements(rows, cols)
    ok, _ = oracle.tolerance_ok(g, v, a, k)
    assert ok.all(), [(int(r), int(c), g[i], v[i]) for i, (r, c) in enumerate(zip(rows, cols)) if not ok[i]][:5]
    assert np.count_nonzero(v) > len(v) // 4
    assert np.array_equal(g, gt)
    assert rc == cc.CCH_OK
    X, R = vr[:5], vr[5:]
    assert np.abs(X @ X.T - np.eye(5)).max() < 1e-10
    assert np.linalg.norm(R, axis=1).max() < 2e-8
    assert np.all(np.diff(ev) >= -1e-12)
