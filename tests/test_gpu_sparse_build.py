"""Classes 2 and 8 built and stored sparse (CCH_PLAN_SPARSE_L2; Sec. 2.2
names the off-diagonal pure-L2 class as the sparse one): the L2 block exists
only as CSR of the determinant pairs within a double substitution.

* small instances: every element of the read-out equals the dense build's bit
  for bit and matches the oracle; sampled elements, class blocks 2, 4 and 8
  and the diagonal equal the dense build's; the CSR structure equals the
  excitation scan's L2 pair list (both triangles); the eigenpairs match LAPACK
  on the oracle's matrix; an instance without continuum rows and one without
  L2 functions;
* the phosphoric-acid size (D = 122815, whose dense matrix is 121 GB): the
  same eigenvalues as the dense build's, sampled elements of every class
  against the oracle, residuals certified by the library;
* a size dense storage cannot hold (D = 250712, 503 GB dense): sampled
  elements of every class against the oracle and the residual certificate.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

SMALL = {
    "tiny": synth.tiny,
    "small": synth.small,
    "wide": synth.wide,
    "l2_only": lambda: synth.make_instance(12, 6, 2, [0, 0], [0, 1], [20, 18], [2, 2], 900, 811, name="l2only"),
    "no_l2": lambda: synth.make_instance(10, 6, 1, 20, [0], 40, 3, 0, 813, name="nol2"),
}


@pytest.mark.parametrize("name", sorted(SMALL))
def test_sparse_build_equals_dense_and_oracle(name):
    import paper_1709_03005_amd as cc
    inst = SMALL[name]()
    D, Dc = inst.dim(), inst.n_cont_rows()
    k = min(5, D)
    print(f"[sparse build] {name} D = {D} Dc = {Dc}", flush=True)
    H, A, K = oracle.Oracle(inst).build(with_abs=True)
    rng = np.random.default_rng(2)
    rows, cols = rng.integers(0, D, 500), rng.integers(0, D, 500)
    with cc.from_instance(inst) as dense, cc.from_instance(inst, sparse_l2=True) as sp:
        dense.build()
        sp.build()
        Gd, Gs = dense.get_matrix(), sp.get_matrix()
        low = sp.get_matrix(lower=True)
        assert np.array_equal(Gs, Gd)
        assert np.array_equal(np.tril(low), np.tril(Gd))
        assert np.array_equal(sp.get_elements(rows, cols), Gd[rows, cols])
        assert np.array_equal(sp.get_diagonal(), dense.get_diagonal())
        if inst.n_l2:
            for cls in (2, 8):
                assert np.array_equal(sp.get_block(cls), dense.get_block(cls))
            for a in range(len(inst.syms)):
                assert np.array_equal(sp.get_block(4, a), dense.get_block(4, a))
            wd, ws = dense.work_counts(), sp.work_counts()
            lab = sp.get_labels(cc.CCH_PAIRS_L2)
            assert ws["l2_lower_elements"] == len(lab["x"])        # structural non-zeros, lower triangle
            assert ws["lower_elements"] == wd["lower_elements"] - wd["l2_lower_elements"] + len(lab["x"])
            # the stored structure: exactly the scan's pairs, mirrored
            nz = np.zeros((inst.n_l2, inst.n_l2), bool)
            nz[lab["x"], lab["y"]] = True
            nz |= nz.T
            Gl = Gs[Dc:, Dc:]
            assert np.all(Gl[~nz] == 0.0)
        with pytest.raises(cc.CchError) as e:
            sp.matrix_device()
        assert e.value.code == cc.CCH_E_STATE
        ev, X, info, rc = sp.davidson(k, tol=1e-9)
    ok, _ = oracle.tolerance_ok(Gs, H, A, K)
    assert ok.all()
    w = np.linalg.eigvalsh(H)[:k]
    scale = max(np.abs(w).max(), 1.0)
    assert rc == cc.CCH_OK
    assert np.all(np.abs(ev - w) <= 1e-10 * np.maximum(np.abs(w), scale)), ev - w
    Xt = X.T
    assert np.abs(H @ Xt - Xt * ev).max() <= 1e-8 * scale


def test_sparse_build_refuses_batching():
    import paper_1709_03005_amd as cc
    inst = synth.tiny()
    with cc.from_instance(inst, sparse_l2=True) as sp:
        with pytest.raises(cc.CchError) as e:
            cc.Batch([sp])
        assert e.value.code == cc.CCH_E_STATE


def _sampled_parity(inst, ctx, rng, n=24):
    D, Dc = inst.dim(), inst.n_cont_rows()
    l2 = lambda m: rng.integers(Dc, D, m)
    ct = lambda m: rng.integers(0, Dc, m)
    near = l2(n)
    rows = np.concatenate([ct(16), l2(n), l2(40), near, l2(8), ct(8)])
    cols = np.concatenate([ct(16), ct(n), l2(40), np.minimum(near + rng.integers(1, 6, n), D - 1), rows[-16:-8],
                           l2(8)])
    g = ctx.get_elements(rows, cols)
    gt = ctx.get_elements(cols, rows)
    v, a, k = oracle.Oracle(inst).elements(rows, cols)
    ok, _ = oracle.tolerance_ok(g, v, a, k)
    assert ok.all(), [(int(r), int(c), g[i], v[i]) for i, (r, c) in enumerate(zip(rows, cols)) if not ok[i]][:5]
    assert np.count_nonzero(v) > len(v) // 4
    assert np.array_equal(g, gt)


def test_sparse_build_l2heavy_size():
    import paper_1709_03005_amd as cc
    inst = synth.l2heavy()
    print(f"[sparse build] l2heavy D = {inst.dim()}", flush=True)
    with cc.from_instance(inst) as dense:
        dense.build()
        ev_d, _, _, rc_d = dense.davidson(5, tol=1e-8, want_vectors=False)
    print("[sparse build] dense solve done", flush=True)
    with cc.from_instance(inst, sparse_l2=True) as sp:
        dev_bytes, _ = sp.plan_info()
        sp.build()
        ev, vr, info, rc = sp.davidson(5, tol=1e-8, residuals=True)
        print(f"[sparse build] l2heavy: device bytes {dev_bytes / 2**30:.1f} GiB (dense 121 GB), "
              f"Davidson {info.iterations} iterations", flush=True)
        _sampled_parity(inst, sp, np.random.default_rng(9))
    assert rc == rc_d == cc.CCH_OK
    assert dev_bytes < 20 * 2**30
    assert np.all(np.abs(ev - ev_d) <= 1e-10 * np.abs(ev_d).max())
    X, R = vr[:5], vr[5:]
    assert np.abs(X @ X.T - np.eye(5)).max() < 1e-10
    assert np.linalg.norm(R, axis=1).max() < 2e-8


def test_sparse_build_beyond_dense_storage():
    import paper_1709_03005_amd as cc
    inst = synth.l2huge()
    D = inst.dim()
    assert 8.0 * D * D > 288e9            # more than one GPU's HBM as a dense matrix
    print(f"[sparse build] l2huge D = {D}", flush=True)
    with cc.from_instance(inst, sparse_l2=True) as sp:
        dev_bytes, _ = sp.plan_info()
        sp.build()
        print(f"[sparse build] l2huge built, device bytes {dev_bytes / 2**30:.1f} GiB", flush=True)
        ev, vr, info, rc = sp.davidson(5, tol=1e-8, residuals=True)
        print(f"[sparse build] l2huge Davidson rc={rc} {info.iterations} iterations", flush=True)
        _sampled_parity(inst, sp, np.random.default_rng(10))
    assert rc == cc.CCH_OK
    X, R = vr[:5], vr[5:]
    assert np.abs(X @ X.T - np.eye(5)).max() < 1e-10
    assert np.linalg.norm(R, axis=1).max() < 2e-8
    assert np.all(np.diff(ev) >= -1e-12)
