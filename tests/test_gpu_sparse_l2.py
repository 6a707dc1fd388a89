"""Davidson with the L2 block as CSR in the mat-vec (CCH_DAV_SPARSE_L2):
the same eigenpairs as the dense mat-vec and as LAPACK on the oracle's
matrix, residuals small on the full matrix read back to the host, for
instances with and without continuum rows (the panel sums are then absent),
with two solves on one build (the CSR is reused) and a rebuild in between
(the CSR is formed again)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

CASES = {
    "tiny": synth.tiny,
    "small": synth.small,
    "l2_only": lambda: synth.make_instance(12, 6, 2, [0, 0], [0, 1], [20, 18], [2, 2], 900, 811, name="l2only"),
    "sparse_l2": lambda: synth.make_instance(20, 8, 1, 10, [0], 60, 3, 3000, 812, name="sparsel2"),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_sparse_l2_matches_dense_and_oracle(name):
    import paper_1709_03005_amd as cc
    inst = CASES[name]()
    D, k = inst.dim(), 5
    print(f"[sparse_l2] {name} D = {D} Dc = {inst.n_cont_rows()}", flush=True)
    H = oracle.Oracle(inst).build()
    w = np.linalg.eigvalsh(H)[:k]
    scale = np.abs(w).max()
    with cc.from_instance(inst) as ctx:
        ctx.build()
        G = ctx.get_matrix()
        ev_d, _, _, rc_d = ctx.davidson(k, tol=1e-9, want_vectors=False)
        ev_s, X, info, rc_s = ctx.davidson(k, tol=1e-9, sparse_l2=True)
        ev_s2, _, _, _ = ctx.davidson(k, tol=1e-9, want_vectors=False, sparse_l2=True)   # CSR reused
        ctx.build()                                                                       # CSR formed again
        ev_s3, _, _, _ = ctx.davidson(k, tol=1e-9, want_vectors=False, sparse_l2=True)
    assert rc_d == rc_s == cc.CCH_OK
    for ev in (ev_d, ev_s, ev_s2, ev_s3):
        assert np.all(np.abs(ev - w) <= 1e-10 * np.maximum(np.abs(w), scale)), (ev - w)
    assert np.array_equal(ev_s, ev_s2) and np.array_equal(ev_s, ev_s3)
    Xt = X.T
    assert np.abs(Xt.T @ Xt - np.eye(k)).max() < 1e-10
    assert np.abs(G @ Xt - Xt * ev_s).max() <= 1e-8 * max(1.0, scale)
