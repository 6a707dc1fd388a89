"""Degenerate and extreme inputs through the C-ABI, each against the oracle
element by element and the Davidson pairs against LAPACK on the oracle's
matrix: no L2 functions, a target symmetry whose continuum irrep is empty
(no rows of its own), one determinant and one state, as many states as
determinants, D = 1, every eigenpair asked for (k = D), the 256-state limit,
and 62 target electrons in two-word determinants (N + 1 = 63)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

CASES = {
    "no_l2": lambda: synth.make_instance(8, 4, 1, 6, [0], 12, 2, 0, 701, name="no_l2"),
    "empty_continuum_irrep": lambda: synth.make_instance(8, 4, 2, [5, 0], [0, 1], [10, 9], [2, 3], 6, 702,
                                                          name="empty_cont"),
    "one_det_one_state": lambda: synth.make_instance(8, 4, 1, 7, [0], 1, 1, 4, 703, name="one_det"),
    "square_ci": lambda: synth.make_instance(8, 4, 1, 5, [0], 6, 6, 3, 704, name="square"),
    "d_equals_1": lambda: synth.make_instance(6, 2, 1, 1, [0], 3, 1, 0, 705, name="d1"),
    "states_256": lambda: synth.make_instance(12, 6, 1, 2, [0], 256, 256, 7, 706, name="s256"),
    "electrons_62": lambda: synth.make_instance(36, 62, 1, 3, [0], 12, 3, 4, 707, name="n62"),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_edge_case_matrix_and_eigenpairs(name):
    import paper_1709_03005_amd as cc
    inst = CASES[name]()
    D = inst.dim()
    print(f"[edges] {name} D = {D}", flush=True)
    H, A, K = oracle.Oracle(inst).build(with_abs=True)
    assert H.shape == (D, D)
    with cc.from_instance(inst) as ctx:
        ctx.build()
        G = ctx.get_matrix()
        ok, _ = oracle.tolerance_ok(G, H, A, K)
        assert ok.all(), np.argwhere(~ok)[:5]
        k = min(D, 5) if name != "no_l2" else D          # no_l2 (D = 12): every pair
        ev, vec, info, rc = ctx.davidson(k, tol=1e-9)
    assert rc == cc.CCH_OK, info.max_residual
    w = np.linalg.eigvalsh(H)[:k]
    scale = np.abs(w).max()
    assert np.all(np.abs(ev - w) <= 1e-10 * np.maximum(np.abs(w), scale)), (ev - w)
    # the vectors: orthonormal, residuals of the oracle matrix small
    X = np.asarray(vec).reshape(k, D).T
    assert np.abs(X.T @ X - np.eye(k)).max() < 1e-10
    assert np.abs(H @ X - X * ev).max() <= 1e-8 * max(1.0, scale)
