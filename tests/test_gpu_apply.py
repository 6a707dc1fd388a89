"""cch_apply (W = H V, the product of every iterative diagonaliser of
Sec. 3.2) against the product formed on the host from the read-out matrix.

* the full product with split-K below D = 16384 (tiny, small, wide,
  medium), the lower-triangle product above it at the item heights it
  picks (mid, D = 20000: 128 rows; the precision instance, D = 40000: 256
  rows, checked on sampled rows), and the sparse-L2 product of a context
  planned with CCH_PLAN_SPARSE_L2;
* block widths 1, 10, 16, 17 and 35 (several 16-vector launches, ragged);
* the error bound 2 D u (|V| |H|) elementwise (u the unit roundoff), which
  covers both sides' rounding for any summation order;
* equal inputs give equal bits; bad arguments are refused.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
U = np.finfo(np.float64).eps / 2


def _check(W, V, Hrows_T, D):
    ref = V @ Hrows_T
    tol = 2 * D * U * (np.abs(V) @ np.abs(Hrows_T)) + 1e-300
    bad = np.abs(W - ref) > tol
    assert not bad.any(), (np.argwhere(bad)[:5], np.abs(W - ref).max())


@pytest.mark.parametrize("name,sparse", [("tiny", False), ("small", False), ("wide", False), ("medium", False),
                                         ("mid", False), ("small", True), ("wide", True)])
def test_apply_equals_host_product(name, sparse):
    import paper_1709_03005_amd as cc
    inst = getattr(synth, name)()
    D = inst.dim()
    print(f"[apply] {name} D = {D} sparse={sparse}", flush=True)
    rng = np.random.default_rng(D)
    with cc.from_instance(inst, sparse_l2=sparse) as ctx:
        ctx.build()
        H = ctx.get_matrix()
        for b in (1, 10, 16, 17, 35):
            V = rng.standard_normal((b, D))
            W = ctx.apply(V)
            _check(W, V, H, D)     # H symmetric: (H V^T)^T = V H
            if b == 17:
                assert np.array_equal(W, ctx.apply(V))


def test_apply_large_item_height_sampled_rows():
    import paper_1709_03005_amd as cc
    inst = synth.precision()
    D = inst.dim()
    print(f"[apply] precision D = {D}", flush=True)
    rng = np.random.default_rng(4)
    rows = np.sort(rng.choice(D, 24, replace=False))
    rows[-1] = D - 1                      # the ragged last strip and item
    with cc.from_instance(inst) as ctx:
        ctx.build()
        Hr = ctx.get_elements(np.repeat(rows, D), np.tile(np.arange(D), len(rows))).reshape(len(rows), D)
        for b in (10, 16):
            V = rng.standard_normal((b, D))
            W = ctx.apply(V)
            _check(W[:, rows], V, Hr.T, D)


def test_apply_refusals():
    import paper_1709_03005_amd as cc
    inst = synth.tiny()
    with cc.from_instance(inst) as ctx:
        with pytest.raises(cc.CchError) as e:
            ctx.apply(np.zeros((1, inst.dim())))
        assert e.value.code == cc.CCH_E_STATE
        ctx.build()
        with pytest.raises(cc.CchError) as e:
            ctx.apply(np.zeros((1, inst.dim() - 1)))
        assert e.value.code == cc.CCH_E_INVALID_ARG
        assert ctx.apply(np.zeros((0, inst.dim()))).shape == (0, inst.dim())
