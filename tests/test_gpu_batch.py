"""Batched build: many instances of uneven size in persistent launches
captured in one hipGraph, tiles chosen by the autotuner. The first eight
instances of the batching workload hold one, two and four target symmetries
(their (tt|cc) and (tc|tc) integrals in the symmetry-packed layout). Every
batched matrix must be bit-identical to the same instance built alone (same
arithmetic order per element), and sampled elements of a one-symmetry and of
the four-symmetry instance must match the oracle. The packed integral input
gives the same matrix, bit for bit, as the dense one."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def test_batch_equals_single_builds():
    import paper_1709_03005_amd as cc
    insts = [synth.batch_instance(i) for i in range(8)]
    print("[batch] dims", [I.dim() for I in insts], "symmetries", [len(I.syms) for I in insts], flush=True)
    assert {len(I.syms) for I in insts} == {1, 2, 4}
    ctxs = [cc.from_instance(I) for I in insts]
    solo = []
    for c in ctxs:
        c.build()
        solo.append(c.get_matrix())
    b = cc.Batch(ctxs, autotune=True)
    info = b.info()
    print("[batch] info", info, flush=True)
    assert info["instances"] == 8 and info["autotuned"] == 1 and info["graph_nodes"] > 0
    for rep in range(2):                       # graph replayed twice
        b.build()
        for c, G in zip(ctxs, solo):
            assert np.array_equal(c.get_matrix(), G)
    print("[batch] device ms", b.time_ms(), flush=True)
    # a second batch of the same shape takes its tiles from the cache
    b2 = cc.Batch(ctxs, autotune=True)
    assert b2.info()["from_cache"] == 1
    b2.build()
    assert np.array_equal(ctxs[3].get_matrix(), solo[3])
    b2.close()
    # oracle check on a one-symmetry and on the four-symmetry instance
    for i in (2, next(j for j, I in enumerate(insts) if len(I.syms) == 4)):
        I = insts[i]
        rng = np.random.default_rng(2)
        D, Dc = I.dim(), I.n_cont_rows()
        rows = np.concatenate([rng.integers(0, Dc, 40), rng.integers(0, D, 40)])
        cols = np.concatenate([rng.integers(0, Dc, 40), rng.integers(0, D, 40)])
        v, a, k = oracle.Oracle(I).elements(rows, cols)
        ok, _ = oracle.tolerance_ok(solo[i][rows, cols], v, a, k)
        assert ok.all(), i
        assert np.count_nonzero(v) > 10
    ev, _, info_d, rc = ctxs[2].davidson(5, tol=1e-9, want_vectors=False)
    assert rc == cc.CCH_OK
    w = np.linalg.eigvalsh(solo[2])[:5]
    assert np.all(np.abs(ev - w) <= 1e-10 * np.abs(w).max())
    b.close()
    for c in ctxs:
        c.close()


def test_batch_rejects_unplanned_and_lowp():
    import paper_1709_03005_amd as cc
    I = synth.tiny()
    c1 = cc.from_instance(I, plan=False)
    with pytest.raises(cc.CchError) as e:
        cc.Batch([c1])
    assert e.value.code == cc.CCH_E_STATE
    c2 = cc.from_instance(I, precision=cc.CCH_PREC_FP32)
    with pytest.raises(cc.CchError) as e:
        cc.Batch([c2])
    assert e.value.code == cc.CCH_E_INVALID_ARG
    c1.close()
    c2.close()


def test_packed_integrals_equal_dense():
    """The same instance from dense and from symmetry-packed (tt|cc) / (tc|tc)
    arrays: identical matrices, bit for bit, for four irreps (including an
    irrep pair with no continuum orbitals) and in several expansion passes."""
    import paper_1709_03005_amd as cc
    dense = synth.make_instance(12, 6, 4, [20, 0, 14, 9], [0, 1, 2, 3], [60, 40, 50, 30], [3, 2, 4, 2], 200, 4401)
    packed = synth.pack_integrals(dense)
    H, A, K = oracle.Oracle(dense).build(with_abs=True)
    with cc.from_instance(dense) as cd, cc.from_instance(packed) as cp:
        cd.build()
        cp.build()
        Gd, Gp = cd.get_matrix(), cp.get_matrix()
        bytes0, _ = cp.plan_info()
        b_elems = cp.work_counts()["relayout_bytes"] / 16.0
    assert np.array_equal(Gd, Gp)
    ok, _ = oracle.tolerance_ok(Gp, H, A, K)
    assert ok.all()
    # a memory budget that splits the expansion into passes over the continuum rows
    with cc.from_instance(packed, plan=False) as cb:
        cb.plan(max_device_bytes=int(bytes0 - 8 * b_elems + 8 * b_elems // 6))
        assert cb.plan_info()[1] >= 2
        cb.build()
        assert np.array_equal(cb.get_matrix(), Gd)
