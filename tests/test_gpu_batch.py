"""Batched build: many instances of uneven size in persistent launches
captured in one hipGraph, tiles chosen by the autotuner. Every batched matrix
must be bit-identical to the same instance built alone (same arithmetic
order per element), and sampled elements of one instance must match the
oracle."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def test_batch_equals_single_builds():
    import paper_1709_03005_amd as cc
    insts = [synth.batch_instance(i) for i in range(8)]
    print("[batch] dims", [I.dim() for I in insts], flush=True)
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
    # oracle check on one instance, Davidson on a batched context
    I = insts[2]
    rng = np.random.default_rng(2)
    D = I.dim()
    rows, cols = rng.integers(0, D, 60), rng.integers(0, D, 60)
    v, a, k = oracle.Oracle(I).elements(rows, cols)
    ok, _ = oracle.tolerance_ok(solo[2][rows, cols], v, a, k)
    assert ok.all()
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
