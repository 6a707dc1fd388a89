"""Continuum electrons of beta spin (cch_add_target_symmetry_spin): triplet
target states coupled with the continuum electron to doublets,
sqrt(2/3) |T, 1> u_beta - sqrt(1/3) |T, 0> u_alpha (the inputs' channels are
S = 1/2 eigenvectors in the Fock space, and the oracle's contracted matrix is
pinned to T^T H T there, in the CPU tests).

* every element of the built matrix matches the oracle within the tolerance
  rule, on one- and two-word instances with one and two target symmetries
  (the symmetry pairs, classes 1/3/5/6/7, class 4 with beta continuum
  electrons, the L2 block), and the lowest eigenpairs match LAPACK on the
  oracle's matrix;
* a batched build gives the same matrix bit for bit;
* refusals: a spin other than 0 or 1, an alpha count that does not match the
  spin.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

CASES = {
    "small": synth.small,
    "wide": synth.wide,
    "two_symmetries": lambda: synth.make_instance(12, 4, 2, [6, 5], [0, 1], [24, 20], [3, 2], 120, 977,
                                                  name="td2"),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_triplet_doublet_matrix_matches_oracle(name):
    import paper_1709_03005_amd as cc
    inst = synth.triplet_doublet(CASES[name](), seed=3)
    assert all(np.any(s.cont_spin == 1) and np.any(s.cont_spin == 0) for s in inst.syms)
    H, A, K = oracle.Oracle(inst).build(with_abs=True)
    D = inst.dim()
    print(f"[triplet] {name} D = {D}", flush=True)
    with cc.from_instance(inst) as ctx:
        ctx.build()
        G = ctx.get_matrix()
        k = min(5, D)
        ev, X, info, rc = ctx.davidson(k, tol=1e-9)
    ok, _ = oracle.tolerance_ok(G, H, A, K)
    assert ok.all(), np.argwhere(~ok)[:5]
    Dc = inst.n_cont_rows()
    assert np.abs(G[:Dc, :Dc] - np.diag(np.diag(G[:Dc, :Dc]))).max() > 0.1
    w = np.linalg.eigvalsh(H)[:k]
    scale = max(np.abs(w).max(), 1.0)
    assert rc == cc.CCH_OK
    assert np.all(np.abs(ev - w) <= 1e-10 * scale), ev - w


def test_triplet_doublet_batched_equals_single():
    import paper_1709_03005_amd as cc
    insts = [synth.triplet_doublet(CASES[n](), seed=3) for n in ("two_symmetries", "wide")]
    singles = []
    for inst in insts:
        with cc.from_instance(inst) as ctx:
            ctx.build()
            singles.append(ctx.get_matrix())
    ctxs = [cc.from_instance(inst) for inst in insts]
    try:
        b = cc.Batch(ctxs)
        try:
            b.build()
        finally:
            b.close()
        for ctx, G in zip(ctxs, singles):
            assert np.array_equal(ctx.get_matrix(), G)
    finally:
        for ctx in ctxs:
            ctx.close()


def test_continuum_spin_refusals():
    import paper_1709_03005_amd as cc
    inst = synth.triplet_doublet(synth.tiny(), seed=3)
    s = inst.syms[0]
    with cc.from_instance(inst, plan=False) as ctx:
        bad = s.cont_spin.copy()
        bad[0] = 2
        with pytest.raises(cc.CchError) as e:
            ctx.add_target_symmetry(s.irrep, s.dets, s.ci, bad)
        assert e.value.code == cc.CCH_E_INPUT
        flipped = 1 - s.cont_spin           # alpha counts no longer match the spins
        with pytest.raises(cc.CchError) as e:
            ctx.add_target_symmetry(s.irrep, s.dets, s.ci, flipped)
        assert e.value.code == cc.CCH_E_INPUT
