"""Target states over multi-determinant CSFs (Eq. 2) through the C-ABI
(cch_add_target_symmetry_csf): the matrix equals the oracle's for the same
states rewritten over determinants (oracle.csf_expand), and bit for bit the
library's own build from those determinant arrays; malformed lists are
refused."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _csfs(dets, seed):
    """One- and two-determinant CSFs covering every determinant once, plus a
    few three-term CSFs that reuse determinants (a determinant in several
    CSFs)."""
    rng = np.random.default_rng(seed)
    M = dets.shape[0]
    perm = rng.permutation(M)
    terms, coef, starts = [], [], [0]
    i = 0
    while i < M:
        k = 1 if (i + 1 == M or rng.random() < 0.5) else 2
        for t in range(k):
            terms.append(dets[perm[i + t]])
            coef.append(1.0 if k == 1 else rng.choice([-1.0, 1.0]) * np.sqrt(0.5))
        starts.append(len(terms))
        i += k
    for _ in range(3):
        for d in rng.choice(M, 3, replace=False):
            terms.append(dets[d])
            coef.append(rng.uniform(-1.0, 1.0))
        starts.append(len(terms))
    return np.array(terms, dtype=np.uint64), np.array(coef), np.array(starts, dtype=np.int32)


def _context(cc, inst, csf, ci):
    terms, coef, starts = csf
    ctx = cc.Context()
    ctx.set_orbitals(inst.n_o, inst.tgt_irrep, inst.n_irrep, inst.n_c, inst.total_irrep)
    ctx.set_integrals(inst.h, inst.tttt, inst.tttc, inst.ttcc, inst.tctc, inst.e_core)
    ctx.add_target_symmetry_csf(inst.syms[0].irrep, starts, terms, coef, ci)
    for s in inst.syms[1:]:
        ctx.add_target_symmetry(s.irrep, s.dets, s.ci)
    ctx.set_l2(inst.l2_dets)
    ctx.plan()
    return ctx


def test_csf_targets_match_oracle_and_determinant_input():
    import dataclasses
    import paper_1709_03005_amd as cc
    inst = synth.small()
    csf = _csfs(inst.syms[0].dets, 31)
    ncsf = len(csf[2]) - 1
    rng = np.random.default_rng(32)
    ci = np.linalg.qr(rng.standard_normal((ncsf, 4)))[0]
    d, C = oracle.csf_expand(csf[0], csf[1], list(csf[2]), ci)
    exp = dataclasses.replace(inst, syms=[synth.TargetSym(inst.syms[0].irrep, d, C)] + inst.syms[1:])
    print("[csf] D =", exp.dim(), "CSFs", ncsf, "dets", d.shape[0], flush=True)
    H, A, K = oracle.Oracle(exp).build(with_abs=True)
    with _context(cc, inst, csf, ci) as ctx:
        ctx.build()
        G = ctx.get_matrix()
    ok, _ = oracle.tolerance_ok(G, H, A, K)
    assert ok.all(), np.argwhere(~ok)[:5]
    with cc.from_instance(exp) as ref:
        ref.build()
        assert np.array_equal(G, ref.get_matrix())


def test_csf_lists_are_checked():
    import paper_1709_03005_amd as cc
    inst = synth.tiny()
    terms, coef, starts = _csfs(inst.syms[0].dets, 5)
    ncsf = len(starts) - 1
    ci = np.linalg.qr(np.random.default_rng(6).standard_normal((ncsf, 3)))[0]
    ctx = cc.Context()
    ctx.set_orbitals(inst.n_o, inst.tgt_irrep, inst.n_irrep, inst.n_c, inst.total_irrep)
    ctx.set_integrals(inst.h, inst.tttt, inst.tttc, inst.ttcc, inst.tctc, inst.e_core)
    irr = inst.syms[0].irrep
    bad = starts.copy()
    bad[0] = 1
    with pytest.raises(cc.CchError) as e:      # csf_start[0] != 0
        ctx.add_target_symmetry_csf(irr, bad, terms, coef, ci)
    assert e.value.code == cc.CCH_E_INPUT
    empty = np.concatenate([starts[:2], starts[1:]])   # CSF 1 has no term
    ci2 = np.vstack([ci, ci[:1]])
    with pytest.raises(cc.CchError) as e:
        ctx.add_target_symmetry_csf(irr, empty, terms, coef, ci2)
    assert e.value.code == cc.CCH_E_INPUT
    nan = coef.copy()
    nan[3] = np.nan
    with pytest.raises(cc.CchError) as e:
        ctx.add_target_symmetry_csf(irr, starts, terms, nan, ci)
    assert e.value.code == cc.CCH_E_INPUT
    with pytest.raises(cc.CchError) as e:      # more states than CSFs
        ctx.add_target_symmetry_csf(irr, starts[:3], terms[:starts[2]], coef[:starts[2]], ci[:2])
    assert e.value.code == cc.CCH_E_INVALID_ARG
    # a well-formed list is accepted after the refusals
    assert ctx.add_target_symmetry_csf(irr, starts, terms, coef, ci) == 0
    ctx.close()
