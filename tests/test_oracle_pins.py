"""Pins of the CPU oracle against what the mathematics fixes (no GPU).

* Slater-Condon elements == Jordan-Wigner Fock-space matrix elements
  (a construction that uses no Slater-Condon rule) on micro instances.
* The contracted matrix == T^T H T with H from the Fock space (Eqs. 4, 5).
* C = I reproduces the uncontracted matrix; a CI rotation C -> CQ maps the
  contracted matrix to (Q x I)^T H (Q x I); Cauchy interlacing between the
  uncontracted and contracted spectra; Hermiticity of independently computed
  triangles; invariance of the spectrum under a relabelling of target orbitals.
* Excitation lists: degree from set differences and sign from the parity of
  the in-place substituted ket, including 64-bit word boundaries (Sec. 2.1).
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import fock
from tests.helpers import contraction_matrix, substitution_sign, uncontracted_functions

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

MICROS = [
    dict(seed=1, n_o=3, n_elec=2, n_c=2),
    dict(seed=2, n_o=3, n_elec=2, n_c=2, n_states=2),
    dict(seed=3, n_o=4, n_elec=2, n_c=1, n_irrep=2, n_states=2),
    dict(seed=4, n_o=4, n_elec=4, n_c=1, n_states=3),
]


def _fock_block(inst):
    HF = fock.fock_hamiltonian(inst)
    funcs = uncontracted_functions(inst)
    n = 2 * inst.n_orb
    idx = [fock.basis_index(f, n) for f in funcs]
    return HF[idx][:, idx].toarray(), funcs


@pytest.mark.parametrize("kw", MICROS)
def test_slater_condon_equals_fock_space(kw):
    inst = synth.micro(**kw)
    Hf, funcs = _fock_block(inst)
    O = oracle.Oracle(inst)
    A = np.array([f for f in funcs for _ in funcs])
    B = np.array([g for _ in funcs for g in funcs])
    sc = O.sc_lists(A, B).reshape(len(funcs), len(funcs))
    assert np.abs(Hf).max() > 0.1
    np.testing.assert_allclose(sc, Hf, rtol=0, atol=1e-13)


@pytest.mark.parametrize("kw", MICROS)
def test_contracted_equals_TtHT_from_fock_space(kw):
    inst = synth.micro(**kw)
    Hf, _ = _fock_block(inst)
    T = contraction_matrix(inst)
    ref = T.T @ Hf @ T
    got = oracle.Oracle(inst).build()
    assert got.shape == ref.shape == (inst.dim(), inst.dim())
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)


def test_two_electron_closed_form():
    """<ab|H|ab> = h_aa + h_bb + (aa|bb) - delta_spin (ab|ba) for N+1 = 2."""
    inst = synth.tiny()
    O = oracle.Oracle(inst)
    no = inst.n_o
    tt = [(0, 1), (0, 2), (3, 8), (4, 19)]                       # both target
    tc = [(2, 2 * (no + 4)), (5, 2 * (no + 7)), (6, 2 * (no + 1))]  # target + continuum
    got = O.sc_lists(np.array(tt + tc), np.array(tt + tc))
    for (a, b), g in zip(tt, got[:len(tt)]):
        P, Q = a // 2, b // 2
        ref = inst.h[P, P] + inst.h[Q, Q] + inst.tttt[P, P, Q, Q]
        if a % 2 == b % 2:
            ref -= inst.tttt[P, Q, Q, P]
        assert abs(g - ref) < 1e-14
    for (a, b), g in zip(tc, got[len(tt):]):
        P, J = a // 2, b // 2 - no
        ref = inst.h[P, P] + inst.h[no + J, no + J] + inst.ttcc[P, P, J, J]
        if a % 2 == b % 2:
            ref -= inst.tctc[P, J, P, J]
        assert abs(g - ref) < 1e-14


def test_identity_contraction_gives_uncontracted():
    """C = I (one state per determinant): the contraction is the identity."""
    inst = synth.micro(7, n_o=3, n_elec=2, n_c=2)
    for s in inst.syms:
        s.ci = np.eye(s.dets.shape[0])
    funcs = uncontracted_functions(inst)
    O = oracle.Oracle(inst)
    A = np.array([f for f in funcs for _ in funcs])
    B = np.array([g for _ in funcs for g in funcs])
    sc = O.sc_lists(A, B).reshape(len(funcs), len(funcs))
    np.testing.assert_allclose(O.build(), sc, rtol=0, atol=1e-14)


def test_ci_rotation_covariance_and_interlacing():
    inst = synth.tiny()
    O = oracle.Oracle(inst)
    H1 = O.build()
    # Cauchy interlacing against the uncontracted matrix
    funcs = uncontracted_functions(inst)
    A = np.array([f for f in funcs for _ in funcs])
    B = np.array([g for _ in funcs for g in funcs])
    Hu = O.sc_lists(A, B).reshape(len(funcs), len(funcs))
    lu = np.linalg.eigvalsh(Hu)
    lc = np.linalg.eigvalsh(H1)
    k = len(lc)
    assert np.all(lu[:k] <= lc + 1e-10)
    assert np.all(lc <= lu[len(lu) - k:] + 1e-10)
    # T^T Hu T reproduces the contracted matrix
    T = contraction_matrix(inst)
    np.testing.assert_allclose(T.T @ Hu @ T, H1, rtol=0, atol=1e-12)
    # rotation of the CI vectors
    rng = np.random.default_rng(5)
    S = inst.syms[0].ci.shape[1]
    Q, _ = np.linalg.qr(rng.standard_normal((S, S)))
    inst.syms[0].ci = inst.syms[0].ci @ Q
    H2 = oracle.Oracle(inst).build()
    nc = int(inst.n_c[0])
    R = np.eye(inst.dim())
    R[:S * nc, :S * nc] = np.kron(Q, np.eye(nc))
    np.testing.assert_allclose(H2, R.T @ H1 @ R, rtol=0, atol=1e-12)


@pytest.mark.parametrize("make", [synth.tiny, synth.small])
def test_hermitian(make):
    H = oracle.Oracle(make()).build()
    assert np.abs(H - H.T).max() < 1e-13
    assert np.abs(H).max() > 1.0


def _permute_target_orbitals(inst, perm):
    """Relabel target orbital p -> perm[p] (same irreps), carrying integrals,
    determinants and CI signs along; L2 dets are reordered the same way."""
    no = inst.n_o
    full = np.concatenate([perm, np.arange(no, inst.n_orb)])
    inv = np.argsort(full)
    h = inst.h[np.ix_(inv, inv)]
    it = np.argsort(perm)
    tttt = inst.tttt[np.ix_(it, it, it, it)]
    tttc = inst.tttc[np.ix_(it, it, it, np.arange(inst.n_cont))]
    ttcc = inst.ttcc[np.ix_(it, it, np.arange(inst.n_cont), np.arange(inst.n_cont))]
    tctc = inst.tctc[np.ix_(it, np.arange(inst.n_cont), it, np.arange(inst.n_cont))]

    def mapdet(d):
        occ = synth.det_to_occ(d)
        new = [2 * int(perm[k // 2]) + (k % 2) for k in occ]
        from tests.helpers import perm_parity
        sign = perm_parity(new)
        return synth.occ_to_det(sorted(new), len(d)), sign
    syms = []
    for s in inst.syms:
        dets = np.zeros_like(s.dets)
        ci = s.ci.copy()
        for m in range(s.dets.shape[0]):
            dets[m], sg = mapdet(s.dets[m])
            ci[m] *= sg
        syms.append(synth.TargetSym(s.irrep, dets, ci))
    l2 = np.zeros_like(inst.l2_dets)
    for l in range(inst.n_l2):
        l2[l], _ = mapdet(inst.l2_dets[l])
    return synth.Instance(n_o=no, n_elec=inst.n_elec, n_irrep=inst.n_irrep,
                          tgt_irrep=inst.tgt_irrep, n_c=inst.n_c, total_irrep=0, h=h,
                          tttt=tttt, tttc=tttc, ttcc=ttcc, tctc=tctc, e_core=inst.e_core,
                          syms=syms, l2_dets=l2)


def test_spectrum_invariant_under_orbital_relabelling():
    inst = synth.tiny()
    l1 = np.linalg.eigvalsh(oracle.Oracle(inst).build())
    perm = np.random.default_rng(3).permutation(inst.n_o)
    inst2 = _permute_target_orbitals(inst, perm)
    H2 = oracle.Oracle(inst2).build()
    l2 = np.linalg.eigvalsh(H2)
    np.testing.assert_allclose(l2, l1, rtol=0, atol=1e-11)


def _check_pairs(res, a_dets, b_dets, lower, cont_slot=None):
    """Every listed pair's degree/label/sign from set differences and the
    in-place substitution parity; and nothing connected is missing."""
    seen = set()
    for x, y, d, lab, ph in zip(res["x"], res["y"], res["deg"], res["label"], res["phase"]):
        A = synth.det_to_occ(a_dets[x])
        B = synth.det_to_occ(b_dets[y])
        if cont_slot is not None:
            bra, ket = B + [cont_slot], A     # continuum function vs L2
        else:
            bra, ket = A, B
        s, holes, parts = substitution_sign(bra, ket)
        assert len(holes) == d
        assert s == ph
        f = [(int(lab) >> (16 * k)) & 0xFFFF for k in range(4)]
        if cont_slot is None:
            exp = [parts[0] if d >= 1 else 0xFFFF, holes[0] if d >= 1 else 0xFFFF,
                   parts[1] if d >= 2 else 0xFFFF, holes[1] if d >= 2 else 0xFFFF]
        else:
            tp = [p for p in parts if p != cont_slot]
            exp = [tp[0] if tp else 0xFFFF, holes[0], holes[1] if d >= 2 else 0xFFFF, 0xFFFF]
        assert f == exp
        seen.add((int(x), int(y)))
    for x in range(len(a_dets)):
        for y in range(len(b_dets) if not lower else x + 1):
            A = set(synth.det_to_occ(a_dets[x]))
            B = set(synth.det_to_occ(b_dets[y]))
            if cont_slot is not None:
                conn = len(B - A) <= 1 and len(A) == len(B) + 1
            else:
                conn = len(A - B) <= 2 and len(A) == len(B)
            assert conn == ((x, y) in seen)


def test_pair_lists_tiny():
    inst = synth.tiny()
    d = inst.syms[0].dets
    _check_pairs(oracle.pairs(d, d), d, d, False)
    _check_pairs(oracle.pairs(inst.l2_dets, inst.l2_dets, lower=True), inst.l2_dets,
                 inst.l2_dets, True)
    _check_pairs(oracle.pairs_l2tgt(inst.l2_dets, d, inst.n_o), inst.l2_dets, d, False,
                 cont_slot=2 * inst.n_o)


def test_pair_lists_cross_word_boundary():
    inst = synth.wide()
    d = inst.syms[0].dets[:60]
    occs = [synth.det_to_occ(x) for x in d]
    assert any(max(o) >= 64 for o in occs) and any(min(o) < 64 for o in occs)
    _check_pairs(oracle.pairs(d, d), d, d, False)
    l2 = inst.l2_dets[:60]
    _check_pairs(oracle.pairs_l2tgt(l2, d, inst.n_o), l2, d, False, cont_slot=2 * inst.n_o)


def test_word_boundary_fixtures():
    """Hand-derived excitation signs at spin-orbitals 63/64/127/128
    (tests/golden/word_boundary.json; derivation in the file)."""
    with open(os.path.join(GOLDEN, "word_boundary.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        deg, holes, parts, sign = oracle.excitation(c["bra"], c["ket"])
        assert deg == c["degree"], c
        assert holes == c["holes"] and parts == c["particles"], c
        assert sign == c["sign"], c
        # uniform shift of every index leaves the sign unchanged
        sh = 64
        deg2, _, _, sign2 = oracle.excitation([k + sh for k in c["bra"]],
                                              [k + sh for k in c["ket"]])
        assert (deg2, sign2) == (deg, sign)


def test_tolerance_rule_catches_planted_error():
    """A planted wrong sign in an exchange term shows up under the rule."""
    inst = synth.tiny()
    O = oracle.Oracle(inst)
    H, A, K = O.build(with_abs=True)
    bad = H.copy()
    bad[70, 3] += 1e-6
    ok, _ = oracle.tolerance_ok(bad, H, A, K)
    assert not ok[70, 3] and ok.sum() == ok.size - 1


def test_sampled_elements_equal_full_build():
    inst = synth.small()
    O = oracle.Oracle(inst)
    H = O.build()
    rng = np.random.default_rng(0)
    D = inst.dim()
    rows = rng.integers(0, D, 200)
    cols = rng.integers(0, D, 200)
    v, a, k = O.elements(rows, cols)
    np.testing.assert_allclose(v, H[rows, cols], rtol=0, atol=1e-13)


# ---------------------------------------------------------------------------
# target energies on the diagonal (Sec. 3.1, classes 1, 3, 5, 6, 7)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kw", MICROS)
def test_target_hamiltonian_equals_fock_space(kw):
    """The N-electron target Hamiltonian == the Jordan-Wigner Fock-space
    operator between the same determinants (no Slater-Condon rule there)."""
    inst = synth.micro(**kw)
    HF = fock.fock_hamiltonian(inst)
    n = 2 * inst.n_orb
    for a, s in enumerate(inst.syms):
        idx = [fock.basis_index(synth.det_to_occ(d), n) for d in s.dets]
        ref = HF[idx][:, idx].toarray()
        got = oracle.target_hamiltonian(inst, a, a)
        assert np.abs(ref).max() > 0.1
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)


def _shared_irrep_instance():
    # symmetries 0 and 1 share irrep 0 (classes 5 and 6 between them), symmetry
    # 2 couples to the other continuum irrep (class 7); a non-zero core energy
    return synth.make_instance(6, 4, 2, [3, 2], [0, 0, 1], [9, 7, 8], [2, 3, 2], 6, 777,
                               e_core=-3.7, name="energies")


def test_energy_mode_equals_removing_target_only_integrals():
    """The energy-mode matrix on the continuum block == the plain build with
    every integral over target orbitals only (h_pq, (pq|rs)) and E_core set to
    zero, plus the energies on the diagonal; class 4 and the L2 block keep the
    plain build's values."""
    import dataclasses
    inst = _shared_irrep_instance()
    no = inst.n_o
    h2 = inst.h.copy()
    h2[:no, :no] = 0.0
    bare = dataclasses.replace(inst, h=h2, tttt=np.zeros_like(inst.tttt), e_core=0.0)
    rng = np.random.default_rng(5)
    E = [rng.uniform(-20.0, -15.0, s.ci.shape[1]) for s in inst.syms]
    got = oracle.energy_mode_matrix(inst, E)
    full = oracle.Oracle(inst).build()
    ref = oracle.Oracle(bare).build()
    Dc = inst.n_cont_rows()
    r = 0
    for a, s in enumerate(inst.syms):
        nc = int(inst.n_c[s.irrep ^ inst.total_irrep])
        for n in range(s.ci.shape[1]):
            for j in range(nc):
                ref[r, r] += E[a][n]
                r += 1
    assert r == Dc
    scale = np.abs(full).max()
    np.testing.assert_allclose(got[:Dc, :Dc], ref[:Dc, :Dc], rtol=0, atol=1e-12 * scale)
    np.testing.assert_array_equal(got[Dc:], full[Dc:])
    np.testing.assert_array_equal(got[:, Dc:], full[:, Dc:])
    # the option changes something: the removed part is not zero
    assert np.abs(got[:Dc, :Dc] - full[:Dc, :Dc]).max() > 0.1


def test_energy_mode_with_target_eigenvectors_reproduces_full_build():
    """With CI vectors that diagonalise the target Hamiltonian and their
    eigenvalues as energies, the option reproduces the plain matrix."""
    inst = synth.make_instance(6, 4, 2, [3, 2], [0, 1], [10, 9], [3, 2], 5, 778,
                               e_core=-2.5, name="eigen")
    E = []
    for a, s in enumerate(inst.syms):
        w, v = np.linalg.eigh(oracle.target_hamiltonian(inst, a, a))
        S = s.ci.shape[1]
        s.ci = np.ascontiguousarray(v[:, :S])
        E.append(w[:S])
    full = oracle.Oracle(inst).build()
    got = oracle.energy_mode_matrix(inst, E)
    np.testing.assert_allclose(got, full, rtol=0, atol=1e-12 * np.abs(full).max())


# ---------------------------------------------------------------------------
# target states over multi-determinant CSFs (Eq. 2)
# ---------------------------------------------------------------------------

def _csf_lists(inst, seed):
    """CSFs of one or two determinants each over the first symmetry's
    determinants (fixed random coefficients), every determinant used."""
    rng = np.random.default_rng(seed)
    dets = inst.syms[0].dets
    M = dets.shape[0]
    perm = rng.permutation(M)
    terms, coef, starts = [], [], [0]
    i = 0
    while i < M:
        k = 1 if (i + 1 == M or rng.random() < 0.4) else 2
        for t in range(k):
            terms.append(dets[perm[i + t]])
            coef.append(1.0 if k == 1 else rng.choice([-1.0, 1.0]) / np.sqrt(2.0))
        starts.append(len(terms))
        i += k
    return np.array(terms, dtype=np.uint64), np.array(coef), starts


def test_csf_expand_single_determinants_is_identity():
    inst = synth.tiny()
    s = inst.syms[0]
    d, C = oracle.csf_expand(s.dets, np.ones(s.dets.shape[0]), list(range(s.dets.shape[0] + 1)), s.ci)
    np.testing.assert_array_equal(d, s.dets)
    np.testing.assert_array_equal(C, s.ci)


@pytest.mark.parametrize("kw", MICROS[:2])
def test_csf_targets_equal_fock_space(kw):
    """Contracted continuum block of CSF-expanded targets == the same elements
    formed in the Fock space from the CSF combinations themselves (the CSF
    vector sum_t coef_t |det_t u_j>, then v^T H v'): neither Slater-Condon nor
    csf_expand on that side."""
    import dataclasses
    inst = synth.micro(**kw)
    terms, coef, starts = _csf_lists(inst, 7)
    ncsf = len(starts) - 1
    rng = np.random.default_rng(8)
    S = min(2, ncsf)
    ci = np.linalg.qr(rng.standard_normal((ncsf, S)))[0]
    d, C = oracle.csf_expand(terms, coef, starts, ci)
    s0 = inst.syms[0]
    exp = dataclasses.replace(inst, syms=[synth.TargetSym(s0.irrep, d, C)], l2_dets=inst.l2_dets[:0])
    got = oracle.Oracle(exp).build()
    HF = fock.fock_hamiltonian(inst)
    n = 2 * inst.n_orb
    nc = int(inst.n_c[s0.irrep ^ inst.total_irrep])
    j0 = inst.cont_range(s0.irrep ^ inst.total_irrep)[0]
    vecs = []
    for st in range(S):
        for j in range(nc):
            v = np.zeros(1 << n)
            for m in range(ncsf):
                for t in range(starts[m], starts[m + 1]):
                    occ = synth.det_to_occ(terms[t]) + [2 * (inst.n_o + j0 + j)]
                    v[fock.basis_index(occ, n)] += coef[t] * ci[m, st]
            vecs.append(v)
    Vm = np.array(vecs).T
    ref = Vm.T @ (HF @ Vm)
    assert got.shape == ref.shape
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("kw", [dict(seed=11, n_o=3, n_elec=2, n_c=2), dict(seed=12, n_o=4, n_elec=2, n_c=1)])
def test_l2_csfs_equal_fock_space(kw):
    """L2 functions as doublet CSFs: the oracle's contracted matrix equals
    V^T H V formed in the Fock space from the CSF combinations themselves
    (the L2 CSF vector sum_t coef_t |det_t>, the continuum functions
    sum_m c_mn |det_m u_j>), with no Slater-Condon rule on that side. The
    doublets are orthonormal Fock-space vectors."""
    inst = synth.l2_spin_adapted(synth.micro(**kw))
    ncsf = len(inst.l2_csf_start) - 1
    assert ncsf >= 2 and np.any(np.diff(inst.l2_csf_start) == 3)
    got = oracle.l2_csf_matrix(inst)
    HF = fock.fock_hamiltonian(inst)
    n = 2 * inst.n_orb
    vecs = []
    for s in inst.syms:
        a = s.irrep ^ inst.total_irrep
        j0, j1 = inst.cont_range(a)
        for st in range(s.ci.shape[1]):
            for j in range(j0, j1):
                v = np.zeros(1 << n)
                for m in range(s.dets.shape[0]):
                    v[fock.basis_index(synth.det_to_occ(s.dets[m]) + [2 * (inst.n_o + j)], n)] += s.ci[m, st]
                vecs.append(v)
    L = []
    for l in range(ncsf):
        v = np.zeros(1 << n)
        for t in range(inst.l2_csf_start[l], inst.l2_csf_start[l + 1]):
            v[fock.basis_index(synth.det_to_occ(inst.l2_dets[t]), n)] += inst.l2_coef[t]
        L.append(v)
    Lm = np.array(L).T
    np.testing.assert_allclose(Lm.T @ Lm, np.eye(ncsf), atol=1e-14)
    Vm = np.array(vecs + L).T
    ref = Vm.T @ (HF @ Vm)
    assert got.shape == ref.shape
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)


TD_MICROS = [dict(seed=1, n_o=3, n_elec=2, n_c=2), dict(seed=3, n_o=4, n_elec=2, n_c=1, n_irrep=2, n_states=2),
             dict(seed=4, n_o=4, n_elec=4, n_c=1, n_states=3)]


@pytest.mark.parametrize("kw", TD_MICROS)
def test_triplet_doublet_channels_are_doublets(kw):
    """The triplet-coupled channel functions of the test inputs are doublets:
    S^2 v = 3/4 v and S_z v = 1/2 v in the Fock space, with the continuum
    electron's spin taken from its determinant (the data the beta-continuum
    parity rests on)."""
    inst = synth.triplet_doublet(synth.micro(**kw), seed=7)
    assert any(np.any(s.cont_spin == 1) for s in inst.syms)
    n = 2 * inst.n_orb
    S2, Sz = fock.spin_squared(n)
    funcs = uncontracted_functions(inst)
    T = contraction_matrix(inst)
    Dc = inst.n_cont_rows()
    V = np.zeros((1 << n, Dc))
    for i, f in enumerate(funcs):
        if i < T.shape[0] - inst.n_l2:
            V[fock.basis_index(f, n)] += T[i, :Dc]
    assert np.abs(V).max() > 0.1
    np.testing.assert_allclose(S2 @ V, 0.75 * V, rtol=0, atol=1e-13)
    np.testing.assert_allclose(Sz @ V, 0.5 * V, rtol=0, atol=1e-13)


@pytest.mark.parametrize("kw", TD_MICROS)
def test_triplet_doublet_contracted_equals_fock_space(kw):
    """Beta continuum electrons (doublet coupling of triplet targets): the
    oracle's contracted matrix, from its build and from its sampled-element
    path, equals T^T H T in the Fock space with each continuum electron at
    2 (n_o + j) + sigma."""
    inst = synth.triplet_doublet(synth.micro(**kw), seed=7)
    Hf, _ = _fock_block(inst)
    T = contraction_matrix(inst)
    ref = T.T @ Hf @ T
    O = oracle.Oracle(inst)
    got = O.build()
    assert got.shape == ref.shape == (inst.dim(), inst.dim())
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)
    r, c = np.meshgrid(np.arange(inst.dim()), np.arange(inst.dim()), indexing="ij")
    np.testing.assert_allclose(O.elements(r.ravel(), c.ravel())[0].reshape(got.shape), ref, rtol=0, atol=1e-13)
    # the spin-flip exchange elements are there: channels of different continuum spin couple
    assert np.abs(ref[:inst.n_cont_rows(), :inst.n_cont_rows()]).max() > 0.1
