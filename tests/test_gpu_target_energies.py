"""Target energies on the diagonal (Sec. 3.1, classes 1, 3, 5, 6 and 7),
through the C-ABI: element parity with the oracle's energy form on an
instance where two target symmetries share a continuum irrep (classes 5 and
6 between them) and a third couples to another (class 7); with CI vectors
that diagonalise the target Hamiltonian the option must give back the plain
matrix and its spectrum; the batched (graph-captured) build must equal the
single one bit for bit; and the option's misuse is refused."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _shared():
    return synth.make_instance(10, 6, 2, [12, 10], [0, 0, 1], [30, 25, 30], [2, 3, 2], 40, 4243,
                               e_core=-5.0, name="energies")


def _energies(inst, seed=9):
    rng = np.random.default_rng(seed)
    return [rng.uniform(-40.0, -35.0, s.ci.shape[1]) for s in inst.syms]


def test_energy_form_matches_oracle():
    import paper_1709_03005_amd as cc
    inst = _shared()
    E = _energies(inst)
    print("[energies] parity D =", inst.dim(), flush=True)
    H, A, K = oracle.energy_mode_matrix(inst, E, with_abs=True)
    with cc.from_instance(inst, target_energies=E) as ctx:
        ctx.build()
        G = ctx.get_matrix()
    ok, _ = oracle.tolerance_ok(G, H, A, K)
    assert ok.all(), np.argwhere(~ok)[:5]
    # the option did change the continuum block
    plain = oracle.Oracle(inst).build()
    Dc = inst.n_cont_rows()
    assert np.abs(G[:Dc, :Dc] - plain[:Dc, :Dc]).max() > 1.0


def test_target_eigenvectors_give_back_the_plain_matrix():
    import paper_1709_03005_amd as cc
    inst = synth.make_instance(10, 6, 2, [12, 10], [0, 1], [30, 28], [3, 2], 30, 4244,
                               e_core=-5.0, name="eigen")
    E = []
    for a, s in enumerate(inst.syms):
        w, v = np.linalg.eigh(oracle.target_hamiltonian(inst, a, a))
        S = s.ci.shape[1]
        s.ci = np.ascontiguousarray(v[:, :S])
        E.append(w[:S])
    print("[energies] eigenvector case D =", inst.dim(), flush=True)
    with cc.from_instance(inst) as c0, cc.from_instance(inst, target_energies=E) as c1:
        c0.build()
        c1.build()
        G0, G1 = c0.get_matrix(), c1.get_matrix()
        ev0, _, _, rc0 = c0.davidson(4, tol=1e-10, want_vectors=False)
        ev1, _, _, rc1 = c1.davidson(4, tol=1e-10, want_vectors=False)
    scale = np.abs(G0).max()
    assert np.abs(G1 - G0).max() <= 1e-12 * scale
    assert rc0 == rc1 == cc.CCH_OK
    assert np.all(np.abs(ev1 - ev0) <= 1e-10 * np.abs(ev0).max())


def test_batched_energy_form_equals_single_build():
    import paper_1709_03005_amd as cc
    insts = [_shared(), synth.tiny()]
    E = _energies(insts[0])
    ctxs = [cc.from_instance(insts[0], target_energies=E), cc.from_instance(insts[1])]
    solo = []
    for c in ctxs:
        c.build()
        solo.append(c.get_matrix())
    b = cc.Batch(ctxs, autotune=False)
    for rep in range(2):
        b.build()
        for c, G in zip(ctxs, solo):
            assert np.array_equal(c.get_matrix(), G)
    b.close()
    for c in ctxs:
        c.close()


def test_option_misuse_is_refused_and_can_be_switched_off():
    import paper_1709_03005_amd as cc
    inst = synth.tiny()
    E = _energies(inst)
    # wrong count, non-finite value
    with cc.from_instance(inst, plan=False) as ctx:
        with pytest.raises(cc.CchError) as e:
            ctx.set_target_energies([np.concatenate(E)[:-1]])
        assert e.value.code == cc.CCH_E_INPUT
        bad = [x.copy() for x in E]
        bad[0][0] = np.nan
        with pytest.raises(cc.CchError) as e:
            ctx.set_target_energies(bad)
        assert e.value.code == cc.CCH_E_INPUT
        # set, then switched off: the plain matrix
        ctx.set_target_energies(E)
        ctx.set_target_energies(None)
        ctx.plan()
        ctx.build()
        G = ctx.get_matrix()
        with pytest.raises(cc.CchError) as e:
            ctx.set_target_energies(E)          # after the plan
        assert e.value.code == cc.CCH_E_STATE
    with cc.from_instance(inst) as ref:
        ref.build()
        assert np.array_equal(G, ref.get_matrix())
    # a symmetry added after the energies: the plan refuses
    with cc.from_instance(inst, plan=False) as ctx:
        ctx.set_target_energies(E)
        s = inst.syms[0]
        ctx.add_target_symmetry(s.irrep, s.dets, s.ci)
        with pytest.raises(cc.CchError) as e:
            ctx.plan()
        assert e.value.code == cc.CCH_E_STATE


def _true_target_states(Hs, inst):
    """CI vectors and energies of the paired instance from the target
    Hamiltonian of each determinant space: the first member of a pair takes
    the lowest S eigenvectors, the second the next S."""
    E = []
    for a in range(0, len(inst.syms), 2):
        w, v = np.linalg.eigh(Hs[a])
        S = inst.syms[a].ci.shape[1]
        inst.syms[a].ci = np.ascontiguousarray(v[:, :S])
        inst.syms[a + 1].ci = np.ascontiguousarray(v[:, S:2 * S])
        E += [w[:S], w[S:2 * S]]
    return E


def test_target_hamiltonian_readout():
    """cch_target_hamiltonian against the oracle's Slater-Condon target
    Hamiltonian, for every pair of symmetries (same and different irreps,
    both orders)."""
    import paper_1709_03005_amd as cc
    inst = _shared()
    with cc.from_instance(inst) as ctx:
        ctx.build()
        for a in range(len(inst.syms)):
            for b in range(len(inst.syms)):
                g = ctx.target_hamiltonian(a, b)
                o = oracle.target_hamiltonian(inst, a, b)
                assert g.shape == o.shape
                np.testing.assert_allclose(g, o, rtol=0, atol=1e-12 * max(1.0, np.abs(o).max()))


def test_true_target_states_paired_symmetries():
    """The target-energy option with true target states: CI vectors and
    energies from the library's own target Hamiltonian (eigh on the host), on
    pairs of symmetries sharing one determinant space (classes 5 and 6 between
    the members of a pair, class 7 across pairs). Every element against the
    oracle's energy form; the plain build with the same CI vectors has the
    same matrix to rounding (the states diagonalise the target Hamiltonian),
    and both share their lowest eigenvalues."""
    import paper_1709_03005_amd as cc
    inst = synth.paired(12, 6, 100, 3, 20, 300, seed=5, name="pairs_small")
    with cc.from_instance(inst) as c0:
        c0.build()
        Hs = {a: c0.target_hamiltonian(a, a) for a in range(0, 4, 2)}
    E = _true_target_states(Hs, inst)
    H, A, K = oracle.energy_mode_matrix(inst, E, with_abs=True)
    with cc.from_instance(inst, target_energies=E) as ce, cc.from_instance(inst) as cp:
        ce.build()
        cp.build()
        G, Gp = ce.get_matrix(), cp.get_matrix()
        b5 = ce.get_block(5, 1, 0)
        b6 = ce.get_block(6, 1, 0)
        ev, _, _, rc = ce.davidson(5, tol=1e-10, want_vectors=False)
        evp, _, _, rcp = cp.davidson(5, tol=1e-10, want_vectors=False)
    ok, _ = oracle.tolerance_ok(G, H, A, K)
    assert ok.all(), np.argwhere(~ok)[:5]
    assert np.abs(b5).max() > 0 and np.abs(b6).max() > 0
    scale = np.abs(H).max()
    assert np.abs(G - Gp).max() < 1e-9 * scale
    assert rc == rcp == cc.CCH_OK
    assert np.abs(ev - evp).max() < 1e-9 * scale
