"""CPU oracle for the close-coupling Hamiltonian: TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package. It shares no code with the GPU library: the two are fed
the same seeded inputs from `synth` and nothing else.

Contents
  * `ccoracle.c` (plain C, built here with gcc): Slater-Condon elements by
    explicit operator application, the CI-contracted matrix by the literal
    sums of Eqs. 4 and 5 (Sec. 2), the pure L2 elements (Sec. 2.2, classes 2
    and 8), and the determinant-pair excitation lists (Sec. 2.1).
  * `fock.py`: an independent Jordan-Wigner Fock-space construction of the
    same Hamiltonian for micro instances, used to pin the Slater-Condon code.
  * `lowest_eigenpairs`: the lowest eigenpairs by LAPACK (numpy.linalg.eigh),
    the plain definition of what the Davidson solve returns.
  * `csf_expand`: target CI vectors over multi-determinant CSFs (Eq. 2)
    rewritten over determinants.
  * `target_hamiltonian` and `energy_mode_matrix`: the N-electron target
    Hamiltonian over the determinants of two target symmetries, and the
    contracted matrix with the target-only integrals of classes 1, 3, 5, 6
    and 7 replaced by target energies on the diagonal (Sec. 3.1).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ccoracle.c")
_LIB = os.path.join(_HERE, "_ccoracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP)."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = C.CDLL(_LIB)
    P = C.c_void_p
    lib.orc_dim.restype = C.c_int64
    lib.orc_dim.argtypes = [P]
    lib.orc_build.restype = None
    lib.orc_build.argtypes = [P, C.c_int64, C.c_int64, P, P, P]
    lib.orc_build_rows.restype = None
    lib.orc_build_rows.argtypes = [P, C.c_int64, P, P, P, P]
    lib.orc_elements.restype = None
    lib.orc_elements.argtypes = [P, C.c_int64, P, P, P, P, P]
    lib.orc_pairs.restype = C.c_int64
    lib.orc_pairs.argtypes = [P, C.c_int, P, C.c_int, C.c_int, C.c_int, C.c_int64,
                              P, P, P, P, P]
    lib.orc_pairs_l2tgt.restype = C.c_int64
    lib.orc_pairs_l2tgt.argtypes = [P, C.c_int, P, C.c_int, C.c_int, C.c_int, C.c_int64,
                                    P, P, P, P, P]
    lib.orc_sc_lists.restype = None
    lib.orc_sc_lists.argtypes = [P, C.c_int, C.c_int64, P, P, P, P]
    lib.orc_excitation.restype = C.c_int
    lib.orc_excitation.argtypes = [P, P, C.c_int, P, P, P]
    lib.orc_num_threads.restype = C.c_int
    lib.orc_set_threads.restype = None
    lib.orc_set_threads.argtypes = [C.c_int]
    _lib = lib
    return lib


class _Ints(C.Structure):
    _fields_ = [("n_o", C.c_int32), ("n_cont", C.c_int32),
                ("h", C.c_void_p), ("tttt", C.c_void_p), ("tttc", C.c_void_p),
                ("ttcc", C.c_void_p), ("tctc", C.c_void_p), ("e_core", C.c_double),
                ("pk_rec", C.c_void_p), ("pk_blk", C.c_void_p), ("n_irrep", C.c_int32),
                ("t_irrep", C.c_void_p), ("c_irrep", C.c_void_p), ("c_local", C.c_void_p),
                ("c_count", C.c_void_p)]


class _Inst(C.Structure):
    _fields_ = [("ints", _Ints), ("n_elec", C.c_int32), ("n_words", C.c_int32),
                ("n_sym", C.c_int32), ("n_l2", C.c_int32), ("total_irrep", C.c_int32),
                ("cont_start", C.c_void_p), ("sym_irrep", C.c_void_p),
                ("sym_ndet", C.c_void_p), ("sym_nstate", C.c_void_p),
                ("sym_dets", C.c_void_p), ("sym_ci", C.c_void_p),
                ("l2_dets", C.c_void_p), ("sym_cspin", C.c_void_p)]


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class Oracle:
    """Holds an instance in the layout the C oracle reads."""

    def __init__(self, inst):
        if getattr(inst, "l2_csf_start", None) is not None:
            raise ValueError("L2 functions given as CSFs: use l2_csf_matrix")
        self.inst = inst
        keep = []

        def c(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            keep.append(a)
            return a
        pk = [None] * 6
        if getattr(inst, "packed", False):
            # the symmetry-packed (tt|cc) / (tc|tc) layout: record and block offsets
            import synth
            rec, blk = synth.packed_layout(inst.tgt_irrep, inst.n_c)
            ci = np.repeat(np.arange(inst.n_irrep), inst.n_c)
            loc = np.concatenate([np.arange(n) for n in inst.n_c]) if inst.n_cont else np.zeros(0)
            pk = [_ptr(c(rec, np.int64)), _ptr(c(blk.ravel(), np.int64)), _ptr(c(inst.tgt_irrep, np.int32)),
                  _ptr(c(ci, np.int32)), _ptr(c(loc, np.int32)), _ptr(c(inst.n_c, np.int32))]
        ints = _Ints(inst.n_o, inst.n_cont, _ptr(c(inst.h, np.float64)),
                     _ptr(c(inst.tttt, np.float64)), _ptr(c(inst.tttc, np.float64)),
                     _ptr(c(inst.ttcc, np.float64)), _ptr(c(inst.tctc, np.float64)),
                     float(inst.e_core), pk[0], pk[1], int(inst.n_irrep), pk[2], pk[3], pk[4], pk[5])
        cs = c(np.concatenate([[0], np.cumsum(inst.n_c)]), np.int32)
        irr = c([s.irrep for s in inst.syms], np.int32)
        nd = c([s.dets.shape[0] for s in inst.syms], np.int32)
        ns = c([s.ci.shape[1] for s in inst.syms], np.int32)
        dets = [c(s.dets, np.uint64) for s in inst.syms]
        cis = [c(s.ci, np.float64) for s in inst.syms]
        dp = c([d.ctypes.data for d in dets] or [0], np.uint64)
        cp = c([x.ctypes.data for x in cis] or [0], np.uint64)
        l2 = c(inst.l2_dets if inst.l2_dets is not None else np.zeros((0, inst.n_words)),
               np.uint64)
        # continuum spin per target determinant (NULL entries: alpha)
        spins = [c(s.cont_spin, np.int8) if getattr(s, "cont_spin", None) is not None else None
                 for s in inst.syms]
        sp = c([x.ctypes.data if x is not None else 0 for x in spins] or [0], np.uint64)
        any_spin = any(x is not None for x in spins)
        self._st = _Inst(ints, inst.n_elec, inst.n_words, len(inst.syms), l2.shape[0],
                         inst.total_irrep, _ptr(cs), _ptr(irr), _ptr(nd), _ptr(ns),
                         _ptr(dp), _ptr(cp), _ptr(l2), _ptr(sp) if any_spin else None)
        self._keep = keep
        self._ints = ints
        self.lib = _load()

    @property
    def dim(self) -> int:
        return int(self.lib.orc_dim(C.byref(self._st)))

    def build(self, r0=0, r1=None, with_abs=False):
        """Rows [r0, r1) of the dense contracted matrix; optionally the
        per-element sum of |terms| and term count."""
        D = self.dim
        r1 = D if r1 is None else min(r1, D)
        H = np.zeros((r1 - r0, D))
        A = np.zeros((r1 - r0, D)) if with_abs else None
        K = np.zeros((r1 - r0, D), dtype=np.int32) if with_abs else None
        self.lib.orc_build(C.byref(self._st), r0, r1, _ptr(H),
                           _ptr(A) if with_abs else None, _ptr(K) if with_abs else None)
        return (H, A, K) if with_abs else H

    def build_rows(self, rows, with_abs=False):
        """Full rows (listed, any order) of the dense contracted matrix."""
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        D = self.dim
        H = np.zeros((rows.size, D))
        A = np.zeros((rows.size, D)) if with_abs else None
        K = np.zeros((rows.size, D), dtype=np.int32) if with_abs else None
        self.lib.orc_build_rows(C.byref(self._st), rows.size, _ptr(rows), _ptr(H),
                                _ptr(A) if with_abs else None, _ptr(K) if with_abs else None)
        return (H, A, K) if with_abs else H

    def elements(self, rows, cols):
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        cols = np.ascontiguousarray(cols, dtype=np.int64)
        n = rows.size
        v = np.zeros(n); a = np.zeros(n); k = np.zeros(n, dtype=np.int32)
        self.lib.orc_elements(C.byref(self._st), n, _ptr(rows), _ptr(cols), _ptr(v),
                              _ptr(a), _ptr(k))
        return v, a, k

    def sc_lists(self, A, B):
        """Slater-Condon <A|H|B> for rows of two int arrays of ascending
        spin-orbital indices over the global index space."""
        A = np.ascontiguousarray(A, dtype=np.int32)
        B = np.ascontiguousarray(B, dtype=np.int32)
        npair, n = A.shape
        out = np.zeros(npair)
        self.lib.orc_sc_lists(C.byref(self._ints), n, npair, _ptr(A), _ptr(B), _ptr(out), None)
        return out


def _pairs_call(fn, args, cap):
    x = np.zeros(cap, np.int32); y = np.zeros(cap, np.int32)
    d = np.zeros(cap, np.int8); lab = np.zeros(cap, np.uint64); ph = np.zeros(cap, np.int8)
    n = fn(*args, cap, _ptr(x), _ptr(y), _ptr(d), _ptr(lab), _ptr(ph))
    if n > cap:
        return _pairs_call(fn, args, int(n))
    return dict(x=x[:n], y=y[:n], deg=d[:n], label=lab[:n], phase=ph[:n])


def pairs(a_dets, b_dets, lower=False):
    """Connected (degree <= 2) determinant pairs, bra a[x], ket b[y]."""
    lib = _load()
    a = np.ascontiguousarray(a_dets, dtype=np.uint64)
    b = np.ascontiguousarray(b_dets, dtype=np.uint64)
    return _pairs_call(lib.orc_pairs, (_ptr(a), a.shape[0], _ptr(b), b.shape[0], a.shape[1],
                                       int(lower)), max(16, a.shape[0] * 4))


def pairs_l2tgt(l2_dets, tgt_dets, n_o):
    """Continuum-L2 connected pairs (x = L2 index, y = target det index)."""
    lib = _load()
    a = np.ascontiguousarray(l2_dets, dtype=np.uint64)
    b = np.ascontiguousarray(tgt_dets, dtype=np.uint64)
    return _pairs_call(lib.orc_pairs_l2tgt, (_ptr(a), a.shape[0], _ptr(b), b.shape[0],
                                             a.shape[1], 2 * n_o), max(16, a.shape[0] * 4))


def excitation(A, B):
    """(degree, holes, particles, sign) of bra A from ket B (occupation lists)."""
    lib = _load()
    A = np.ascontiguousarray(A, dtype=np.int32)
    B = np.ascontiguousarray(B, dtype=np.int32)
    h = np.zeros(3, np.int32); p = np.zeros(3, np.int32); s = np.zeros(1, np.int32)
    deg = lib.orc_excitation(_ptr(A), _ptr(B), len(A), _ptr(h), _ptr(p), _ptr(s))
    k = deg if 0 <= deg <= 2 else 0
    return deg, list(h[:k]), list(p[:k]), int(s[0])


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (timing only)."""
    _load().orc_set_threads(int(n))


def lowest_eigenpairs(H, k):
    """The k lowest eigenpairs of a dense symmetric matrix (LAPACK syevd)."""
    w, v = np.linalg.eigh(H)
    return w[:k], v[:, :k]


def _occ_lists(dets):
    """Occupation lists of bitstring determinants (bit k of word k // 64 set
    means spin-orbital k is occupied), tested one bit at a time."""
    dets = np.asarray(dets, dtype=np.uint64)
    out = []
    for d in dets:
        out.append([64 * w + b for w in range(d.shape[0]) for b in range(64)
                    if (int(d[w]) >> b) & 1])
    return np.array(out, dtype=np.int32)


def csf_expand(dets, coef, starts, ci):
    """Target CI vectors over CSFs (Eq. 2) rewritten over determinants: CSF m
    is sum_t coef[t] |dets[t]> for t in [starts[m], starts[m+1]); phi_n =
    sum_m ci[m, n] eta_m = sum_d (sum over the terms of d of coef * ci[m, n]) |d>.
    Returns the distinct determinants in order of first appearance and their
    coefficients [n_det, n_states]; terms are added in input order."""
    dets = np.asarray(dets, dtype=np.uint64)
    index, order = {}, []
    for t in range(dets.shape[0]):
        key = tuple(int(w) for w in dets[t])
        if key not in index:
            index[key] = len(order)
            order.append(t)
    C = np.zeros((len(order), ci.shape[1]))
    for m in range(len(starts) - 1):
        for t in range(starts[m], starts[m + 1]):
            d = index[tuple(int(w) for w in dets[t])]
            for n in range(ci.shape[1]):
                C[d, n] += coef[t] * ci[m, n]
    return np.ascontiguousarray(dets[order]), C


def target_hamiltonian(inst, a, b):
    """<eta_am|H|eta_bm'> over the N-electron target determinants of target
    symmetries a (rows) and b (columns): the Hamiltonian of the target problem
    of Eq. 2 (target orbitals only, E_core on the diagonal), element by
    element by the Slater-Condon rules."""
    A = _occ_lists(inst.syms[a].dets)
    B = _occ_lists(inst.syms[b].dets)
    ma, mb = A.shape[0], B.shape[0]
    v = Oracle(inst).sc_lists(np.repeat(A, mb, axis=0), np.tile(B, (ma, 1)))
    return v.reshape(ma, mb)


def energy_mode_matrix(inst, energies, with_abs=False):
    """The contracted matrix with target energies on the diagonal (Sec. 3.1,
    the option of classes 1, 3, 5, 6 and 7). In a continuum element
    <(a,n,j)|H|(b,n',j')> the terms made of target orbitals only add up to
    delta_jj' (C_a^T H_T C_b)_nn', E_core included (the continuum electron is
    a spectator of them); they are removed and delta_ab delta_nn' delta_jj'
    E_an is added. energies[a] holds the S_a energies of symmetry a. With
    with_abs, the sum of |terms| and the term count of each element, for
    the tolerance rule, cover the removed and added terms too."""
    O = Oracle(inst)
    if with_abs:
        H, Ha, K = O.build(with_abs=True)
    else:
        H = O.build()
    row0, r = [], 0
    for s in inst.syms:
        row0.append(r)
        r += s.ci.shape[1] * int(inst.n_c[s.irrep ^ inst.total_irrep])
    for a, sa in enumerate(inst.syms):
        nc = int(inst.n_c[sa.irrep ^ inst.total_irrep])
        for b, sb in enumerate(inst.syms):
            if sb.irrep != sa.irrep or nc == 0:
                continue          # different continuum orbitals: no j = j'
            HT = target_hamiltonian(inst, a, b)
            P = sa.ci.T @ HT @ sb.ci
            Pa = np.abs(sa.ci).T @ np.abs(HT) @ np.abs(sb.ci)
            Sa_, Sb_ = sa.ci.shape[1], sb.ci.shape[1]
            for n in range(Sa_):
                for n2 in range(Sb_):
                    add = (energies[a][n] if (a == b and n == n2) else 0.0) - P[n, n2]
                    for j in range(nc):
                        i, k = row0[a] + n * nc + j, row0[b] + n2 * nc + j
                        H[i, k] += add
                        if with_abs:
                            Ha[i, k] += Pa[n, n2] + abs(energies[a][n]) * (a == b and n == n2)
                            K[i, k] += HT.size + 1
    return (H, Ha, K) if with_abs else H


def l2_csf_terms(inst):
    """(distinct L2 determinants in order of first appearance, the index of
    each term's determinant among them) of an instance whose L2 functions are
    CSFs."""
    index, ud, term = {}, [], []
    for d in inst.l2_dets:
        key = tuple(int(x) for x in d)
        if key not in index:
            index[key] = len(ud)
            ud.append(d)
        term.append(index[key])
    return np.array(ud, dtype=np.uint64).reshape(-1, inst.n_words), np.array(term, dtype=np.int64)


def l2_csf_matrix(inst, with_abs=False):
    """The contracted matrix when the L2 functions are CSFs (Eq. 1, second
    sum over configuration state functions chi_l = sum_t coef_t |det_t>): the
    plain definition, T^T H T, where H is the oracle's matrix over the
    continuum functions and the distinct L2 determinants, and T is the
    identity on the continuum rows with T[det(t), l] = coef_t. With with_abs,
    the sums of |terms| and the term counts of the tolerance rule carried
    through the same contraction."""
    import dataclasses
    ud, term = l2_csf_terms(inst)
    det_inst = dataclasses.replace(inst, l2_dets=ud, l2_csf_start=None, l2_coef=None)
    O = Oracle(det_inst)
    if with_abs:
        H, A, K = O.build(with_abs=True)
    else:
        H = O.build()
    Dc = det_inst.n_cont_rows()
    ncsf = len(inst.l2_csf_start) - 1
    T = np.zeros((Dc + len(ud), Dc + ncsf))
    T[:Dc, :Dc] = np.eye(Dc)
    for l in range(ncsf):
        for t in range(inst.l2_csf_start[l], inst.l2_csf_start[l + 1]):
            T[Dc + term[t], Dc + l] += inst.l2_coef[t]
    Hc = T.T @ H @ T
    if not with_abs:
        return Hc
    Ta, Tn = np.abs(T), (T != 0).astype(np.float64)
    return Hc, Ta.T @ A @ Ta, np.rint(Tn.T @ K @ Tn).astype(np.int64)


def tolerance_ok(g, o, abss, cnt, rel=1e-10):
    """Element parity rule: |g - o| <= max(rel*|o|, 2*K*u*A), with A the sum of
    |terms| and K the number of terms of the oracle's sum (a forward-error
    bound of recursive FP64 summation, so two correct summation orders may
    differ by it). Returns (mask_ok, mask_judged_by_floor)."""
    u = 2.0 ** -53
    floor = 2.0 * np.maximum(cnt, 1) * u * abss
    relb = rel * np.abs(o)
    err = np.abs(g - o)
    return err <= np.maximum(relb, floor), (err > relb) & (err <= floor)
