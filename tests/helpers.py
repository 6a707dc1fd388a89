"""Shared test helpers: basis bookkeeping written from the definitions
(Eq. 1 basis, Eq. 2 contraction), independent of both the oracle's C code
and the GPU library."""
from __future__ import annotations

import itertools

import numpy as np
import scipy.linalg.lapack as lapack

import synth


def uncontracted_functions(inst):
    """(N+1)-electron determinants of the uncontracted basis, in the order
    (symmetry i, target det m, continuum j) then L2 l; continuum electron
    u_j = spin-orbital 2*(n_o + j) + sigma_m, last (sigma_m the determinant's
    continuum spin, alpha unless given)."""
    funcs = []
    for s in inst.syms:
        a = s.irrep ^ inst.total_irrep
        j0, j1 = inst.cont_range(a)
        spin = getattr(s, "cont_spin", None)
        for m in range(s.dets.shape[0]):
            occ = synth.det_to_occ(s.dets[m])
            sig = 0 if spin is None else int(spin[m])
            for j in range(j0, j1):
                funcs.append(occ + [2 * (inst.n_o + j) + sig])
    for l in range(inst.n_l2):
        funcs.append(synth.det_to_occ(inst.l2_dets[l]))
    return funcs


def contraction_matrix(inst):
    """T = (+)_i (C_i x I_nc) (+) I_L2, mapping contracted rows (i, n, j)
    to uncontracted (i, m, j)."""
    blocks = []
    for s in inst.syms:
        a = s.irrep ^ inst.total_irrep
        nc = int(inst.n_c[a])
        blocks.append(np.kron(s.ci, np.eye(nc)))
    blocks.append(np.eye(inst.n_l2))
    rows = sum(b.shape[0] for b in blocks)
    cols = sum(b.shape[1] for b in blocks)
    T = np.zeros((rows, cols))
    r = c = 0
    for b in blocks:
        T[r:r + b.shape[0], c:c + b.shape[1]] = b
        r += b.shape[0]
        c += b.shape[1]
    return T


def perm_parity(seq):
    """(-1)^(number of inversions)."""
    inv = 0
    for a, b in itertools.combinations(range(len(seq)), 2):
        inv += seq[a] > seq[b]
    return -1 if inv % 2 else 1


def substitution_sign(A, B):
    """Sign s with A = s * (ket B with each hole replaced in place by its
    particle): the parity of the permutation that sorts the substituted ket.
    Holes/particles paired in ascending order."""
    holes = sorted(set(B) - set(A))
    parts = sorted(set(A) - set(B))
    sub = list(B)
    for h, p in zip(holes, parts):
        sub[sub.index(h)] = p
    return perm_parity(sub), holes, parts


def negative_inertia(A):
    """Number of negative eigenvalues of the symmetric matrix A (destroyed),
    from the 1x1 and 2x2 blocks of its Bunch-Kaufman factorisation."""
    n = A.shape[0]
    Af = A.T                      # C-ordered symmetric == Fortran-ordered, no copy
    lw = lapack.dsytrf_lwork(n, lower=1)
    ldu, ipiv, info = lapack.dsytrf(Af, lower=1, overwrite_a=1, lwork=int(lw[0]))
    assert info >= 0, info
    neg = 0
    i = 0
    while i < n:
        if ipiv[i] > 0:           # 1x1 block
            neg += ldu[i, i] < 0
            i += 1
        else:                     # 2x2 block [[a, b], [b, c]] in rows i, i+1
            a, b, c = ldu[i, i], ldu[i + 1, i], ldu[i + 1, i + 1]
            ev = np.linalg.eigvalsh(np.array([[a, b], [b, c]]))
            neg += int((ev < 0).sum())
            i += 2
    return neg
