"""Jordan-Wigner Fock-space Hamiltonian for micro instances (TEST ONLY).

An independent route to the matrix elements of Eq. 3 (Sec. 2): the
second-quantised Hamiltonian
    H = sum_pq h_pq a+_p a_q + 1/2 sum_pqrs (pq|rs) a+_p a+_r a_s a_q + E_core
is assembled as a sparse matrix on the whole Fock space of n spin-orbitals,
with the textbook Jordan-Wigner annihilators built from Kronecker products,
    a_k = Z x ... x Z x s- x 1 x ... x 1   (k factors Z, s- = |0><1|).
No Slater-Condon rule is used. With mode 0 as the most significant factor,
the ascending determinant a+_k1 a+_k2 ... |0> (k1 < k2 < ...) is exactly the
basis vector with those modes occupied (coefficient +1), so <A|H|B> is a plain
matrix entry.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _annihilators(n):
    Z = sp.csr_matrix(np.diag([1.0, -1.0]))
    Id = sp.identity(2, format="csr")
    sm = sp.csr_matrix(np.array([[0.0, 1.0], [0.0, 0.0]]))
    ops = []
    for k in range(n):
        m = sp.identity(1, format="csr")
        for f in range(n):
            m = sp.kron(m, Z if f < k else (sm if f == k else Id), format="csr")
        ops.append(m)
    return ops


def spin_orbital_integrals(inst, X_spatial):
    """Dense spin-orbital tensors over all n = 2*n_orb spin-orbitals.
    X_spatial(p, q, r, s) gives the spatial (pq|rs) for global orbitals."""
    n = 2 * inst.n_orb
    h = np.zeros((n, n))
    g = np.zeros((n, n, n, n))
    for a in range(n):
        for b in range(n):
            if a % 2 == b % 2:
                h[a, b] = inst.h[a // 2, b // 2]
    for a in range(n):
        for b in range(n):
            if a % 2 != b % 2:
                continue
            for c in range(n):
                for d in range(n):
                    if c % 2 != d % 2:
                        continue
                    g[a, b, c, d] = X_spatial(a // 2, b // 2, c // 2, d // 2)
    return h, g


def full_spatial_eri(inst):
    """(pq|rs) over all orbitals for the integral classes that exist (at most
    two continuum indices), assembled from the stored arrays by the 8-fold
    permutational symmetry of real orbitals; entries with more than two
    continuum indices are never needed and left at zero."""
    no, nc = inst.n_o, inst.n_cont
    n = no + nc
    E = np.zeros((n, n, n, n))
    t, c = slice(0, no), slice(no, n)
    E[t, t, t, t] = inst.tttt
    # (pq|rj) and its images (pq|jr), (rj|pq), (jr|pq)
    E[t, t, t, c] = inst.tttc
    E[t, t, c, t] = inst.tttc.transpose(0, 1, 3, 2)
    E[t, c, t, t] = inst.tttc.transpose(2, 3, 0, 1)
    E[c, t, t, t] = inst.tttc.transpose(3, 2, 0, 1)
    # (pq|jj') and (jj'|pq)
    E[t, t, c, c] = inst.ttcc
    E[c, c, t, t] = inst.ttcc.transpose(2, 3, 0, 1)
    # (pj|qj') and its images (jp|qj'), (pj|j'q), (jp|j'q)
    E[t, c, t, c] = inst.tctc
    E[c, t, t, c] = inst.tctc.transpose(1, 0, 2, 3)
    E[t, c, c, t] = inst.tctc.transpose(0, 1, 3, 2)
    E[c, t, c, t] = inst.tctc.transpose(1, 0, 3, 2)
    return E


def fock_hamiltonian(inst):
    """Sparse Fock-space H over n = 2*(n_o + n_cont) spin-orbitals."""
    n = 2 * inst.n_orb
    if n > 14:
        raise ValueError("Fock space too large for the brute force")
    E = full_spatial_eri(inst)
    a = _annihilators(n)
    ad = [x.T.tocsr() for x in a]
    dim = 1 << n
    H = sp.csr_matrix((dim, dim))
    for p in range(n):
        for q in range(n):
            if p % 2 != q % 2:
                continue
            v = inst.h[p // 2, q // 2]
            if v != 0.0:
                H = H + v * (ad[p] @ a[q])
    for p in range(n):
        for q in range(n):
            if p % 2 != q % 2:
                continue
            for r in range(n):
                for s in range(n):
                    if r % 2 != s % 2:
                        continue
                    v = E[p // 2, q // 2, r // 2, s // 2]
                    if v == 0.0:
                        continue
                    H = H + (0.5 * v) * (ad[p] @ ad[r] @ a[s] @ a[q])
    H = H + inst.e_core * sp.identity(dim, format="csr")
    return H.tocsr()


def basis_index(occ, n):
    """Fock basis index of an occupation list (mode 0 most significant)."""
    idx = 0
    for k in occ:
        idx |= 1 << (n - 1 - k)
    return idx


def spin_squared(n):
    """S^2 = S- S+ + Sz^2 + Sz on the Fock space of n spin-orbitals (spin of
    mode k is k % 2, alpha = 0), with S+ = sum_k a+_{2k} a_{2k+1} and
    Sz = (1/2) sum_k (n_{2k} - n_{2k+1}); returns (S^2, Sz)."""
    a = _annihilators(n)
    ad = [x.T.tocsr() for x in a]
    dim = 1 << n
    Sp = sp.csr_matrix((dim, dim))
    Sz = sp.csr_matrix((dim, dim))
    for k in range(n // 2):
        Sp = Sp + ad[2 * k] @ a[2 * k + 1]
        Sz = Sz + 0.5 * (ad[2 * k] @ a[2 * k] - ad[2 * k + 1] @ a[2 * k + 1])
    Sm = Sp.T.tocsr()
    return (Sm @ Sp + Sz @ Sz + Sz).tocsr(), Sz.tocsr()
