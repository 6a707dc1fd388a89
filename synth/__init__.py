"""Seeded synthetic inputs for the close-coupling Hamiltonian build.

This module only draws random numbers and enumerates determinants; it holds
none of the Hamiltonian arithmetic. Both the CPU oracle and the GPU library
are fed from it, so it must never import either of them.

What is generated (the paper's problem statement, Sec. 2, Eqs. 1-2):
  * orbital symmetries: an abelian point group with irreps 0..n_irrep-1 whose
    product is XOR; target orbital p has irrep p mod n_irrep; continuum
    orbitals come n_c[a] per irrep a, irrep-major, after all target orbitals;
  * real one-electron integrals h (all orbitals) and the two-electron classes
    with at most two continuum indices (each N+1 function holds at most one
    continuum electron): tttt, tttc, ttcc, tctc (chemists' notation);
  * target determinants per target symmetry, as bitstrings over target
    spin-orbitals k = 2*orbital + spin (alpha = 0), 64 per uint64 word;
  * target CI vectors (Eq. 2): orthonormal columns from a seeded QR;
  * L2 determinants with N+1 electrons in target orbitals (Eq. 1, second sum).

Distributions (global orbital indices in the decay factors):
  h_pq ~ N(0, 1) * exp(-|p-q|/4), zero unless irrep(p) == irrep(q);
  (pq|rs) ~ N(0, 0.1) * exp(-(|p-q|+|r-s|)/4), drawn once per 8-fold
  canonical index, zero unless irrep(p)^irrep(q)^irrep(r)^irrep(s) == 0.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Instance", "TargetSym", "make_instance", "det_to_occ", "occ_to_det",
    "tiny", "small", "wide", "medium", "precision", "learned_test",
    "learned_train", "batch_instance", "micro", "boundary", "mid", "CONFIGS",
]


@dataclass
class TargetSym:
    irrep: int
    dets: np.ndarray      # uint64 [M, W]
    ci: np.ndarray        # float64 [M, S] row-major
    cont_spin: np.ndarray = None   # int8 [M]: continuum spin per det (0 alpha, 1 beta); None: alpha


@dataclass
class Instance:
    n_o: int
    n_elec: int                  # N, target electrons
    n_irrep: int
    tgt_irrep: np.ndarray        # uint8 [n_o]
    n_c: np.ndarray              # int32 [n_irrep], continuum orbitals per irrep
    total_irrep: int
    h: np.ndarray                # [n_orb, n_orb]
    tttt: np.ndarray             # [n_o, n_o, n_o, n_o]      (pq|rs)
    tttc: np.ndarray             # [n_o, n_o, n_o, n_cont]   (pq|rj)
    ttcc: np.ndarray             # [n_o, n_o, n_cont, n_cont] (pq|jj')
    tctc: np.ndarray             # [n_o, n_cont, n_o, n_cont] (pj|qj')
    e_core: float
    syms: list = field(default_factory=list)   # list[TargetSym]
    l2_dets: np.ndarray = None   # uint64 [n_l2, W]
    name: str = ""
    seed: int = 0
    packed: bool = False         # ttcc / tctc hold the symmetry-packed layout (packed_layout)
    # L2 functions as CSFs: function l = sum of l2_coef[t] |l2_dets[t]> over
    # t in [l2_csf_start[l], l2_csf_start[l + 1]) (None: one determinant each)
    l2_csf_start: np.ndarray = None
    l2_coef: np.ndarray = None

    @property
    def n_cont(self) -> int:
        return int(np.sum(self.n_c))

    @property
    def n_orb(self) -> int:
        return self.n_o + self.n_cont

    @property
    def n_words(self) -> int:
        return (2 * self.n_o + 63) // 64

    @property
    def cont_irrep(self) -> np.ndarray:
        return np.repeat(np.arange(self.n_irrep, dtype=np.uint8), self.n_c)

    @property
    def orb_irrep(self) -> np.ndarray:
        return np.concatenate([self.tgt_irrep, self.cont_irrep]).astype(np.uint8)

    @property
    def n_l2(self) -> int:
        if self.l2_csf_start is not None:
            return int(len(self.l2_csf_start) - 1)
        return 0 if self.l2_dets is None else int(self.l2_dets.shape[0])

    def cont_range(self, irrep: int) -> tuple[int, int]:
        """Continuum orbitals of one irrep, as a [start, stop) range of j."""
        off = int(np.sum(self.n_c[:irrep]))
        return off, off + int(self.n_c[irrep])

    def dim(self) -> int:
        d = self.n_l2
        for s in self.syms:
            a = s.irrep ^ self.total_irrep
            d += s.ci.shape[1] * int(self.n_c[a])
        return d

    def n_cont_rows(self) -> int:
        return self.dim() - self.n_l2


# ----------------------------------------------------------------------------
# bitstring helpers (pure data conversion)
# ----------------------------------------------------------------------------

def occ_to_det(occ, n_words: int) -> np.ndarray:
    w = np.zeros(n_words, dtype=np.uint64)
    for k in occ:
        w[k >> 6] |= np.uint64(1) << np.uint64(k & 63)
    return w


def det_to_occ(det) -> list:
    occ = []
    for wi, word in enumerate(np.asarray(det, dtype=np.uint64)):
        word = int(word)
        b = 0
        while word:
            if word & 1:
                occ.append(64 * wi + b)
            word >>= 1
            b += 1
    return occ


# ----------------------------------------------------------------------------
# integrals
# ----------------------------------------------------------------------------

def _irreps(n_o, n_irrep, n_c):
    tgt = (np.arange(n_o) % n_irrep).astype(np.uint8)
    cont = np.repeat(np.arange(n_irrep, dtype=np.uint8), n_c)
    return tgt, cont


def _gen_integrals(rng, n_o, tgt_irrep, cont_irrep, sd2=0.1, skip_cc=False):
    n_cont = len(cont_irrep)
    n_orb = n_o + n_cont
    oi = np.concatenate([tgt_irrep, cont_irrep]).astype(np.int64)
    g = np.arange(n_orb, dtype=np.float64)          # global orbital index

    # one-electron: symmetric, decaying, symmetry-blocked
    x = rng.standard_normal((n_orb, n_orb))
    x = np.tril(x) + np.tril(x, -1).T
    h = x * np.exp(-np.abs(g[:, None] - g[None, :]) / 4.0)
    h[oi[:, None] != oi[None, :]] = 0.0

    t = np.arange(n_o)
    ti = oi[:n_o]
    # tttt: canonical over pq >= rs with p >= q, r >= s
    P, Q, R, S = np.meshgrid(t, t, t, t, indexing="ij")
    pq = np.maximum(P, Q) * (np.maximum(P, Q) + 1) // 2 + np.minimum(P, Q)
    rs = np.maximum(R, S) * (np.maximum(R, S) + 1) // 2 + np.minimum(R, S)
    key = np.maximum(pq, rs) * (np.maximum(pq, rs) + 1) // 2 + np.minimum(pq, rs)
    npair = n_o * (n_o + 1) // 2
    draws = rng.standard_normal(npair * (npair + 1) // 2) * sd2
    tttt = draws[key] * np.exp(-(np.abs(P - Q) + np.abs(R - S)) / 4.0)
    tttt[(ti[P] ^ ti[Q] ^ ti[R] ^ ti[S]) != 0] = 0.0
    del P, Q, R, S, pq, rs, key

    gc = g[n_o:]
    ci = oi[n_o:]
    # tttc (pq|rj): symmetric in p, q only
    tttc = np.empty((n_o, n_o, n_o, n_cont))
    for p in range(n_o):
        for q in range(p + 1):
            blk = rng.standard_normal((n_o, n_cont)) * sd2
            blk *= np.exp(-(abs(p - q) + np.abs(t[:, None] - gc[None, :])) / 4.0)
            blk[(ti[p] ^ ti[q] ^ ti[:, None] ^ ci[None, :]) != 0] = 0.0
            tttc[p, q] = blk
            tttc[q, p] = blk
    if skip_cc:
        return h, tttt, tttc, None, None
    # ttcc (pq|jj'): symmetric in p, q and in j, j'
    ttcc = np.empty((n_o, n_o, n_cont, n_cont))
    dcc = np.exp(-np.abs(gc[:, None] - gc[None, :]) / 4.0)
    mcc = (ci[:, None] ^ ci[None, :])
    for p in range(n_o):
        for q in range(p + 1):
            x = rng.standard_normal((n_cont, n_cont)) * sd2
            x = np.tril(x) + np.tril(x, -1).T
            x *= dcc * math.exp(-abs(p - q) / 4.0)
            x[(mcc ^ ti[p] ^ ti[q]) != 0] = 0.0
            ttcc[p, q] = x
            ttcc[q, p] = x
    # tctc (pj|qj'): symmetric under (p,j) <-> (q,j')
    tctc = np.empty((n_o, n_cont, n_o, n_cont))
    for p in range(n_o):
        dp = np.exp(-np.abs(p - gc) / 4.0)
        for q in range(p + 1):
            dq = np.exp(-np.abs(q - gc) / 4.0)
            x = rng.standard_normal((n_cont, n_cont)) * sd2
            if p == q:
                x = np.tril(x) + np.tril(x, -1).T
            x *= dp[:, None] * dq[None, :]
            x[(mcc ^ ti[p] ^ ti[q]) != 0] = 0.0
            tctc[p, :, q, :] = x
            tctc[q, :, p, :] = x.T
    return h, tttt, tttc, ttcc, tctc


def packed_layout(tgt_irrep, n_c):
    """Offsets of the symmetry-packed two-continuum integrals. For the target
    pair (P, Q), with x = irrep(P) ^ irrep(Q), one record holds a block per
    continuum irrep ca: the n_c[ca] x n_c[ca ^ x] values of (P Q | j j') (for
    ttcc) or (P j | Q j') (for tctc), j of irrep ca and j' of irrep ca ^ x,
    row-major; every other value is zero by symmetry. Returns rec (n_o^2 + 1
    record offsets, pair P * n_o + Q) and blk (blk[x][ca], offsets inside a
    record)."""
    n_c = np.asarray(n_c, dtype=np.int64)
    ni = len(n_c)
    blk = np.zeros((ni, ni), np.int64)
    size = np.zeros(ni, np.int64)
    for x in range(ni):
        off = 0
        for ca in range(ni):
            blk[x, ca] = off
            off += n_c[ca] * n_c[ca ^ x]
        size[x] = off
    ti = np.asarray(tgt_irrep, dtype=np.int64)
    rec = np.concatenate([[0], np.cumsum(size[(ti[:, None] ^ ti[None, :]).ravel()])]).astype(np.int64)
    return rec, blk


def pack_integrals(inst):
    """The instance with ttcc and tctc in the symmetry-packed layout (pure
    data movement from the dense arrays)."""
    if inst.packed:
        return inst
    rec, blk = packed_layout(inst.tgt_irrep, inst.n_c)
    n_o, ni = inst.n_o, inst.n_irrep
    cs = np.concatenate([[0], np.cumsum(inst.n_c)])
    ttcc = np.zeros(rec[-1])
    tctc = np.zeros(rec[-1])
    for P in range(n_o):
        for Q in range(n_o):
            x = int(inst.tgt_irrep[P]) ^ int(inst.tgt_irrep[Q])
            r0 = rec[P * n_o + Q]
            for ca in range(ni):
                cb = ca ^ x
                o = r0 + blk[x, ca]
                nab = inst.n_c[ca] * inst.n_c[cb]
                ttcc[o:o + nab] = inst.ttcc[P, Q, cs[ca]:cs[ca + 1], cs[cb]:cs[cb + 1]].ravel()
                tctc[o:o + nab] = inst.tctc[P, cs[ca]:cs[ca + 1], Q, cs[cb]:cs[cb + 1]].ravel()
    out = Instance(**{f: getattr(inst, f) for f in inst.__dataclass_fields__})
    out.ttcc, out.tctc, out.packed = ttcc, tctc, True
    return out


def unpack_integrals(inst):
    """The instance with dense ttcc and tctc rebuilt from the packed layout
    (pure data movement; zeros where symmetry forbids a value)."""
    if not inst.packed:
        return inst
    rec, blk = packed_layout(inst.tgt_irrep, inst.n_c)
    n_o, ni, nc = inst.n_o, inst.n_irrep, inst.n_cont
    cs = np.concatenate([[0], np.cumsum(inst.n_c)])
    ttcc = np.zeros((n_o, n_o, nc, nc))
    tctc = np.zeros((n_o, nc, n_o, nc))
    for P in range(n_o):
        for Q in range(n_o):
            x = int(inst.tgt_irrep[P]) ^ int(inst.tgt_irrep[Q])
            r0 = rec[P * n_o + Q]
            for ca in range(ni):
                cb = ca ^ x
                o = r0 + blk[x, ca]
                sh = (inst.n_c[ca], inst.n_c[cb])
                n = sh[0] * sh[1]
                ttcc[P, Q, cs[ca]:cs[ca + 1], cs[cb]:cs[cb + 1]] = inst.ttcc[o:o + n].reshape(sh)
                tctc[P, cs[ca]:cs[ca + 1], Q, cs[cb]:cs[cb + 1]] = inst.tctc[o:o + n].reshape(sh)
    out = Instance(**{f: getattr(inst, f) for f in inst.__dataclass_fields__})
    out.ttcc, out.tctc, out.packed = ttcc, tctc, False
    return out


def _gen_packed_cc(rng, n_o, tgt_irrep, n_c, sd2=0.1):
    """ttcc and tctc drawn directly in the packed layout, with the law of the
    dense generator (N(0, sd2) times the decay in global orbital indices,
    (pq|jj') symmetric in p, q and in j, j', (pj|qj') symmetric under
    (p, j) <-> (q, j'), symmetry zeros not stored)."""
    n_c = np.asarray(n_c, dtype=np.int64)
    ni = len(n_c)
    rec, blk = packed_layout(tgt_irrep, n_c)
    ti = np.asarray(tgt_irrep, dtype=np.int64)
    cs = np.concatenate([[0], np.cumsum(n_c)])
    gc = n_o + np.arange(int(cs[-1]), dtype=np.float64)
    ttcc = np.zeros(rec[-1])
    tctc = np.zeros(rec[-1])

    def view(arr, P, Q, ca):
        x = int(ti[P] ^ ti[Q])
        o = rec[P * n_o + Q] + blk[x, ca]
        return arr[o:o + n_c[ca] * n_c[ca ^ x]].reshape(n_c[ca], n_c[ca ^ x])

    for p in range(n_o):
        dp = np.exp(-np.abs(p - gc) / 4.0)
        for q in range(p + 1):
            x = int(ti[p] ^ ti[q])
            dq = np.exp(-np.abs(q - gc) / 4.0)
            for ca in range(ni):
                cb = ca ^ x
                ja, jb = slice(cs[ca], cs[ca + 1]), slice(cs[cb], cs[cb + 1])
                # (pq|jj'): blocks (ca, cb) and (cb, ca) are transposes; (ca, ca) symmetric
                if ca <= cb:
                    X = rng.standard_normal((n_c[ca], n_c[cb])) * sd2
                    if ca == cb:
                        X = np.tril(X) + np.tril(X, -1).T
                    X *= np.exp(-np.abs(gc[ja][:, None] - gc[jb][None, :]) / 4.0) * math.exp(-abs(p - q) / 4.0)
                    view(ttcc, p, q, ca)[:] = X
                    view(ttcc, p, q, cb)[:] = X.T
                    view(ttcc, q, p, ca)[:] = X
                    view(ttcc, q, p, cb)[:] = X.T
                # (pj|qj'): record (q, p) holds the transposes; p == q symmetric blocks
                Y = rng.standard_normal((n_c[ca], n_c[cb])) * sd2
                if p == q:
                    if ca > cb:
                        continue          # filled as the transpose of block cb
                    if ca == cb:
                        Y = np.tril(Y) + np.tril(Y, -1).T
                Y *= dp[ja][:, None] * dq[jb][None, :]
                view(tctc, p, q, ca)[:] = Y
                view(tctc, q, p, cb)[:] = Y.T
    return ttcc, tctc


# ----------------------------------------------------------------------------
# determinant spaces
# ----------------------------------------------------------------------------

def _strings(n_o, n_e, max_level):
    """Occupation strings of one spin with at most max_level excitations
    from the aufbau string, as (level, tuple(occupied orbitals))."""
    ref = list(range(n_e))
    virt = list(range(n_e, n_o))
    out = []
    for lev in range(0, max_level + 1):
        if lev > min(n_e, n_o - n_e):
            break
        for holes in itertools.combinations(ref, lev):
            keep = [o for o in ref if o not in holes]
            for parts in itertools.combinations(virt, lev):
                out.append((lev, tuple(sorted(keep + list(parts)))))
    return out


def _det_space(rng, n_o, n_a, n_b, tgt_irrep, irrep, count):
    """CISD-like determinant space: alpha/beta strings by excitation level
    from the aufbau reference, combined, filtered by irrep, ordered by
    (total level, seeded key); the first `count` are taken."""
    n_words = (2 * n_o + 63) // 64
    tir = np.asarray(tgt_irrep, dtype=np.int64)
    for max_level in range(2, 2 * n_o + 1):
        sa = _strings(n_o, n_a, max_level)
        sb = _strings(n_o, n_b, max_level)
        la = np.array([l for l, _ in sa]); lb = np.array([l for l, _ in sb])
        ia = np.array([np.bitwise_xor.reduce(tir[list(o)]) if o else 0 for _, o in sa])
        ib = np.array([np.bitwise_xor.reduce(tir[list(o)]) if o else 0 for _, o in sb])
        cand = []
        for x_l in range(max_level + 1):
            xs = np.nonzero(la == x_l)[0]
            for y_l in range(max_level + 1 - x_l):
                ys = np.nonzero(lb == y_l)[0]
                if len(xs) == 0 or len(ys) == 0:
                    continue
                X, Y = np.meshgrid(xs, ys, indexing="ij")
                X = X.ravel(); Y = Y.ravel()
                ok = (ia[X] ^ ib[Y]) == irrep
                cand.append(np.stack([np.full(ok.sum(), x_l + y_l), X[ok], Y[ok]], 1))
        cand = np.concatenate(cand) if cand else np.zeros((0, 3), dtype=np.int64)
        if len(cand) >= count:
            break
    else:
        raise ValueError("determinant space too small for the requested count")
    keys = rng.random(len(cand))
    order = np.lexsort((keys, cand[:, 0]))[:count]
    dets = np.zeros((count, n_words), dtype=np.uint64)
    for r, c in enumerate(order):
        _, x, y = cand[c]
        occ = [2 * o for o in sa[x][1]] + [2 * o + 1 for o in sb[y][1]]
        dets[r] = occ_to_det(sorted(occ), n_words)
    return dets


def _ci(rng, m, s):
    a = rng.standard_normal((m, s))
    q, r = np.linalg.qr(a)
    sg = np.sign(np.diag(r))
    sg[sg == 0] = 1.0
    return np.ascontiguousarray(q * sg[None, :])


# ----------------------------------------------------------------------------
# instances
# ----------------------------------------------------------------------------

def make_instance(n_o, n_elec, n_irrep, n_c, sym_irreps, n_det, n_states,
                  n_l2, seed, e_core=0.0, name="", total_irrep=0, packed=False):
    """n_c: continuum orbitals per irrep (int or list); sym_irreps: irreps of
    the target symmetries; n_det/n_states: per symmetry (int or list).
    packed: (tt|cc) and (tc|tc) drawn directly in the symmetry-packed layout
    (never dense; a different draw order from the dense generator)."""
    if n_elec % 2:
        raise ValueError("n_elec must be even (n_alpha = n_beta = N/2)")
    rng = np.random.default_rng(seed)
    if np.isscalar(n_c):
        n_c = [int(n_c)] * n_irrep
    n_c = np.asarray(n_c, dtype=np.int32)
    nsym = len(sym_irreps)
    n_det = [n_det] * nsym if np.isscalar(n_det) else list(n_det)
    n_states = [n_states] * nsym if np.isscalar(n_states) else list(n_states)
    tgt_irrep, cont_irrep = _irreps(n_o, n_irrep, n_c)
    if packed:
        h, tttt, tttc, _, _ = _gen_integrals(rng, n_o, tgt_irrep, cont_irrep, skip_cc=True)
        ttcc, tctc = _gen_packed_cc(rng, n_o, tgt_irrep, n_c)
    else:
        h, tttt, tttc, ttcc, tctc = _gen_integrals(rng, n_o, tgt_irrep, cont_irrep)
    na = nb = n_elec // 2
    syms = []
    for irr, m, s in zip(sym_irreps, n_det, n_states):
        dets = _det_space(rng, n_o, na, nb, tgt_irrep, irr, m)
        syms.append(TargetSym(int(irr), dets, _ci(rng, m, s)))
    l2 = _det_space(rng, n_o, na + 1, nb, tgt_irrep, total_irrep, n_l2) if n_l2 else \
        np.zeros((0, (2 * n_o + 63) // 64), dtype=np.uint64)
    return Instance(n_o=n_o, n_elec=n_elec, n_irrep=n_irrep, tgt_irrep=tgt_irrep,
                    n_c=n_c, total_irrep=total_irrep, h=h, tttt=tttt, tttc=tttc,
                    ttcc=ttcc, tctc=tctc, e_core=float(e_core), syms=syms,
                    l2_dets=l2, name=name, seed=seed, packed=packed)


def tiny(seed=101):
    """10 target orbitals, N=6, 40 dets in 1 symmetry, 3 states, 20 continuum
    orbitals, 50 L2 configurations: D = 110."""
    return make_instance(10, 6, 1, 20, [0], 40, 3, 50, seed, name="tiny")


def small(seed=111):
    """Multi-tile parity case: 2 symmetries (irreps 0, 1) x 120 dets x 4 states,
    40 continuum orbitals per irrep, 300 L2 functions: D = 620."""
    return make_instance(12, 6, 2, [40, 37], [0, 1], [120, 97], [4, 3], 301, seed,
                         name="small")


def wide(seed=121):
    """Two-word determinants (36 target orbitals = 72 spin-orbitals): the
    64-bit word boundary is crossed by occupied orbitals and excitations."""
    return make_instance(36, 8, 1, 30, [0], 150, 5, 200, seed, name="wide")


def medium(seed=202):
    """30 target orbitals, N=10, 4 symmetries x 500 dets x 5 states,
    150 continuum orbitals per irrep, 5000 L2: D = 8000."""
    return make_instance(30, 10, 4, 150, [0, 1, 2, 3], 500, 5, 5000, seed,
                         name="medium")


def precision(seed=303):
    """40 target orbitals, N=12, 8000 dets, 1 symmetry, 40 states,
    300 continuum orbitals, 28000 L2: D = 40000."""
    return make_instance(40, 12, 1, 300, [0], 8000, 40, 28000, seed,
                         name="precision")


def learned_test(seed=999):
    """40 target orbitals, N=12, 8000 dets, 50 states, 400 continuum,
    40000 L2: D = 60000."""
    return make_instance(40, 12, 1, 400, [0], 8000, 50, 40000, seed,
                         name="learned_test")


def l2heavy(seed=808):
    """Shaped like the paper's phosphoric-acid case (a small contracted part,
    a large L2 part, N = 122815 in total): 40 target orbitals, N=12, 2000
    target determinants in 1 symmetry, 4 states x 178 continuum orbitals = 712
    contracted rows, 122103 L2 functions; about 0.9 GB of integrals."""
    return make_instance(40, 12, 1, 178, [0], 2000, 4, 122103, seed, name="l2heavy")


def paired(n_o=30, n_elec=10, n_det=500, n_states=5, n_c=150, n_l2=5000, seed=222, name="medium_pairs"):
    """Target states in pairs of symmetries that share one determinant space
    and so one continuum irrep (the emulation of singlet and triplet target
    states of one spatial symmetry, Fig. 2; classes 5 and 6 appear between the
    two members of a pair): two irreps, four target symmetries with irreps
    0, 0, 1, 1 where the second member of each pair holds the same
    determinants as the first. The CI vectors are random orthonormal
    placeholders: the caller replaces them by eigenvectors of the target
    Hamiltonian (the lowest n_states for the first member, the next n_states
    for the second). Defaults: the medium shape, D = 4 x 5 x 150 + 5000 =
    8000."""
    inst = make_instance(n_o, n_elec, 2, n_c, [0, 0, 1, 1], n_det, n_states, n_l2, seed, name=name)
    inst.syms[1].dets = inst.syms[0].dets.copy()
    inst.syms[3].dets = inst.syms[2].dets.copy()
    return inst


def l2huge(seed=818):
    """The phosphoric-acid shape with twice its L2 functions: 40 target
    orbitals, N=12, 2000 target determinants in 1 symmetry, 4 states x 178
    continuum orbitals = 712 contracted rows, 250000 L2 functions
    (D = 250712: a dense matrix would need 503 GB)."""
    return make_instance(40, 12, 1, 178, [0], 2000, 4, 250000, seed, name="l2huge")


def l2_spin_adapted(inst):
    """The instance with its L2 functions rewritten as doublet CSFs (Eq. 1's
    second sum over configuration state functions): the L2 determinants are
    grouped by spatial occupation; a group with one open shell is one CSF of
    one determinant; a group with three open shells a < b < c (two alpha
    electrons, one beta) gives the two doublets of the genealogical coupling,
    (a b) triplet: (2|aA bA cB> - |aA bB cA> - |aB bA cA>)/sqrt(6), and
    (a b) singlet: (|aA bB cA> - |aB bA cA>)/sqrt(2) (A = alpha, B = beta; the
    determinants are ascending products, and the open-shell spin-orbitals keep
    their relative order in all three, so the coefficients need no further
    sign); groups with five or more open shells are left out. Pure data: the
    determinant lists and coupling coefficients of the input."""
    W = inst.n_words
    groups = {}
    order = []
    for idx, d in enumerate(inst.l2_dets):
        occ = det_to_occ(d)
        spatial = {}
        for k in occ:
            spatial[k >> 1] = spatial.get(k >> 1, 0) + 1
        key = tuple(sorted(spatial.items()))
        if key not in groups:
            groups[key] = []
            order.append(key)
        groups[key].append(idx)
    starts, dets, coef = [0], [], []
    r6, r2 = 1.0 / math.sqrt(6.0), 1.0 / math.sqrt(2.0)
    for key in order:
        members = groups[key]
        opens = [o for o, n in key if n == 1]
        if len(opens) == 1:
            dets.append(inst.l2_dets[members[0]])
            coef.append(1.0)
            starts.append(len(dets))
        elif len(opens) == 3:
            a, b, c = opens
            closed = [2 * o + sp for o, n in key if n == 2 for sp in (0, 1)]

            def det(sa, sb, sc):
                return occ_to_det(sorted(closed + [2 * a + sa, 2 * b + sb, 2 * c + sc]), W)
            have = {tuple(inst.l2_dets[m]) for m in members}
            aab, aba, baa = det(0, 0, 1), det(0, 1, 0), det(1, 0, 0)
            if not all(tuple(x) in have for x in (aab, aba, baa)):
                continue          # an incomplete spin family: left out
            for terms in ((aab, 2 * r6), (aba, -r6), (baa, -r6)), ((aba, r2), (baa, -r2)):
                for dd, cf in terms:
                    dets.append(dd)
                    coef.append(cf)
                starts.append(len(dets))
    out = Instance(**{f: getattr(inst, f) for f in inst.__dataclass_fields__})
    out.l2_dets = np.array(dets, dtype=np.uint64).reshape(-1, W)
    out.l2_csf_start = np.array(starts, dtype=np.int32)
    out.l2_coef = np.array(coef, dtype=np.float64)
    return out


def _spin_flips(occ, to_alpha):
    """Occupation lists reached by turning one electron of a singly occupied
    orbital from beta to alpha (to_alpha) or from alpha to beta; the two
    spin-orbitals 2k, 2k + 1 are adjacent, so every such ladder step has
    sign +1 on ascending determinants."""
    s = set(occ)
    out = []
    for k in sorted({o >> 1 for o in occ}):
        src, dst = (2 * k + 1, 2 * k) if to_alpha else (2 * k, 2 * k + 1)
        if src in s and dst not in s:
            out.append(sorted((s - {src}) | {dst}))
    return out


def triplet_doublet(inst, n_states=None, seed=0):
    """The instance with each target symmetry's states replaced by triplet
    target states coupled with the continuum electron to doublets (total
    S = M_S = 1/2), the coupling of triplet targets the paper's CSF-driven
    build allows (Eq. 2): channel function
        sqrt(2/3) |T, M=1> u_beta - sqrt(1/3) |T, M=0> u_alpha.
    |T, 1> lies in the M_S = 1 determinants reached by turning one beta
    electron of a singly occupied orbital of the symmetry's determinants
    alpha, projected on S = 1 (the null space of S+ there), with seeded
    orthonormal coefficients; |T, 0> = S- |T, 1> / sqrt(2). The continuum spin
    is given per determinant: 1 (beta) for the M_S = 1 ones, 0 for the
    M_S = 0 ones. Pure data: ladder operators on occupation lists."""
    import scipy.linalg
    rng = np.random.default_rng(seed)
    W = inst.n_words
    syms = []
    for s in inst.syms:
        m1, idx1 = [], {}
        for d in s.dets:
            for o in _spin_flips(det_to_occ(d), True):
                if tuple(o) not in idx1:
                    idx1[tuple(o)] = len(m1)
                    m1.append(o)
        if not m1:
            raise ValueError("no M_S = 1 determinant reachable")
        m2, idx2, sp_rows = [], {}, []
        for c, o in enumerate(m1):
            for o2 in _spin_flips(o, True):
                if tuple(o2) not in idx2:
                    idx2[tuple(o2)] = len(m2)
                    m2.append(o2)
                sp_rows.append((idx2[tuple(o2)], c))
        Splus = np.zeros((len(m2), len(m1)))
        for r, c in sp_rows:
            Splus[r, c] += 1.0
        Z = scipy.linalg.null_space(Splus) if len(m2) else np.eye(len(m1))
        S = min(n_states or s.ci.shape[1], Z.shape[1])
        if S < 1:
            raise ValueError("no triplet in the M_S = 1 space")
        Q, _ = np.linalg.qr(rng.standard_normal((Z.shape[1], S)))
        c1 = Z @ Q
        m0, idx0, sm_rows = [], {}, []
        for c, o in enumerate(m1):
            for o0 in _spin_flips(o, False):
                if tuple(o0) not in idx0:
                    idx0[tuple(o0)] = len(m0)
                    m0.append(o0)
                sm_rows.append((idx0[tuple(o0)], c))
        Sminus = np.zeros((len(m0), len(m1)))
        for r, c in sm_rows:
            Sminus[r, c] += 1.0
        c0 = Sminus @ c1 / math.sqrt(2.0)
        dets = np.array([occ_to_det(o, W) for o in m1 + m0], dtype=np.uint64).reshape(-1, W)
        ci = np.vstack([math.sqrt(2.0 / 3.0) * c1, -math.sqrt(1.0 / 3.0) * c0])
        spin = np.concatenate([np.ones(len(m1), np.int8), np.zeros(len(m0), np.int8)])
        syms.append(TargetSym(s.irrep, dets, np.ascontiguousarray(ci), spin))
    out = Instance(**{f: getattr(inst, f) for f in inst.__dataclass_fields__})
    out.syms = syms
    return out


def _active_dets(rng, n_o, n_a, n_b, tgt_irrep, irrep, active, count):
    """Determinants with n_a alpha and n_b beta electrons, all in the listed
    active orbitals, of one irrep, in seeded order; the first `count`."""
    n_words = (2 * n_o + 63) // 64
    tir = np.asarray(tgt_irrep, dtype=np.int64)
    cand = []
    for oa in itertools.combinations(active, n_a):
        for ob in itertools.combinations(active, n_b):
            r = 0
            for o in oa + ob:
                r ^= int(tir[o])
            if r == irrep:
                cand.append(sorted([2 * o for o in oa] + [2 * o + 1 for o in ob]))
    if len(cand) < count:
        raise ValueError("active space too small for the requested count")
    order = np.argsort(rng.random(len(cand)), kind="stable")[:count]
    return np.stack([occ_to_det(cand[i], n_words) for i in order])


def boundary(words, seed=131):
    """Determinants straddling every 64-bit word boundary of a 3- or 4-word
    bitstring (Sec. 2.1 reports wrong masks at multiples of 64): N = 4
    electrons in eight active orbitals placed on both sides of spin-orbitals
    64 and 128 (3 words: 66 target orbitals) or 64, 128 and 192 (4 words:
    100 target orbitals), two irreps, two target symmetries of 300 and 280
    determinants with 4 and 3 states, 12 continuum orbitals per irrep and
    400 L2 functions: D = 484."""
    if words == 3:
        n_o, active = 66, [0, 1, 31, 32, 62, 63, 64, 65]
    elif words == 4:
        n_o, active = 100, [0, 31, 32, 63, 64, 95, 96, 99]
    else:
        raise ValueError("words must be 3 or 4")
    rng = np.random.default_rng(seed + words)
    n_irrep, n_elec, n_c = 2, 4, 12
    tgt_irrep, cont_irrep = _irreps(n_o, n_irrep, [n_c] * n_irrep)
    h, tttt, tttc, ttcc, tctc = _gen_integrals(rng, n_o, tgt_irrep, cont_irrep)
    syms = []
    for irr, m, st in ((0, 300, 4), (1, 280, 3)):
        dets = _active_dets(rng, n_o, 2, 2, tgt_irrep, irr, active, m)
        syms.append(TargetSym(irr, dets, _ci(rng, m, st)))
    l2 = _active_dets(rng, n_o, 3, 2, tgt_irrep, 0, active, 400)
    return Instance(n_o=n_o, n_elec=n_elec, n_irrep=n_irrep, tgt_irrep=tgt_irrep,
                    n_c=np.full(n_irrep, n_c, np.int32), total_irrep=0, h=h, tttt=tttt,
                    tttc=tttc, ttcc=ttcc, tctc=tctc, e_core=0.0, syms=syms, l2_dets=l2,
                    name=f"boundary{words}", seed=seed + words)


def mid(seed=313):
    """The precision shape at half size, for checks that need the whole
    matrix on the host: 40 target orbitals, N = 12, 4000 determinants in one
    symmetry, 20 states, 300 continuum orbitals, 14000 L2 functions:
    D = 20000 (two-word determinants)."""
    return make_instance(40, 12, 1, 300, [0], 4000, 20, 14000, seed, name="mid")


def _batch_like(rng, seed, d_lo, d_hi, name, max_int_bytes=256 << 20, packed=False):
    """Draw (D, n_o, symmetries, states, continuum, N) from the batch ranges;
    draws whose (tt|cc) + (tc|tc) storage would exceed max_int_bytes (dense,
    or in the symmetry-packed layout with packed=True), whose L2 count would
    be negative, or whose L2 space is too small are redrawn."""
    while True:
        d = int(rng.integers(d_lo, d_hi + 1))
        n_o = int(rng.integers(12, 41))
        n_sym = int(rng.choice([1, 2, 4]))
        n_irrep = n_sym
        s = int(rng.integers(5, 31))
        nc = int(rng.integers(50, 201))
        n_elec = int(rng.choice([4, 6, 8, 10, 12]))
        n_l2 = d - n_sym * s * nc
        n_cont = n_sym * nc
        # packed: each target pair keeps n_irrep blocks of nc x nc values
        cc_bytes = 16 * n_o * n_o * (n_irrep * nc * nc if packed else n_cont * n_cont)
        if n_l2 < 0 or cc_bytes > max_int_bytes:
            continue
        na = n_elec // 2
        if n_l2 > math.comb(n_o, na + 1) * math.comb(n_o, na) // (4 * n_irrep):
            continue
        break
    m = max(s, int(rng.integers(2 * s, 8 * s + 1)))
    return make_instance(n_o, n_elec, n_irrep, nc, list(range(n_sym)), m, s, n_l2,
                         seed, name=name, packed=packed)


def batch_instance(i):
    """One of the 64 batched instances: D ~ U[500, 6000], 12-40 target
    orbitals, 1, 2 or 4 target symmetries (as many irreps), 5-30 states,
    50-200 continuum orbitals per irrep; (tt|cc) and (tc|tc) in the
    symmetry-packed layout, at most 1 GiB of them."""
    rng = np.random.default_rng(400 + i)
    return _batch_like(rng, 400 + i, 500, 6000, f"batch{i}", max_int_bytes=1 << 30, packed=True)


def learned_train(i):
    rng = np.random.default_rng(500 + i)
    return _batch_like(rng, 500 + i, 2000, 20000, f"train{i}")


def micro(seed, n_o=3, n_elec=2, n_c=2, n_irrep=1, n_det=None, n_states=None,
          n_l2=None):
    """Instances small enough for a Fock-space brute force: all N-electron
    determinants of the requested irreps may be used."""
    rng = np.random.default_rng(seed)
    n_irrep_syms = list(range(n_irrep))
    tgt_irrep, _ = _irreps(n_o, n_irrep, [n_c] * n_irrep)
    na = n_elec // 2
    # count available dets per irrep
    dets_avail = []
    for irr in n_irrep_syms:
        cnt = 0
        for oa in itertools.combinations(range(n_o), na):
            for ob in itertools.combinations(range(n_o), na):
                r = 0
                for o in oa + ob:
                    r ^= int(tgt_irrep[o])
                cnt += (r == irr)
        dets_avail.append(cnt)
    nd = [min(dets_avail[i], n_det if n_det else dets_avail[i]) for i in n_irrep_syms]
    ns = [max(1, min(nd[i], n_states if n_states else max(1, nd[i] // 2)))
          for i in n_irrep_syms]
    cnt_l2 = 0
    for oa in itertools.combinations(range(n_o), na + 1):
        for ob in itertools.combinations(range(n_o), na):
            r = 0
            for o in oa + ob:
                r ^= int(tgt_irrep[o])
            cnt_l2 += (r == 0)
    nl2 = cnt_l2 if n_l2 is None else min(cnt_l2, n_l2)
    return make_instance(n_o, n_elec, n_irrep, n_c, n_irrep_syms, nd, ns, nl2,
                         int(rng.integers(1 << 30)), name=f"micro{seed}")


CONFIGS = {
    "tiny": tiny, "small": small, "wide": wide, "medium": medium,
    "precision": precision, "learned_test": learned_test, "l2heavy": l2heavy,
    "boundary3": lambda: boundary(3), "boundary4": lambda: boundary(4), "mid": mid, "l2huge": l2huge,
    "medium_pairs": paired,
}
