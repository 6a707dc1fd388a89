"""Host checks of two readings the full-spectrum solver builds on (Sec. 3.2;
the device code is tested against LAPACK in test_gpu_eig_all.py):

* the compact WY factor of a product of Householder reflectors H_1 ... H_k =
  I - V T V^T, formed by blocks: T = [[T1, -T1 (V1^T V2) T2], [0, T2]] equals
  the column recurrence T[0:i, i] = -tau_i T[0:i, 0:i] V[:, 0:i]^T v_i and
  reproduces the product of the reflectors;
* multisection on Sturm counts (8 interior points per round, the interval
  kept between the last point with count <= k and the first with count > k)
  ends on the same pair of adjacent doubles as bisection, and each midpoint
  is within rounding of LAPACK's eigenvalue.
"""
import numpy as np
import pytest


def _reflectors(rng, m, nb):
    V = np.tril(rng.standard_normal((m, nb)), -1)
    V[np.arange(nb), np.arange(nb)] = 1.0
    tau = 2.0 / (V * V).sum(axis=0)
    return V, tau


def _t_columns(G, tau):
    nb = len(tau)
    T = np.zeros((nb, nb))
    for i in range(nb):
        T[:i, i] = -tau[i] * (T[:i, :i] @ G[:i, i])
        T[i, i] = tau[i]
    return T


def _t_blocks(G, tau, leaf=16):
    nb = len(tau)
    if nb <= leaf:
        return _t_columns(G, tau)
    h = 1 << (max(nb - 1, 1).bit_length() - 1)   # the largest power of two below nb
    T1 = _t_blocks(G[:h, :h], tau[:h], leaf)
    T2 = _t_blocks(G[h:, h:], tau[h:], leaf)
    T = np.zeros((nb, nb))
    T[:h, :h] = T1
    T[h:, h:] = T2
    T[:h, h:] = -T1 @ (G[:h, h:] @ T2)
    return T


@pytest.mark.parametrize("nb", [1, 5, 16, 17, 33, 64, 100, 128])
def test_compact_wy_by_blocks(nb):
    rng = np.random.default_rng(nb)
    m = 160
    V, tau = _reflectors(rng, m, nb)
    G = V.T @ V
    Tb = _t_blocks(G, tau)
    assert np.abs(Tb - _t_columns(G, tau)).max() <= 1e-13 * np.abs(Tb).max()
    H = np.eye(m)
    for k in range(nb):
        H = H @ (np.eye(m) - tau[k] * np.outer(V[:, k], V[:, k]))
    assert np.abs(np.eye(m) - V @ Tb @ V.T - H).max() <= 1e-13


def _sturm(d, e2, x, pivmin):
    c = 0
    q = d[0] - x
    if abs(q) < pivmin:
        q = -pivmin
    c += q < 0
    for i in range(1, len(d)):
        q = d[i] - x - e2[i - 1] / q
        if abs(q) < pivmin:
            q = -pivmin
        c += q < 0
    return c


def _bisect(d, e2, k, lo, hi, pivmin):
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if _sturm(d, e2, mid, pivmin) > k:
            hi = mid
        else:
            lo = mid
    return lo, hi


def _multisect(d, e2, k, lo, hi, pivmin, g=8):
    f = [(j + 1) / (g + 1) for j in range(g)]
    for _ in range(200):
        xs = [lo + (hi - lo) * fj for fj in f]
        inside = [lo < x < hi for x in xs]
        if not any(inside):
            break
        cs = [_sturm(d, e2, x, pivmin) if ins else 0 for x, ins in zip(xs, inside)]
        h = min([x for x, ins, c in zip(xs, inside, cs) if ins and c > k] + [hi])
        lo = max([x for x, ins, c in zip(xs, inside, cs) if ins and c <= k and x < h] + [lo])
        hi = h
    return lo, hi


def test_multisection_ends_where_bisection_does():
    rng = np.random.default_rng(3)
    n = 24
    d = rng.standard_normal(n)
    e = rng.standard_normal(n - 1)
    d[6:10] = 0.5
    e[7] = 1e-9                            # a nearly split pair
    e2 = e * e
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    w = np.linalg.eigvalsh(T)
    nrm = np.abs(T).sum(axis=1).max()
    for k in range(n):
        a = _bisect(d, e2, k, -nrm, nrm, 1e-300)
        b = _multisect(d, e2, k, -nrm, nrm, 1e-300)
        assert a == b
        assert abs(0.5 * (b[0] + b[1]) - w[k]) <= 1e-13 * nrm
