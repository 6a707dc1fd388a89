"""The Rayleigh-Ritz eigensolver of the Davidson iteration (cch_subspace_eig)
on matrices chosen to break it: every size class up to 96 (one to several
16-wide MFMA tiles and ragged tails), Davidson-shaped bordered diagonals with
couplings down to 1e-12, tight and exactly repeated eigenvalues, split
tridiagonals, scalar and rank-one matrices, extreme scales. Eigenvalues
against LAPACK (NumPy eigh) within 1e-13 ||G||, eigenvectors checked by
orthogonality and residual. Exactly repeated eigenvalues may take the Jacobi
fallback; the other cases must not."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _sym(M):
    return 0.5 * (M + M.T)


def _cases():
    rng = np.random.default_rng(11)
    out = []
    for n in [1, 2, 3, 4, 7, 16, 17, 31, 40, 63, 64, 65, 80, 95, 96]:
        M = rng.standard_normal((n, n))
        out.append((f"random{n}", M + M.T, False))
    for m0, nb in [(0, 20), (10, 10), (20, 10), (50, 10), (70, 10), (80, 16), (86, 10)]:
        n = m0 + nb
        G = np.zeros((n, n))
        G[:m0, :m0] = np.diag(np.sort(rng.uniform(-7, 5, m0)))
        B = rng.standard_normal((nb, m0)) * np.logspace(-12, -1, m0)[None, :]
        G[m0:, :m0] = B
        G[:m0, m0:] = B.T
        C = rng.standard_normal((nb, nb)) * 0.3
        G[m0:, m0:] = C + C.T + np.diag(rng.uniform(-3, 3, nb))
        out.append((f"bordered{m0}+{nb}", G, False))
    n = 40
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    out.append(("cluster1e-8", Q @ np.diag(np.linspace(0, 1e-8, n) + 3) @ Q.T, False))
    ev = np.sort(rng.uniform(-1, 1, n))
    ev[5:9] = ev[5]
    out.append(("repeated", Q @ np.diag(ev) @ Q.T, None))
    blk = rng.standard_normal((10, 10))
    out.append(("identical_blocks", np.kron(np.eye(4), blk + blk.T), None))
    out.append(("diagonal", np.diag(rng.uniform(-1, 1, 30)), False))
    out.append(("scalar", 2.5 * np.eye(30), None))
    out.append(("rank_one", np.ones((12, 12)), None))
    out.append(("zero", np.zeros((5, 5)), False))
    W = np.diag(np.abs(np.arange(-10, 11)).astype(float)) + np.diag(np.ones(20), 1) + np.diag(np.ones(20), -1)
    out.append(("wilkinson21", W, False))
    M = rng.standard_normal((50, 50))
    out.append(("scale1e150", (M + M.T) * 1e150, False))
    out.append(("scale1e-150", (M + M.T) * 1e-150, False))
    return out


CASES = _cases()


def _check(G, th, Y):
    n = G.shape[0]
    w = np.linalg.eigvalsh(_sym(G))
    nrm = max(np.abs(w).max(), np.finfo(float).tiny)
    assert np.all(np.diff(th) >= -1e-14 * nrm)
    assert np.abs(th - w).max() <= 1e-13 * nrm, np.abs(th - w).max() / nrm
    assert np.abs(Y.T @ Y - np.eye(n)).max() <= 1e-13
    assert np.abs(_sym(G) @ Y - Y * th[None, :]).max() <= 1e-13 * nrm


@pytest.fixture(scope="module")
def ctx():
    import paper_1709_03005_amd as cc
    c = cc.Context()
    yield c
    c.close()


@pytest.mark.parametrize("name,G,fb_expected", CASES, ids=[c[0] for c in CASES])
def test_subspace_eig(ctx, name, G, fb_expected):
    import paper_1709_03005_amd as cc
    print(f"[rr] {name} n={G.shape[0]}", flush=True)
    th, Y, fb = ctx.subspace_eig(G, cc.CCH_EIG_AUTO)
    _check(G, th, Y)
    if fb_expected is not None:
        assert fb == fb_expected


@pytest.mark.parametrize("name,G,fb_expected", CASES[::4], ids=[c[0] for c in CASES[::4]])
def test_subspace_eig_jacobi(ctx, name, G, fb_expected):
    import paper_1709_03005_amd as cc
    th, Y, fb = ctx.subspace_eig(G, cc.CCH_EIG_JACOBI)
    _check(G, th, Y)
    assert not fb


def test_input_validation(ctx):
    import paper_1709_03005_amd as cc
    with pytest.raises(cc.CchError):
        ctx.subspace_eig(np.eye(97))
