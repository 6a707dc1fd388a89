"""cch_subspace_eig_noalloc (the allocation-free form of cch_subspace_eig,
for callers that cannot allocate device memory) against cch_subspace_eig,
through the C ABI: the same kernels on the same input give the same bits.
Two calls in a row share the per-GPU scratch array, the second with a
smaller matrix, for host and for device arrays; the fallback counter starts
at zero on every call; sizes beyond the scratch limit are refused."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _sym(n, seed):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n))
    return M + M.T


def _call(cc, fn, ctx, G, method, dev):
    """(theta, Y, fallback, status) of one entry point, host or device arrays."""
    import torch
    m = G.shape[0]
    fb = C.c_int32(-1)
    if dev:
        tG = torch.from_numpy(G).cuda()
        tT = torch.zeros(m, dtype=torch.float64, device="cuda")
        tY = torch.zeros((m, m), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        rc = fn(ctx.h, C.c_void_p(tG.data_ptr()), m, m, C.c_void_p(tT.data_ptr()), C.c_void_p(tY.data_ptr()), m,
                method, C.byref(fb), cc.CCH_MEM_DEVICE)
        return tT.cpu().numpy(), tY.cpu().numpy(), fb.value, rc
    theta = np.zeros(m)
    Y = np.zeros((m, m))
    rc = fn(ctx.h, G.ctypes.data_as(C.c_void_p), m, m, theta.ctypes.data_as(C.c_void_p),
            Y.ctypes.data_as(C.c_void_p), m, method, C.byref(fb), cc.CCH_MEM_HOST)
    return theta, Y, fb.value, rc


@pytest.mark.parametrize("dev", [False, True])
@pytest.mark.parametrize("method_name", ["auto", "jacobi"])
def test_noalloc_matches_allocating_entry_point(dev, method_name):
    import torch
    assert torch.cuda.is_available()
    import paper_1709_03005_amd as cc
    method = cc.CCH_EIG_AUTO if method_name == "auto" else cc.CCH_EIG_JACOBI
    with cc.Context(0, torch.cuda.current_stream().cuda_stream) as ctx:
        for m, seed in ((96, 1), (37, 2)):       # second call smaller than the first
            G = _sym(m, seed)
            t0, Y0, f0, r0 = _call(cc, cc.lib.cch_subspace_eig, ctx, G, method, dev)
            t1, Y1, f1, r1 = _call(cc, cc.lib.cch_subspace_eig_noalloc, ctx, G, method, dev)
            print(f"[noalloc dev={dev} {method_name}] m={m} status {r0}/{r1} fallback {f0}/{f1}", flush=True)
            assert r0 == cc.CCH_OK and r1 == cc.CCH_OK
            assert np.array_equal(t0, t1)
            assert np.array_equal(Y0, Y1)
            assert f0 == f1 == 0
            w = np.linalg.eigvalsh(G)
            assert np.abs(t1 - w).max() <= 1e-12 * np.abs(w).max()


def test_noalloc_refuses_oversize():
    import torch
    import paper_1709_03005_amd as cc
    with cc.Context(0, torch.cuda.current_stream().cuda_stream) as ctx:
        G = _sym(97, 3)
        th = np.zeros(97)
        Y = np.zeros((97, 97))
        fb = C.c_int32()
        rc = cc.lib.cch_subspace_eig_noalloc(ctx.h, G.ctypes.data_as(C.c_void_p), 97, 97,
                                             th.ctypes.data_as(C.c_void_p), Y.ctypes.data_as(C.c_void_p), 97,
                                             cc.CCH_EIG_AUTO, C.byref(fb), cc.CCH_MEM_HOST)
        assert rc == cc.CCH_E_INVALID_ARG
        assert "96" in ctx.last_error()
        # the context and the scratch stay usable
        t, _, fell = ctx.subspace_eig_noalloc(_sym(12, 4))
        assert not fell
        assert np.abs(t - np.linalg.eigvalsh(_sym(12, 4))).max() < 1e-12 * 20
