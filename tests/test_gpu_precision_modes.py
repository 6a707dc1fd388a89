"""Reduced-precision expansion products (FP32; split-BF16 with s slices)
against the FP64 oracle. The max-abs element error and the eigenvalue error
of each mode are printed; bounds: split-BF16 with 7 slices agrees with the
oracle to 1e-12 of the largest element (56 bits per operand, exact slice
products), FP32 and 3-slice BF16 to 1e-5 (24-bit operands)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

_cache = {}


def _oracle(name):
    if name not in _cache:
        inst = synth.CONFIGS[name]()
        H = oracle.Oracle(inst).build()
        _cache[name] = (inst, H, np.linalg.eigvalsh(H))
    return _cache[name]


@pytest.mark.parametrize("name", ["small", "wide"])
@pytest.mark.parametrize("mode,slices,bound", [("fp32", 0, 1e-5), ("bf16", 7, 1e-12), ("bf16", 3, 1e-5)])
def test_precision_mode(name, mode, slices, bound):
    import paper_1709_03005_amd as cc
    inst, H, w = _oracle(name)
    prec = cc.CCH_PREC_FP32 if mode == "fp32" else cc.CCH_PREC_SPLIT_BF16
    with cc.from_instance(inst, precision=prec, split_slices=slices) as ctx:
        ctx.build()
        G = ctx.get_matrix()
        ev, _, info, rc = ctx.davidson(5, tol=1e-8, want_vectors=False)
    assert np.array_equal(G, G.T)
    scale = np.abs(H).max()
    err = np.abs(G - H).max()
    eerr = np.abs(ev - w[:5]).max()
    print(f"[{name} {mode}{slices or ''}] max-abs element error {err:.3e} (rel {err / scale:.3e}), "
          f"eigenvalue error {eerr:.3e}")
    assert err <= bound * scale
    assert rc == cc.CCH_OK
    assert eerr <= max(10 * bound * scale, 1e-10 * np.abs(w).max())
    # only the continuum-continuum block changes with the mode
    Dc = inst.n_cont_rows()
    np.testing.assert_allclose(G[Dc:], H[Dc:], rtol=0, atol=1e-12 * scale)


def test_bad_precision_options():
    import paper_1709_03005_amd as cc
    inst = synth.tiny()
    ctx = cc.from_instance(inst, plan=False)
    with pytest.raises(cc.CchError) as e:
        ctx.plan(precision=7)
    assert e.value.code == cc.CCH_E_INVALID_ARG
    with pytest.raises(cc.CchError) as e:
        ctx.plan(precision=cc.CCH_PREC_SPLIT_BF16, split_slices=9)
    assert e.value.code == cc.CCH_E_INVALID_ARG
    ctx.close()
