"""Device-memory budget: a budget below the one-pass plan splits the expansion
product into passes over the continuum orbitals and the matrix is the same,
bit for bit; a budget that cannot hold one orbital per pass is refused with
CCH_E_OOM before anything runs; a split context cannot join a batch."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,frac,min_passes", [("small", 5, 2), ("wide", 5, 2), ("medium", 5, 1),
                                                   ("medium", 40, 2)])
def test_multipass_equals_single_pass(name, frac, min_passes):
    import paper_1709_03005_amd as cc
    inst = synth.CONFIGS[name]()
    with cc.from_instance(inst) as ref:
        ref.build()
        G0 = ref.get_matrix()
        bytes0, passes0 = ref.plan_info()
        b_elems = ref.work_counts()["relayout_bytes"] / 16.0   # integral-row elements of all pairs
    assert passes0 == 1
    # the integral rows of all pairs replaced by 1/frac of their size: one shared
    # buffer, each pair laid out before its product, in one or more passes
    budget = int(bytes0 - 8 * b_elems + 8 * b_elems // frac)
    with cc.from_instance(inst, plan=False) as ctx:
        ctx.plan(max_device_bytes=budget)
        got_bytes, passes = ctx.plan_info()
        print(f"[{name}] one pass {bytes0} B, budget {budget} B -> {got_bytes} B in {passes} passes", flush=True)
        assert passes >= min_passes and got_bytes <= budget
        ctx.build()
        G = ctx.get_matrix()
        with pytest.raises(cc.CchError):
            cc.Batch([ctx])
    assert np.array_equal(G, G0)


def test_budget_too_small_is_refused():
    import paper_1709_03005_amd as cc
    inst = synth.small()
    with cc.from_instance(inst) as ref:
        bytes0, _ = ref.plan_info()
        b_elems = ref.work_counts()["relayout_bytes"] / 16.0
    with cc.from_instance(inst, plan=False) as ctx:
        with pytest.raises(cc.CchError) as e:
            ctx.plan(max_device_bytes=int(bytes0 - 8 * b_elems + 8))
        assert e.value.code == cc.CCH_E_OOM
