"""Host-side pieces of the benchmark (no GPU): every kernel family keyed for
counter-measured traffic resolves to a source region (its marker lines are
still in the file), the regions are not empty, and the refusal of a run on
several GPUs comes back as one JSON line with a non-zero exit status."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_contract", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_families_resolve_to_source():
    b = _bench()
    for family in b.KERNEL_SOURCE:
        assert b.source_hash(family) is not None, family
    for (_, family), entry in b.TRAFFIC.items():
        assert family in b.KERNEL_SOURCE
        assert len(entry[0]) == 16 and entry[1] > 0 and entry[2] > 0


def test_several_gpus_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus_requested"] == 2 and "one GPU" in line["error"]
