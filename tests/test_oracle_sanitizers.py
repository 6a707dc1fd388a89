"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (gcc).

`oracle/sancheck.c` is compiled with ccoracle.c and both sanitizers, reads an
instance whose every array sits in a heap block of exactly its size, builds
the whole contracted matrix, a sample of elements and the excitation pair
lists, and writes them back. A sanitizer report ends the run with a non-zero
status; the outputs must equal the ordinary (OpenMP, -O2) build's bit for bit.
Instances: one word (tiny, micro), the 64-bit word boundary (wide), the
symmetry-packed integral layout, and three words (spin-orbitals across 128).
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_DIR = os.path.join(os.path.dirname(HERE), "oracle")


@pytest.fixture(scope="module")
def sancheck(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("san") / "sancheck")
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-o", exe, os.path.join(ORACLE_DIR, "sancheck.c"), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower():
        pytest.skip("gcc has no sanitizer runtime here: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    return exe


def _dump(inst, path, rows, cols):
    recs = []

    def rec(a, dt):
        recs.append(np.ascontiguousarray(a, dtype=dt).tobytes())
    packed = bool(getattr(inst, "packed", False))
    rec([inst.n_o, inst.n_cont, inst.n_elec, inst.n_words, len(inst.syms),
         0 if inst.l2_dets is None else inst.l2_dets.shape[0], inst.total_irrep, inst.n_irrep,
         int(packed), len(rows)], np.int32)
    rec([inst.e_core], np.float64)
    for a in (inst.h, inst.tttt, inst.tttc, inst.ttcc, inst.tctc):
        rec(a, np.float64)
    if packed:
        prec, blk = synth.packed_layout(inst.tgt_irrep, inst.n_c)
        rec(prec, np.int64)
        rec(blk.ravel(), np.int64)
        rec(inst.tgt_irrep, np.int32)
        rec(np.repeat(np.arange(inst.n_irrep), inst.n_c), np.int32)
        rec(np.concatenate([np.arange(n) for n in inst.n_c]), np.int32)
        rec(inst.n_c, np.int32)
    rec(np.concatenate([[0], np.cumsum(inst.n_c)]), np.int32)
    rec([s.irrep for s in inst.syms], np.int32)
    rec([s.dets.shape[0] for s in inst.syms], np.int32)
    rec([s.ci.shape[1] for s in inst.syms], np.int32)
    for s in inst.syms:
        rec(s.dets, np.uint64)
        rec(s.ci, np.float64)
    rec(inst.l2_dets if inst.l2_dets is not None else np.zeros((0, inst.n_words)), np.uint64)
    rec(rows, np.int64)
    rec(cols, np.int64)
    with open(path, "wb") as f:
        for b in recs:
            f.write(np.int64(len(b)).tobytes())
            f.write(b)


def _read(path, D, n_sample):
    raw = open(path, "rb").read()
    off = 0
    H = np.frombuffer(raw, np.float64, D * D, off).reshape(D, D)
    off += 8 * D * D
    v = np.frombuffer(raw, np.float64, n_sample, off)
    off += 8 * n_sample
    lists = []
    for _ in range(2):
        n = int(np.frombuffer(raw, np.int64, 1, off)[0])
        off += 8
        x = np.frombuffer(raw, np.int32, n, off); off += 4 * n
        y = np.frombuffer(raw, np.int32, n, off); off += 4 * n
        d = np.frombuffer(raw, np.int8, n, off); off += n
        p = np.frombuffer(raw, np.int8, n, off); off += n
        lists.append(dict(x=x, y=y, deg=d, phase=p))
    assert off == len(raw)
    return H, v, lists


INSTANCES = {
    "tiny": synth.tiny,
    "micro": lambda: synth.micro(7, n_o=4, n_elec=2, n_c=3, n_irrep=2),
    "wide": synth.wide,
    "packed": lambda: synth.make_instance(8, 4, 2, [4, 3], [0, 1], [10, 8], [3, 2], 24, 917,
                                          packed=True, name="packed_san"),
    "three_words": lambda: synth.boundary(3),
}


@pytest.mark.parametrize("name", sorted(INSTANCES))
def test_oracle_clean_under_sanitizers(sancheck, tmp_path, name):
    inst = INSTANCES[name]()
    orc = oracle.Oracle(inst)
    D = orc.dim
    rng = np.random.default_rng(5)
    rows, cols = rng.integers(0, D, 64), rng.integers(0, D, 64)
    fin, fout = str(tmp_path / "inst.bin"), str(tmp_path / "out.bin")
    _dump(inst, fin, rows, cols)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24", OMP_NUM_THREADS="2")
    r = subprocess.run([sancheck, fin, fout], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    H, v, (tt, lt) = _read(fout, D, len(rows))
    assert np.array_equal(H, orc.build())
    assert np.array_equal(v, orc.elements(rows, cols)[0])
    ref = oracle.pairs(inst.syms[0].dets, inst.syms[0].dets, lower=True)
    for key in ("x", "y", "deg", "phase"):
        assert np.array_equal(tt[key], ref[key]), key
    if inst.l2_dets is not None and inst.l2_dets.shape[0]:
        ref = oracle.pairs_l2tgt(inst.l2_dets, inst.syms[0].dets, inst.n_o)
        assert len(lt["x"]) == len(ref["x"]) > 0
        for key in ("x", "y", "deg", "phase"):
            assert np.array_equal(lt[key], ref[key]), key
