"""Benchmark: CI-contracted close-coupling Hamiltonian build + Davidson on one MI355X.

One step = the whole hot path on one batch of synthetic input, inputs already
resident in HBM: cch_build (excitation scans, target densities, relayout,
FP64 MFMA expansion, class 4, classes 2/8, mirror) followed by cch_davidson
(lowest k eigenpairs to residual tol, FP64, diagonal correction). This is the
plain form. Default workload: the learned-preconditioner test instance, the
largest single-GPU configuration (40 target orbitals, N = 12, 8000 dets x 50
states, 400 continuum orbitals, 40000 L2; D = 60000; lowest 10 to 1e-8).

Beside the timed plain steps, the chosen forms are timed on the same matrix
(outside the timed region): the Davidson solve with the trained network's
correction (learned workload), with the L2 block as CSR in the mat-vec, and,
on the precision workload, the reduced-precision expansion products.

Workloads: learned (default), medium (D = 8000), medium_te (D = 8000, true
target states with their energies on the diagonal; classes 5 and 6 between
symmetries sharing a determinant space), tiny, small, precision (D = 40000),
l2heavy (D = 122815), batch (64 instances, batched vs one after another).

Prints ONE JSON line. `value` = lower-triangle Hamiltonian elements per second
of the whole plain step (build + solve); the build-only rate and the
time-to-eigenpairs are separate fields.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Hamiltonian elements/s + Davidson time-to-eigenpairs, plain vs chosen form"
HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6
# FP64 vector peak from the unit counts: 256 CUs x 4 SIMDs x 16 lanes x 2 flops
# (one FMA per lane per cycle) x 2.4 GHz = 78.6 TFLOP/s
FP64_VALU_PEAK_TFLOPS = 78.6

# HBM bytes per launch of a workload's kernels: rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes (KiB per dispatch, averaged over one step), scaled by what
# the same counters read for a plain 512 MiB device copy (bench.py --workload
# copy: FETCH_SIZE reads half the bytes, WRITE_SIZE all of them). Keyed by
# workload and kernel family, with the hash of the family's source text when
# counted (the region of its file between two marker lines, or the whole
# file): a family whose source has changed since reports null. The relayout
# entry is the sum of its two launches (J and K layouts), the mat-vec entry the
# sum of the product and its reduction of partial sums.
COUNTER_SCALE = {"FETCH_SIZE": 2.0, "WRITE_SIZE": 1.0}
KERNEL_SOURCE = {
    # family: (file, first marker line, marker line after the region), None = whole file
    "matvec": ("k_davidson.hip", "// K8 from the lower triangle only", "// K9: tall-skinny products"),
    "expansion_gemm": ("k_gemm.hip", "// K5: C = A * B", "// Persistent form over many"),
    "relayout": ("k_gemm.hip", "// K0: B[k][jj*ncb + jj']", "// K5: C = A * B"),
    "class4": ("k_class4.hip", None, None),
    "l2_block": ("k_l2.hip", "// Classes 2 and 8", "// L2 functions given as CSFs"),
    "mirror": ("k_misc.hip", "// H[c][r] = H[r][c]", "__global__ void k_diag"),
    "rayleigh_ritz": ("k_rr.hip", None, None),
}
TRAFFIC = {
    # (workload, family): (sha256 prefix of the family's source, FETCH_SIZE KiB, WRITE_SIZE KiB)
    ("medium", "rayleigh_ritz"): ("ad413139aab2388c", 53.878, 25.493),
    ("medium", "l2_block"): ("238d74161bdf3234", 22104.250, 98764.125),
    # the product instances of one solve (49 of three vector groups, 7 of one,
    # 2 of two, 1 of four) averaged per launch, plus the reduction
    ("learned", "matvec"): ("7818879eb813e1ad", 7412237.1, 567456.0),
    ("learned", "expansion_gemm"): ("7eeac111dbc075d6", 16520452.1, 1562812.5),
    ("learned", "relayout"): ("29b301ee4afa7f1b", 2000324.2, 4000000.0),
    ("learned", "class4"): ("1c100f7420acfa5b", 5756553.2, 10223622.8),
    ("learned", "l2_block"): ("238d74161bdf3234", 1770334.4, 6273721.4),
    ("learned", "mirror"): ("e5a76a20e4f84e29", 7038936.4, 14062968.8),
}


def source_hash(kernel):
    """sha256 prefix of a kernel family's source text, or None."""
    import hashlib
    f, a, b = KERNEL_SOURCE[kernel]
    path = os.path.join(ROOT, "paper_1709_03005_amd", "csrc", f)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if a is not None:
        i = text.find(a)
        j = text.find(b, i + 1) if i >= 0 else -1
        if i < 0 or j < 0:
            return None
        text = text[i:j]
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def traffic_bytes(kernel, workload):
    """Counter-measured HBM bytes per launch, or None."""
    t = TRAFFIC.get((workload, kernel))
    if t is None or source_hash(kernel) != t[0]:
        return None
    return 1024.0 * (t[1] * COUNTER_SCALE["FETCH_SIZE"] + t[2] * COUNTER_SCALE["WRITE_SIZE"])


WORKLOADS = {
    # name: (generator, k, tol, CPU-baseline mode)
    "learned": ("learned_test", 10, 1e-8, "elements"),
    "medium": ("medium", 10, 1e-8, "rows"),
    # true target states on the diagonal (target-energy option), two pairs of
    # symmetries sharing a determinant space: classes 5 and 6 in the build
    "medium_te": ("medium_pairs", 10, 1e-8, "rows"),
    "tiny": ("tiny", 5, 1e-8, "rows"),
    "small": ("small", 10, 1e-8, "rows"),
    "precision": ("precision", 10, 1e-8, "elements"),
    "l2heavy": ("l2heavy", 10, 1e-8, "elements"),   # D = 122815, dense matrix of 121 GB
    "l2huge": ("l2huge", 10, 1e-8, "elements"),     # D = 250712, only with the sparse L2 build
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _oracle_rate(O, inst, mode, budget_s, rng):
    """(elements/s, sample description, oracle seconds, (rows, cols, values))
    of the oracle on a bounded sample of the matrix (see cpu_baseline)."""
    import numpy as np
    D = inst.dim()
    Dc = inst.n_cont_rows()
    if mode == "elements":
        counts = {"cont_cont": Dc * (Dc + 1) / 2, "l2_cont": float(inst.n_l2) * Dc,
                  "l2_l2": inst.n_l2 * (inst.n_l2 + 1) / 2}
        per_el, n_tot, t_tot = {}, 0, 0.0
        got_r, got_c, got_v = [], [], []
        for cls, cnt in counts.items():
            if cnt == 0:
                continue
            n_s, t_c, n_c = 16, 0.0, 0
            while t_c < budget_s / 3 and n_c < (1 << 17):
                if cls == "cont_cont":
                    r = rng.integers(0, Dc, n_s); c = rng.integers(0, Dc, n_s)
                elif cls == "l2_cont":
                    r = rng.integers(Dc, D, n_s); c = rng.integers(0, Dc, n_s)
                else:
                    r = rng.integers(Dc, D, n_s); c = rng.integers(Dc, D, n_s)
                r, c = np.maximum(r, c), np.minimum(r, c)
                t = time.perf_counter()
                v, _, _ = O.elements(r, c)
                t_c += time.perf_counter() - t
                got_r.append(r); got_c.append(c); got_v.append(v)
                n_c += n_s
                n_s *= 2
            per_el[cls] = t_c / n_c
            n_tot += n_c
            t_tot += t_c
            log(f"cpu baseline {cls}: {n_c} elements in {t_c:.1f} s")
        total = sum(counts.values())
        est = sum(counts[c] * per_el[c] for c in per_el)
        desc = (f"{n_tot} seeded lower-triangle elements of the same matrix, drawn per block class "
                f"({', '.join(f'{c}: {per_el[c] * 1e6:.1f} us/element' for c in per_el)}), "
                f"weighted by the class sizes; {t_tot:.1f} s of oracle time")
        return total / est, desc, t_tot, tuple(np.concatenate(x) for x in (got_r, got_c, got_v))
    groups = 0
    t_total = 0.0
    n_el = 0
    got_r, got_c, got_v = [], [], []
    while t_total < budget_s * 0.5 and groups < 8:
        rows_c = []
        r0 = 0
        for sy in inst.syms:
            nc = int(inst.n_c[sy.irrep ^ inst.total_irrep])
            S = sy.ci.shape[1]
            if nc:
                jj = int(rng.integers(nc))
                rows_c += [r0 + n * nc + jj for n in range(S)]
            r0 += S * nc
        n_l2_rows = max(1, int(round(len(rows_c) * inst.n_l2 / max(Dc, 1))))
        rows_l = list(Dc + rng.choice(inst.n_l2, size=min(n_l2_rows, inst.n_l2), replace=False))
        rows = np.array(rows_c + rows_l, dtype=np.int64)
        t = time.perf_counter()
        Hr = O.build_rows(rows)
        t_total += time.perf_counter() - t
        n_el += rows.size * D
        groups += 1
        pick = rng.integers(0, D, 64)
        got_r.append(np.repeat(rows, pick.size)); got_c.append(np.tile(pick, rows.size))
        got_v.append(np.asarray(Hr)[:, pick].ravel())
        log(f"cpu baseline group {groups}: {rows.size} rows, {t_total:.1f} s")
    desc = (f"{groups} stratified row groups of the same matrix ({n_el // D} full rows: one continuum "
            f"orbital x all states per symmetry + L2 rows in proportion), {t_total:.1f} s")
    return n_el / t_total, desc, t_total, tuple(np.concatenate(x) for x in (got_r, got_c, got_v))


def cpu_baseline(inst, mode="rows", budget_s=20.0):
    """The CPU oracle, timed on a bounded sample of the same matrix, with all
    the host's threads and with one thread.

    mode "rows": stratified groups of full rows, each group the rows of one
    continuum orbital (all states) per target symmetry plus L2 rows in the
    matrix's continuum : L2 proportion; elements/s over full rows (both
    triangles, as the oracle computes them).

    mode "elements": for matrices where one continuum row alone takes the
    oracle minutes (thousands of target determinants), the oracle's
    per-element path on a seeded sample of each block class of the lower
    triangle (continuum-continuum, L2-continuum, L2-L2); the per-class
    times per element are weighted by the class sizes into one rate for the
    whole lower triangle.

    Returns the baseline record and the sampled oracle elements (rows, cols,
    values), against which the benchmark states the error of every form."""
    import numpy as np

    import oracle
    O = oracle.Oracle(inst)
    nthr = oracle.num_threads()
    v_all, d_all, t_all, sample = _oracle_rate(O, inst, mode, budget_s, np.random.default_rng(7))
    oracle.set_threads(1)
    try:
        v_one, d_one, t_one, _ = _oracle_rate(O, inst, mode, budget_s / 2, np.random.default_rng(8))
    finally:
        oracle.set_threads(nthr)
    rec = {"value": v_all, "unit": "elements/s", "cores": nthr, "kind": "oracle", "sample": d_all,
           "seconds": t_all,
           "single_thread": {"value": v_one, "unit": "elements/s", "cores": 1, "sample": d_one,
                             "seconds": t_one}}
    return rec, sample


def bench_eig_all(args):
    """Every eigenpair of the medium workload's built matrix (D = 8000) by
    cch_eig_all (Householder tridiagonalisation, multisection, twisted
    factorisations, MFMA back-transformation), device phase times from the
    library's HIP events; the roofline entries are the reduction's HBM bytes
    and the back-transformation's FP64 MFMA flops."""
    import numpy as np
    import torch

    import paper_1709_03005_amd as cc
    import synth

    inst = synth.CONFIGS["medium"]()
    torch.cuda.init()
    stream = torch.cuda.current_stream().cuda_stream
    ctx = cc.from_instance(inst, device=0, stream=stream)
    ctx.build()
    D = inst.dim()
    # results stay in HBM (device arrays): the phase times hold no copy to the host
    for _ in range(args.warmup):
        ctx.eig_all(vectors=True, device=True)
    tri, evs, vecs, walls = [], [], [], []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        w, V, info = ctx.eig_all(vectors=True, device=True)
        walls.append(time.perf_counter() - t0)
        tri.append(info.tridiag_ms)
        evs.append(info.eigenvalues_ms)
        vecs.append(info.vectors_ms)
    dev_ms = float(np.mean(tri) + np.mean(evs) + np.mean(vecs))
    # a residual sample: the lowest, a middle and the highest pairs against the
    # built matrix, the products formed on the device by cch_apply
    sel = [0, 1, D // 2, D - 1]
    w = w.cpu().numpy()
    V = V[sel].cpu().numpy()
    HV = ctx.apply(np.ascontiguousarray(V))
    res = float(max(np.linalg.norm(HV[i] - w[e] * V[i]) for i, e in enumerate(sel)))
    ctx.close()
    tri_ms, vec_ms = float(np.mean(tri)), float(np.mean(vecs))
    out = {
        "metric": "eigenpairs/s (full spectrum, FP64)",
        "value": D / (dev_ms * 1e-3),
        "unit": "eigenpairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dev_ms, "wall_ms_per_step": 1e3 * float(np.mean(walls)),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "eig_all", "matrix": "medium (D = 8000) built matrix", "dim": D},
        "phase_ms": {"tridiagonalisation": tri_ms, "eigenvalues": float(np.mean(evs)), "vectors": vec_ms},
        "kernels": {
            "tridiagonalisation": {"bound": "hbm", "achieved": info.tridiag_bytes / (tri_ms * 1e-3) / 1e9,
                                   "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                   "note": "lower triangle of the trailing block: 8 B per element per column (its product) + 16 B per element per 32-column panel (its update)"},
            "vectors": {"bound": "mfma", "achieved": info.backtransform_flops / (vec_ms * 1e-3) / 1e12,
                        "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "note": "back-transformation 2 n^3 flops over the whole vector phase (twisted "
                                "factorisations and cluster orthogonalisation included): a lower bound"},
        },
        "clusters": int(info.clusters), "clustered_eigenvalues": int(info.clustered),
        "max_residual_sample": res,
    }
    for v in out["kernels"].values():
        v["frac"] = v["achieved"] / v["peak"]
    print(json.dumps(out))
    return out


def bench_batch(args):
    """64 seeded instances (D ~ U[500, 6000]) built one after another with
    cch_build (plain) and together with cch_batch_build (persistent launches
    in one hipGraph, autotuned); elements/s of both on the same GPU."""
    import numpy as np
    import torch

    import paper_1709_03005_amd as cc
    import synth
    t = time.perf_counter()
    insts = [synth.batch_instance(i) for i in range(args.instances)]
    print(f"[bench] batch of {len(insts)} generated in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.init()
    ctxs = [cc.from_instance(I) for I in insts]
    lower = sum(c.work_counts()["lower_elements"] for c in ctxs)
    # plain: one cch_build per instance, back to back
    for c in ctxs:
        c.build()
    for c in ctxs:
        c.sync()
    plain = []
    for _ in range(max(1, args.steps)):
        t0 = time.perf_counter()
        for c in ctxs:
            c.build()
        for c in ctxs:
            c.sync()
        plain.append(time.perf_counter() - t0)
    t = time.perf_counter()
    b = cc.Batch(ctxs, autotune=True)
    tune_s = time.perf_counter() - t
    for _ in range(args.warmup):
        b.build()
    batched, dev = [], []
    for _ in range(max(1, args.steps)):
        t0 = time.perf_counter()
        b.build()
        batched.append(time.perf_counter() - t0)
        dev.append(b.time_ms())
    info = b.info()
    ms = float(np.median(batched)) * 1e3
    out = {
        "metric": METRIC, "value": lower / (ms * 1e-3), "unit": "elements/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic (64 seeded instances)",
        "config": {"workload": "batch", "instances": len(insts), "dims": [I.dim() for I in insts],
                   "target_symmetries": [len(I.syms) for I in insts],
                   "integrals": "symmetry-packed (tt|cc), (tc|tc)", "total_lower_elements": lower},
        "batched_device_ms": float(np.median(dev)),
        "plain_ms": float(np.median(plain)) * 1e3,
        "plain_elements_per_s": lower / float(np.median(plain)),
        "speedup_vs_plain": float(np.median(plain)) / float(np.median(batched)),
        "batch_info": info, "autotune_and_capture_s": tune_s,
    }
    b.close()
    for c in ctxs:
        c.close()
    print(json.dumps(out))


def _prec(name, cc):
    if name == "fp64":
        return cc.CCH_PREC_FP64, 0
    if name == "fp32":
        return cc.CCH_PREC_FP32, 0
    if name.startswith("bf16x"):
        return cc.CCH_PREC_SPLIT_BF16, int(name[5:])
    raise SystemExit(f"unknown precision form {name}")


def _solve_stats(ctx, cc, k, tol, reps, **kw):
    """Median wall time (ms), iterations and eigenvalues of `reps` solves."""
    import numpy as np
    ms, it, ev, rc = [], [], None, None
    for _ in range(reps):
        ev, _, info, rc = ctx.davidson(k, tol=tol, want_vectors=False, **kw)
        ms.append(info.seconds * 1e3)
        it.append(info.iterations)
    return float(np.median(ms)), int(np.median(it)), np.array(ev), int(rc), info


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="learned",
                    choices=sorted(WORKLOADS) + ["batch", "copy", "eig_all", "peaks"],
                    help="copy: three plain 512 MiB device copies, the calibration run for HBM counters; "
                         "peaks: the measured copy rate and FP64 issue rates beside the published peaks")
    ap.add_argument("--instances", type=int, default=64, help="batch workload: number of instances")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="time the plain step only (no chosen forms)")
    ap.add_argument("--precision", default="fp64",
                    help="expansion GEMM form of the timed step: fp64, fp32, or bf16xS (split-BF16, S slices)")
    ap.add_argument("--precond", default="jacobi", choices=["jacobi", "mlp"],
                    help="Davidson correction of the timed step: diagonal (Jacobi) or the trained network "
                         "(paper_1709_03005_amd/mlp_weights.npy)")
    ap.add_argument("--restart", default="auto", choices=["auto", "thick", "prev"],
                    help="Davidson restart of the timed step: the library's default (auto), the lowest 2k Ritz "
                         "vectors (thick), or with the previous Ritz vectors kept (prev)")
    ap.add_argument("--sparse-l2", action="store_true",
                    help="timed step with the L2 block as CSR of its non-zeros in the mat-vec")
    ap.add_argument("--sparse-build", action="store_true",
                    help="classes 2 and 8 built and stored as CSR (cch_plan CCH_PLAN_SPARSE_L2); implied by l2huge")
    ap.add_argument("--target-energies", action="store_true",
                    help="build classes 1, 3, 5, 6, 7 with target energies on the diagonal in place of "
                         "the target-only integrals (synthetic energies; the timing does not depend on them)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "ccham runs on one GPU per process (no multi-GPU path); --gpus must be 1",
                          "n_gpus_requested": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1709_03005_amd as cc
    import synth

    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "eig_all":
        return bench_eig_all(args)
    if args.workload == "copy":
        n = 64 << 20
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"workload": "copy", "bytes_per_copy": n * 8, "copies": 3}))
        return None
    if args.workload == "peaks":
        # the roofline denominators confirmed on this device: a plain device copy
        # (bytes read + written) and the FP64 issue rates of cch_probe_fp64
        n = 64 << 20
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        best = None
        for _ in range(6):
            e0.record()
            b.copy_(a)
            e1.record()
            e1.synchronize()
            t = e0.elapsed_time(e1)
            best = t if best is None else min(best, t)
        rates = cc.probe_fp64(0, torch.cuda.current_stream().cuda_stream)
        print(json.dumps({"workload": "peaks", "copy_GBps": 2 * n * 8 / (best * 1e-3) / 1e9,
                          "copy_bytes": 2 * n * 8, "fp64_tflops": rates,
                          "published": {"hbm_GBps": HBM_PEAK_GBS, "fp64_mfma_tflops": FP64_MFMA_PEAK_TFLOPS,
                                        "fp64_vector_tflops": FP64_VALU_PEAK_TFLOPS}}))
        return None
    gen, k, tol, cpu_mode = WORKLOADS[args.workload]
    t_gen = time.perf_counter()
    inst = synth.CONFIGS[gen]()
    t_gen = time.perf_counter() - t_gen
    log(f"workload {args.workload}: D={inst.dim()} generated in {t_gen:.1f} s")

    torch.cuda.init()
    stream = torch.cuda.current_stream().cuda_stream
    prec, slices = _prec(args.precision, cc)
    energies = None
    if args.target_energies:
        energies = [-1.0 - 0.01 * np.arange(sym.ci.shape[1]) for sym in inst.syms]
    if args.workload == "medium_te":
        # the target states: eigenvectors of each determinant space's target
        # Hamiltonian (read from a build of the library, diagonalised on the
        # host as a target CI program would); the first member of a pair takes
        # the lowest S, the second the next S, with their energies
        t = time.perf_counter()
        c0 = cc.from_instance(inst, device=0, stream=stream)
        c0.build()
        energies = []
        for a in range(0, len(inst.syms), 2):
            w, v = np.linalg.eigh(c0.target_hamiltonian(a, a))
            S = inst.syms[a].ci.shape[1]
            inst.syms[a].ci = np.ascontiguousarray(v[:, :S])
            inst.syms[a + 1].ci = np.ascontiguousarray(v[:, S:2 * S])
            energies += [w[:S], w[S:2 * S]]
        c0.close()
        log(f"target states from the target Hamiltonian in {time.perf_counter() - t:.1f} s")
    t_up = time.perf_counter()
    ctx = cc.from_instance(inst, device=0, stream=stream, plan=False)   # inputs host -> HBM
    if energies is not None:
        ctx.set_target_energies(energies)
    ctx.sync()
    upload_s = time.perf_counter() - t_up
    sparse_build = args.sparse_build or args.workload == "l2huge"
    t = time.perf_counter()
    ctx.plan(precision=prec, split_slices=slices, sparse_l2=sparse_build)
    ctx.sync()
    plan_s = time.perf_counter() - t
    log(f"planned in {plan_s:.1f} s")
    lower = ctx.work_counts()["lower_elements"]
    net = None
    if args.precond == "mlp" or (args.workload == "learned" and not args.no_forms):
        net = cc.Mlp(device=0, stream=stream)
        net.set_weights(np.load(os.path.join(ROOT, "paper_1709_03005_amd", "mlp_weights.npy")))
        ctx.set_mlp(net)
    pc = cc.CCH_PRECOND_MLP if args.precond == "mlp" else cc.CCH_PRECOND_JACOBI
    restart = {"auto": cc.CCH_RESTART_AUTO, "thick": cc.CCH_RESTART_THICK, "prev": cc.CCH_RESTART_PREV}[args.restart]

    def step():
        ctx.build()
        ev, _, info, rc = ctx.davidson(k, tol=tol, want_vectors=False, precond=pc, sparse_l2=args.sparse_l2,
                                       restart=restart)
        return ev, info, rc

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")
    builds, phases, dav_s, dav_it, mv_ms, mv_n, resid, rcs = [], [], [], [], [], [], [], []
    rr_ms, rr_fl, rr_n, rr_fb = [], [], [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ev, info, rc = step()
        bt, ph = ctx.build_time()
        builds.append(bt)
        phases.append(ph)
        dav_s.append(info.seconds)
        dav_it.append(info.iterations)
        mv_ms.append(info.matvec_ms)
        mv_n.append(info.matvec_launches)
        rr_ms.append(info.rr_ms)
        rr_fl.append(info.rr_flops)
        rr_n.append(info.rr_calls)
        rr_fb.append(info.rr_fallbacks)
        resid.append(info.max_residual)
        rcs.append(rc)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"{args.steps} timed steps in {wall:.2f} s")
    ms_step = wall / args.steps * 1e3
    build_ms = float(np.median(builds))
    ph = np.median(np.array(phases), axis=0)
    names = ["scan", "target_densities", "relayout", "expansion_gemm", "class4", "l2_block", "mirror_diag"]
    phase_ms = {n: float(v) for n, v in zip(names, ph[:7])}
    work = ctx.work_detail()
    ev_plain = np.array(ev)

    # roofline figures per kernel family (algorithmic work / measured device time)
    D = inst.dim()
    # dense H from D = 16384 on: the lower triangle read once per 16 vectors
    # (each element used for both of its products); below, the whole of H
    symmetric_mv = D >= 16384 and not args.sparse_l2
    mv_bytes = 4.0 * D * (D + 1.0) if symmetric_mv else 8.0 * D * D
    mv_avg_ms = float(np.sum(mv_ms) / max(np.sum(mv_n), 1))

    def entry(bound, work_units, ms, peak, unit, scale, total_ms=None, **extra):
        """work_units of algorithmic work done in ms of device time; total_ms:
        the kernel's device time per step when ms covers one launch"""
        achieved = work_units / max(ms * 1e-3, 1e-12) / scale
        return dict(bound=bound, achieved=achieved, peak=peak, unit=unit,
                    total_ms_per_step=ms if total_ms is None else total_ms, **extra)

    kernels = {
        "matvec": entry("hbm", mv_bytes, mv_avg_ms, HBM_PEAK_GBS, "GB/s", 1e9, total_ms=float(np.mean(mv_ms)),
                        avg_ms=mv_avg_ms, launches_per_step=float(np.mean(mv_n)),
                        note=("4 D (D + 1) bytes per launch (the lower triangle of H read once; the "
                              "product and its reduction of partial sums)") if symmetric_mv else
                        "8 D^2 bytes per launch (H read once)"),
        "expansion_gemm": entry("mfma", work["gemm_flops"], phase_ms["expansion_gemm"], FP64_MFMA_PEAK_TFLOPS,
                                "TFLOP/s", 1e12, note="2 x rows x cols x K per symmetry pair, FP64 MFMA"),
        "class4": entry("mfma", work["class4_flops"], phase_ms["class4"], FP64_MFMA_PEAK_TFLOPS, "TFLOP/s", 1e12,
                        note="2 S n_c flops per term of a connected L2 x target pair (Eq. 5), FP64 MFMA "
                             "(16 states x 16 continuum orbitals per tile); phase time includes its L2 x "
                             "target scan"),
        "densities": entry("alu", work["density_flops"], phase_ms["target_densities"], FP64_VALU_PEAK_TFLOPS,
                           "TFLOP/s", 1e12,
                           note="transition densities of Eq. 8 (one multiply-add per (n, n') row per density "
                                "update); the phase also holds the target pair values, the projection and "
                                "the bucket sort, so this is a lower bound of the density kernel's rate"),
        "l2_block": entry("hbm", 8.0 * work["l2_lower_elements"], phase_ms["l2_block"], HBM_PEAK_GBS, "GB/s",
                          1e9, note="8 B written per lower-triangle L2 element"),
        "relayout": entry("hbm", work["relayout_bytes"], phase_ms["relayout"], HBM_PEAK_GBS, "GB/s", 1e9),
        "mirror": entry("hbm", work["mirror_bytes"], phase_ms["mirror_diag"], HBM_PEAK_GBS, "GB/s", 1e9,
                        note="16 B per element above the diagonal; phase includes the diagonal copy"),
    }
    rr_avg_ms = float(np.sum(rr_ms) / max(np.sum(rr_n), 1))
    kernels["rayleigh_ritz"] = {
        "bound": "alu", "achieved": float(np.sum(rr_fl)) / max(float(np.sum(rr_ms)) * 1e-3, 1e-12) / 1e12,
        "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "avg_ms": rr_avg_ms,
        "launches_per_step": float(np.mean(rr_n)), "total_ms_per_step": float(np.mean(rr_ms)),
        "fallbacks_per_step": float(np.mean(rr_fb)),
        "note": "one workgroup per solve (m <= 96): latency-bound; flops = (10/3) m^3 per solve"}
    for name, v in kernels.items():
        v["frac"] = v["achieved"] / v["peak"]
        v["traffic"] = traffic_bytes(name, args.workload)
    dom = max(kernels, key=lambda n: kernels[n]["total_ms_per_step"])
    r = kernels[dom]
    roof = {"kernel": dom, "bound": r["bound"], "achieved": r["achieved"], "peak": r["peak"],
            "unit": r["unit"], "frac": r["frac"], "traffic": r["traffic"]}

    out = {
        "metric": METRIC,
        "value": lower / (ms_step * 1e-3),
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded generator: decaying random integrals, CISD-like determinant spaces, "
                "random orthonormal CI vectors)",
        "config": {"workload": args.workload, "dim": D, "n_cont_rows": inst.n_cont_rows(), "n_l2": inst.n_l2,
                   "n_target_orbitals": inst.n_o, "n_electrons": inst.n_elec,
                   "symmetries": len(inst.syms), "k": k, "tol": tol},
        "form": {"precision": args.precision, "precond": args.precond, "restart": args.restart,
                 "sparse_l2": bool(args.sparse_l2),
                 "sparse_build": bool(sparse_build), "device_bytes": ctx.plan_info()[0],
                 "target_energies": energies is not None,
                 "target_states": "target-Hamiltonian eigenvectors" if args.workload == "medium_te"
                 else ("random orthonormal, synthetic energies" if energies is not None else "random orthonormal")},
        "build_ms": build_ms,
        "build_elements_per_s": lower / (build_ms * 1e-3),
        "davidson_ms": float(np.median(dav_s)) * 1e3,
        # the solve's wall time above starts while the asynchronous build still runs
        "solve_ms_excluding_build": ms_step - build_ms,
        "davidson_iterations": int(np.median(dav_it)),
        "davidson_max_residual": float(np.max(resid)),
        "davidson_status": [int(x) for x in rcs],
        "lowest_eigenvalue": float(ev_plain[0]),
        "phase_ms": phase_ms,
        "kernels": kernels,
        "work": work,
        "plan_s": plan_s,
        "upload_s": upload_s,
        # whole job with the host -> HBM upload of the inputs counted once (not `value`)
        "pcie_inclusive_elements_per_s": lower / (upload_s + plan_s + ms_step * 1e-3),
        "roofline": roof,
    }
    sample = None
    if not args.no_cpu_baseline:
        out["cpu_baseline"], sample = cpu_baseline(inst, cpu_mode)

    def errors(c2):
        """Max-abs error of sampled elements against the oracle's values (read
        back with cch_get_elements, so large matrices need no host copy)."""
        if sample is None:
            return None
        rs, cs, vs = sample
        g = c2.get_elements(rs, cs)
        return {"max_abs_error_vs_oracle": float(np.abs(g - vs).max()), "elements": int(vs.size),
                "max_abs_oracle_element": float(np.abs(vs).max())}

    out["parity_sample"] = errors(ctx)
    forms = {}
    if not args.no_forms:
        reps = 3
        if args.workload in ("learned", "l2heavy", "precision", "medium") and not sparse_build:
            # the whole step with classes 2 and 8 built and stored sparse
            c2 = cc.from_instance(inst, device=0, stream=stream, sparse_l2=True)
            bt2, st2, it2 = [], [], []
            for rep in range(reps + 1):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                c2.build()
                ev2, _, inf2, rc2 = c2.davidson(k, tol=tol, want_vectors=False)
                torch.cuda.synchronize()
                if rep:
                    st2.append((time.perf_counter() - t0) * 1e3)
                    bt2.append(c2.build_time()[0])
                    it2.append(inf2.iterations)
            lw2 = c2.work_counts()["lower_elements"]
            forms["sparse_l2_build"] = {
                "ms_per_step": float(np.median(st2)), "build_ms": float(np.median(bt2)),
                "iterations": int(np.median(it2)), "status": int(rc2),
                "lower_elements": lw2, "elements_per_s": lw2 / (float(np.median(st2)) * 1e-3),
                "device_bytes": c2.plan_info()[0], "dense_device_bytes": ctx.plan_info()[0],
                "max_abs_eigenvalue_difference": float(np.abs(np.array(ev2) - ev_plain).max()),
                "element_error": errors(c2),
                "note": "classes 2 and 8 built and stored as CSR of the structural non-zeros (lower_elements "
                        "counts the dense parts and those non-zeros); the solve reads the panels and the CSR"}
            c2.close()
        if args.workload in ("learned", "l2heavy", "precision", "medium") and not sparse_build:
            ms_s, it_s, ev_s, rc_s, _ = _solve_stats(ctx, cc, k, tol, reps, sparse_l2=True)
            forms["sparse_l2_matvec"] = {"davidson_ms": ms_s, "iterations": it_s, "status": rc_s,
                                         "max_abs_eigenvalue_difference": float(np.abs(ev_s - ev_plain).max()),
                                         "note": "L2 block as CSR in the mat-vec (CSR formed in each solve "
                                                 "after a build: inside the first solve's time)"}
        if net is not None and args.precond != "mlp":
            ms_m, it_m, ev_m, rc_m, inf_m = _solve_stats(ctx, cc, k, tol, reps, precond=cc.CCH_PRECOND_MLP)
            ms_j, it_j, _, _, _ = _solve_stats(ctx, cc, k, tol, reps)
            forms["mlp_preconditioner"] = {
                "davidson_ms": ms_m, "iterations": it_m, "status": rc_m, "fallbacks": int(inf_m.fallbacks),
                "jacobi_ms": ms_j, "jacobi_iterations": it_j, "time_gain": ms_j / ms_m,
                "iteration_gain": it_j / max(it_m, 1),
                "max_abs_eigenvalue_difference": float(np.abs(ev_m - ev_plain).max())}
        if args.workload == "precision" and prec == cc.CCH_PREC_FP64:
            for name in ("fp32", "bf16x3", "bf16x7"):
                p2, s2 = _prec(name, cc)
                c2 = cc.from_instance(inst, device=0, stream=stream, precision=p2, split_slices=s2,
                                      target_energies=energies)
                bt2, gm2 = [], []
                for _ in range(reps + 1):
                    c2.build()
                    b2, ph2 = c2.build_time()
                    bt2.append(b2)
                    gm2.append(ph2[3])
                ms2, it2, ev2, rc2, _ = _solve_stats(c2, cc, k, tol, 1)
                diag = c2.get_diagonal()
                forms[name] = {"build_ms": float(np.median(bt2[1:])),
                               "expansion_ms": float(np.median(gm2[1:])),
                               "fp64_expansion_ms": phase_ms["expansion_gemm"],
                               "davidson_ms": ms2, "status": rc2,
                               "max_abs_eigenvalue_error_vs_fp64": float(np.abs(ev2 - ev_plain).max()),
                               "diagonal_nonzero": bool(np.abs(diag).max() > 0),
                               "element_error": errors(c2)}
                c2.close()
    out["chosen_forms"] = forms
    if net is not None:
        ctx.set_mlp(None)
        net.close()
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
