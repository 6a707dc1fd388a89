"""Benchmark: CI-contracted close-coupling Hamiltonian build + Davidson on one MI355X.

One step = the whole hot path on one batch of synthetic input, inputs already
resident in HBM: cch_build (excitation scans, target densities, relayout,
FP64 MFMA expansion, class 4, classes 2/8, mirror) followed by cch_davidson
(lowest k eigenpairs to residual tol, FP64). Default workload: the medium
configuration (30 target orbitals, N = 10, 4 symmetries x 500 dets x 5 states,
150 continuum orbitals per irrep, 5000 L2; D = 8000; lowest 10 to 1e-8).

Workloads: medium (default), tiny, small, precision (D = 40000), learned
(D = 60000; --precond mlp solves with the trained network and reports the
Jacobi solve of the same matrix beside it), batch (64 instances, batched vs
one after another).

Prints ONE JSON line. `value` = lower-triangle Hamiltonian elements per second
of the whole step (build + solve); the build-only rate and the
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

# HBM bytes per launch of the medium workload's kernels: rocprofv3 FETCH_SIZE
# and WRITE_SIZE passes (KiB per dispatch, averaged over one step), scaled by
# what the same counters read for a plain 512 MiB device copy (bench.py
# --workload copy: FETCH_SIZE reads half the bytes, WRITE_SIZE all of them).
# Keyed by the source file of the kernel and its hash when counted: a kernel
# changed since reports null.
COUNTER_SCALE = {"FETCH_SIZE": 2.0, "WRITE_SIZE": 1.0}
TRAFFIC = {
    # name: (source, sha256 prefix, FETCH_SIZE KiB, WRITE_SIZE KiB)
    "rayleigh_ritz": ("k_rr.hip", "ad413139aab2388c", 53.878, 25.493),
    "matvec": ("k_davidson.hip", "c2ad709cede732f3", 252272.643, 17904.762),
    "expansion_gemm": ("k_gemm.hip", "8cbf1a6f5665b209", 40280.400, 3533.656),
    "l2_block": ("k_l2.hip", "777ee4e8faee8121", 22100.938, 98766.094),
}


def traffic_bytes(kernel, workload):
    """Counter-measured HBM bytes per launch, or None."""
    import hashlib
    t = TRAFFIC.get(kernel)
    if t is None or workload != "medium":
        return None
    src = os.path.join(ROOT, "paper_1709_03005_amd", "csrc", t[0])
    if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != t[1]:
        return None
    return 1024.0 * (t[2] * COUNTER_SCALE["FETCH_SIZE"] + t[3] * COUNTER_SCALE["WRITE_SIZE"])


WORKLOADS = {
    # name: (generator, k, tol, CPU-baseline mode)
    "medium": ("medium", 10, 1e-8, "rows"),
    "tiny": ("tiny", 5, 1e-8, "rows"),
    "small": ("small", 10, 1e-8, "rows"),
    "precision": ("precision", 10, 1e-8, "elements"),
    "learned": ("learned_test", 10, 1e-8, "elements"),
    "l2heavy": ("l2heavy", 10, 1e-8, "elements"),   # D = 122815, dense matrix of 121 GB
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(inst, mode="rows", budget_s=20.0):
    """The CPU oracle, timed on a bounded sample of the same matrix.

    mode "rows": stratified groups of full rows, each group the rows of one
    continuum orbital (all states) per target symmetry plus L2 rows in the
    matrix's continuum : L2 proportion; elements/s over full rows (both
    triangles, as the oracle computes them).

    mode "elements": for matrices where one continuum row alone takes the
    oracle minutes (thousands of target determinants), the oracle's
    per-element path on a seeded sample of each block class of the lower
    triangle (continuum-continuum, L2-continuum, L2-L2); the per-class
    times per element are weighted by the class sizes into one rate for the
    whole lower triangle."""
    import numpy as np

    import oracle
    O = oracle.Oracle(inst)
    D = inst.dim()
    Dc = inst.n_cont_rows()
    rng = np.random.default_rng(7)
    if mode == "elements":
        counts = {"cont_cont": Dc * (Dc + 1) / 2, "l2_cont": float(inst.n_l2) * Dc,
                  "l2_l2": inst.n_l2 * (inst.n_l2 + 1) / 2}
        per_el, n_tot, t_tot = {}, 0, 0.0
        for cls, cnt in counts.items():
            if cnt == 0:
                continue
            n_s, t_c, n_c = 16, 0.0, 0
            while t_c < budget_s / 6 and n_c < (1 << 17):
                if cls == "cont_cont":
                    r = rng.integers(0, Dc, n_s); c = rng.integers(0, Dc, n_s)
                elif cls == "l2_cont":
                    r = rng.integers(Dc, D, n_s); c = rng.integers(0, Dc, n_s)
                else:
                    r = rng.integers(Dc, D, n_s); c = rng.integers(Dc, D, n_s)
                r, c = np.maximum(r, c), np.minimum(r, c)
                t = time.perf_counter()
                O.elements(r, c)
                t_c += time.perf_counter() - t
                n_c += n_s
                n_s *= 2
            per_el[cls] = t_c / n_c
            n_tot += n_c
            t_tot += t_c
            log(f"cpu baseline {cls}: {n_c} elements in {t_c:.1f} s")
        total = sum(counts.values())
        est = sum(counts[c] * per_el[c] for c in per_el)
        return {"value": total / est, "unit": "elements/s", "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"{n_tot} seeded lower-triangle elements of the same matrix, drawn per block class "
                          f"({', '.join(f'{c}: {per_el[c] * 1e6:.1f} us/element' for c in per_el)}), "
                          f"weighted by the class sizes; {t_tot:.1f} s of oracle time",
                "seconds": t_tot}
    groups = 0
    t_total = 0.0
    n_el = 0
    while t_total < budget_s * 0.5 and groups < 8:
        rows_c = []
        r0 = 0
        for s in inst.syms:
            nc = int(inst.n_c[s.irrep ^ inst.total_irrep])
            S = s.ci.shape[1]
            if nc:
                jj = int(rng.integers(nc))
                rows_c += [r0 + n * nc + jj for n in range(S)]
            r0 += S * nc
        n_l2_rows = max(1, int(round(len(rows_c) * inst.n_l2 / max(Dc, 1))))
        rows_l = list(Dc + rng.choice(inst.n_l2, size=min(n_l2_rows, inst.n_l2), replace=False))
        rows = np.array(rows_c + rows_l, dtype=np.int64)
        t = time.perf_counter()
        O.build_rows(rows)
        t_total += time.perf_counter() - t
        n_el += rows.size * D
        groups += 1
        log(f"cpu baseline group {groups}: {rows.size} rows, {t_total:.1f} s")
    return {"value": n_el / t_total, "unit": "elements/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{groups} stratified row groups of the same matrix ({n_el // D} full rows: one continuum "
                      f"orbital x all states per symmetry + L2 rows in proportion), {t_total:.1f} s",
            "seconds": t_total}


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
                   "total_lower_elements": lower},
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="medium", choices=sorted(WORKLOADS) + ["batch", "copy"],
                    help="copy: three plain 512 MiB device copies, the calibration run for HBM counters")
    ap.add_argument("--instances", type=int, default=64, help="batch workload: number of instances")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", default="fp64",
                    help="expansion GEMM form: fp64, fp32, or bf16xS (split-BF16 with S slices)")
    ap.add_argument("--precond", default="jacobi", choices=["jacobi", "mlp"],
                    help="Davidson correction: diagonal (Jacobi) or the trained network "
                         "(paper_1709_03005_amd/mlp_weights.npy)")
    ap.add_argument("--sparse-l2", action="store_true",
                    help="Davidson mat-vec with the L2 block as CSR of its non-zeros (formed in each solve)")
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
    if args.workload == "copy":
        n = 64 << 20
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"workload": "copy", "bytes_per_copy": n * 8, "copies": 3}))
        return None
    gen, k, tol, cpu_mode = WORKLOADS[args.workload]
    t_gen = time.perf_counter()
    inst = synth.CONFIGS[gen]()
    t_gen = time.perf_counter() - t_gen
    log(f"workload {args.workload}: D={inst.dim()} generated in {t_gen:.1f} s")

    torch.cuda.init()
    stream = torch.cuda.current_stream().cuda_stream
    if args.precision == "fp64":
        prec, slices = cc.CCH_PREC_FP64, 0
    elif args.precision == "fp32":
        prec, slices = cc.CCH_PREC_FP32, 0
    elif args.precision.startswith("bf16x"):
        prec, slices = cc.CCH_PREC_SPLIT_BF16, int(args.precision[5:])
    else:
        raise SystemExit(f"unknown --precision {args.precision}")
    t_up = time.perf_counter()
    ctx = cc.from_instance(inst, device=0, stream=stream, plan=False)   # inputs host -> HBM
    if args.target_energies:
        ctx.set_target_energies([-1.0 - 0.01 * np.arange(sym.ci.shape[1]) for sym in inst.syms])
    ctx.sync()
    upload_s = time.perf_counter() - t_up
    t = time.perf_counter()
    ctx.plan(precision=prec, split_slices=slices)
    ctx.sync()
    plan_s = time.perf_counter() - t
    log(f"planned in {plan_s:.1f} s")
    work = ctx.work_counts()
    lower = work["lower_elements"]
    net = None
    if args.precond == "mlp":
        net = cc.Mlp(device=0, stream=stream)
        net.set_weights(np.load(os.path.join(ROOT, "paper_1709_03005_amd", "mlp_weights.npy")))
        ctx.set_mlp(net)
    pc = cc.CCH_PRECOND_MLP if net is not None else cc.CCH_PRECOND_JACOBI

    def step():
        ctx.build()
        ev, _, info, rc = ctx.davidson(k, tol=tol, want_vectors=False, precond=pc, sparse_l2=args.sparse_l2)
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

    # roofline figures per kernel family (algorithmic work / measured device time)
    D = inst.dim()
    mv_bytes = 8.0 * D * D                               # H streamed once per launch
    mv_avg_ms = float(np.sum(mv_ms) / max(np.sum(mv_n), 1))
    kernels = {
        "matvec": {"bound": "hbm", "achieved": mv_bytes / (mv_avg_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                   "unit": "GB/s", "avg_ms": mv_avg_ms, "launches_per_step": float(np.mean(mv_n)),
                   "total_ms_per_step": float(np.mean(mv_ms))},
        "expansion_gemm": {"bound": "mfma",
                           "achieved": work["gemm_flops"] / (phase_ms["expansion_gemm"] * 1e-3) / 1e12,
                           "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "total_ms_per_step": phase_ms["expansion_gemm"]},
        "l2_block": {"bound": "hbm",
                     "achieved": 8.0 * work["l2_lower_elements"] / (phase_ms["l2_block"] * 1e-3) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "total_ms_per_step": phase_ms["l2_block"]},
        "relayout": {"bound": "hbm", "achieved": work["relayout_bytes"] / max(phase_ms["relayout"], 1e-9) / 1e6,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "total_ms_per_step": phase_ms["relayout"]},
    }
    rr_avg_ms = float(np.sum(rr_ms) / max(np.sum(rr_n), 1))
    kernels["rayleigh_ritz"] = {
        "bound": "alu", "achieved": float(np.sum(rr_fl)) / max(float(np.sum(rr_ms)) * 1e-3, 1e-12) / 1e12,
        "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "avg_ms": rr_avg_ms,
        "launches_per_step": float(np.mean(rr_n)), "total_ms_per_step": float(np.mean(rr_ms)),
        "fallbacks_per_step": float(np.mean(rr_fb)),
        "note": "one workgroup per solve (m <= 96): latency-bound; flops = (10/3) m^3 per solve"}
    for v in kernels.values():
        v["frac"] = v["achieved"] / v["peak"]
    dom = max(kernels, key=lambda n: kernels[n]["total_ms_per_step"])
    roof = dict(kernels[dom])
    for name, v in kernels.items():
        v["traffic"] = traffic_bytes(name, args.workload)
    roof = {"kernel": dom, "bound": roof["bound"], "achieved": roof["achieved"], "peak": roof["peak"],
            "unit": roof["unit"], "frac": roof["frac"], "traffic": kernels[dom]["traffic"]}

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
        "build_ms": build_ms,
        "build_elements_per_s": lower / (build_ms * 1e-3),
        "davidson_ms": float(np.median(dav_s)) * 1e3,
        "davidson_iterations": int(np.median(dav_it)),
        "davidson_max_residual": float(np.max(resid)),
        "davidson_status": [int(r) for r in rcs],
        "lowest_eigenvalue": float(ev[0]),
        "phase_ms": phase_ms,
        "kernels": kernels,
        "work": work,
        "plan_s": plan_s,
        "upload_s": upload_s,
        # whole job with the host -> HBM upload of the inputs counted once (not `value`)
        "pcie_inclusive_elements_per_s": lower / (upload_s + plan_s + ms_step * 1e-3),
        "roofline": roof,
    }
    if prec != cc.CCH_PREC_FP64:
        # error of this form against the FP64 build (itself checked against the oracle)
        G = ctx.get_matrix()
        ev_lo = np.array(ev)
        ref = cc.from_instance(inst, device=0, stream=stream)
        ref.build()
        H64 = ref.get_matrix()
        ev64, _, _, _ = ref.davidson(k, tol=tol, want_vectors=False)
        ref.close()
        out["precision_error"] = {
            "mode": args.precision,
            "max_abs_element_error": float(np.abs(G - H64).max()),
            "max_abs_element": float(np.abs(H64).max()),
            "max_abs_eigenvalue_error": float(np.abs(ev_lo - ev64).max()),
            "reference": "FP64 build of the same inputs (parity-checked against the oracle)",
        }
        del G, H64
    out["precision"] = args.precision
    out["target_energies"] = bool(args.target_energies)
    out["sparse_l2"] = bool(args.sparse_l2)
    out["precond"] = args.precond
    if net is not None:
        # the plain (Jacobi) solve of the same matrix, outside the timed region
        ev_j, _, inf_j, rc_j = ctx.davidson(k, tol=tol, want_vectors=False)
        out["precond_ab"] = {
            "mlp_ms": out["davidson_ms"], "mlp_iterations": out["davidson_iterations"],
            "mlp_fallbacks": int(info.fallbacks),
            "jacobi_ms": inf_j.seconds * 1e3, "jacobi_iterations": int(inf_j.iterations),
            "jacobi_status": int(rc_j),
            "time_gain": inf_j.seconds * 1e3 / out["davidson_ms"],
            "max_abs_eigenvalue_difference": float(np.abs(np.array(ev) - ev_j).max()),
        }
        ctx.set_mlp(None)
        net.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inst, cpu_mode)
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
