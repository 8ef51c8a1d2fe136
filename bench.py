#!/usr/bin/env python3
"""Benchmark: refined QTT-inverse solve on one MI355X.

Workload (one "step"): solve A sigma = F for K = 8 right-hand sides at L = 7
(N = 8^7 = 2,097,152), A of ranks [1,24,32,32,32,32,24,1], to relative
residual 1e-8 by iterative refinement with the compressed inverse:
sigma += Ainv r in BF16 (FP32 accumulation), r = F - A sigma in FP64.  The
compressed inverse (ranks <= 32) is computed in the untimed setup on the GPU
by Newton-Hotelling-Schulz from the first-order inverse of the seeded
operator pair.  The same refinement with Ainv applied in FP64 ("plain FP64")
is timed beside it, and the FP32 inverse as a third variant; the first-order
inverse is timed too, for comparison.  F is seeded N(0,1); everything is
resident in HBM before timing starts.

Prints ONE JSON line.  Extra keys beyond the driver contract: latency
percentiles, the plain-FP64 and FP32-inverse runs, the roofline of the
dominant kernel (the FP64 core pair of the residual apply) and of the BF16
core step, the flexible-GMRES solve, the operator with diagonals, the
compressed product, uneven batching, serving traces, the compressed "QTT
solve", and the CPU oracle baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 (matrix and vector)
PEAK_FP32_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
# the sources whose hash the committed HBM-traffic figures are tied to: every
# file the sweep's kernels and their launches are built from (the TT-format
# operations, qtt_tt*, are not part of a sweep)
def kernel_sources():
    import glob
    csrc = os.path.join(ROOT, "paper_1511_06029_amd", "csrc")
    files = glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.hpp"))
    return sorted(f for f in files if not os.path.basename(f).startswith("qtt_tt"))


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--tune", action="store_true",
                   help="run the tile autotuner first (default: the built-in shapes, which the "
                        "committed profiles measure)")
    p.add_argument("--no-tune", action="store_true", help=argparse.SUPPRESS)
    p.add_argument("--no-batched", action="store_true")
    p.add_argument("--no-compressed", action="store_true",
                   help="skip the compressed matrix-vector product timing")
    p.add_argument("--no-nti", action="store_true",
                   help="skip the timing of the operator with diagonals (a I + B K W C)")
    p.add_argument("--no-fgmres", action="store_true",
                   help="skip the flexible-GMRES solve of the same workload")
    p.add_argument("--no-serving", action="store_true",
                   help="skip the serving traces (BF16 and FP64 inverses, and the lower arrival rate)")
    p.add_argument("--serving-requests", type=int, default=32)
    p.add_argument("--no-tt", action="store_true",
                   help="skip the TT-format legs (compressed 'QTT solve' and Newton-Schulz inversion)")
    p.add_argument("--copy-probe", action="store_true",
                   help="only run a device copy of known size (HBM counter calibration)")
    p.add_argument("--first-order-inverse", action="store_true",
                   help="solve with the first-order inverse instead of the Newton-Schulz one")
    p.add_argument("--variants", default="mixed,sched,fp32s,bf16,fp64,fp32",
                   help="inverse dtypes to time (fp32s: FP32 cores, products from split BF16 "
                        "operands; sched: the BF16 copy in the first pass, fp32s after it; mixed: "
                        "sched, with the residual updated by A's split FP32 copy below 1e-5); "
                        "the first is the reported value")
    return p.parse_args()


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if xs else None


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 "
                                   "(the multi-GPU sharding is described, not built)"}))
        sys.exit(2)

    import torch
    from paper_1511_06029_amd import inputs as I
    from paper_1511_06029_amd import qtt as Q

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe:
        copy_probe(torch)
        return

    w = I.WORKLOADS["refine_L7"]
    L, ranks, K, rtol = w["L"], w["ranks"], w["K"], w["rtol"]
    N = 8 ** L
    Ac, Aic = I.perturbed_identity_pair(ranks, [8] * L, seed=w["core_seed"], eps=w["eps"])
    F_h = I.rhs(N, K, seed=w["rhs_seed"])
    variants = [v.strip() for v in args.variants.split(",") if v.strip()]

    A = Q.qtt_matrix_load(Ac, dtypes=("fp64",))
    scheduled = [v for v in variants if v in ("sched", "mixed")]
    inv_dtypes = tuple(sorted({DT(v) for v in variants} | {"fp64"} | ({"bf16"} if scheduled else set())))
    Ai0 = Q.qtt_matrix_load(Aic, dtypes=inv_dtypes)
    F = Q.to_block(F_h)
    # setup (untimed): the compressed inverse at the operator's ranks (<= 32),
    # computed on the GPU by Newton-Hotelling-Schulz from the first-order
    # inverse; the headline solves use it
    torch.cuda.synchronize()
    t_inv = time.perf_counter()
    if args.first_order_inverse:
        Ai, inv_info = Ai0, {"method": "first-order inverse (identity minus the perturbation)"}
    else:
        Ai, hist, ns_steps, _ = Q.qtt_invert_newton_schulz(A, Ai0, 1e-10, max_rank=32, max_iter=6, theta=0.1,
                                                           seed=5, dtypes=inv_dtypes, raise_on_cap=False)
        torch.cuda.synchronize()
        inv_info = {"method": "Newton-Hotelling-Schulz on the GPU from the first-order inverse, ranks held at "
                              "<= 32 (qtt_invert_newton_schulz, eps 1e-10, theta 0.1)",
                    "seconds": round(time.perf_counter() - t_inv, 2), "steps": ns_steps,
                    "residual_history": [float(f"{h:.3e}") for h in hist], "ranks": Ai.ranks}
    Aic = Q.qtt_matrix_cores(Ai)
    # each variant's inverse handle and compute dtype; fp32s is a second FP32
    # handle of the same inverse with the split-product configuration pinned on
    # its interior cores
    inv_h = {v: (Ai, v) for v in variants + ["fp64"]}
    if "fp32s" in variants or scheduled:
        Ais = Q.qtt_matrix_load(Aic, dtypes=("fp32",))
        Q.qtt_use_split_products(Ais)
        for v in ("fp32s", "sched", "mixed"):
            inv_h[v] = (Ais, "fp32")       # sched, mixed: their later passes (the first applies Ai's BF16 copy)
    # mixed: A's own split-product FP32 copy updates the residual (r -= A dx)
    # in the passes that start below 1e-5 of ||F|| (about 2e-11 of ||F|| off
    # the true residual at that size; the true residuals are recomputed in
    # FP64 after the timed solves)
    As = None
    if "mixed" in variants:
        As = Q.qtt_matrix_load(Ac, dtypes=("fp32",))
        Q.qtt_use_split_products(As)

    def schedule(v):
        if v == "sched":
            return dict(first=Ai, first_compute="bf16", first_passes=1)
        if v == "mixed":
            return dict(first=Ai, first_compute="bf16", first_passes=1, A_lo=As, lo_compute="fp32", lo_below=1e-5)
        return {}

    Sig = Q.empty_block(N, K)
    ws_bytes = max(Q.qtt_solve_schedule_workspace_bytes(A, inv_h[v][0], inv_h[v][1], K, **schedule(v))
                   for v in variants)
    ws = Q.workspace(ws_bytes)
    stream = torch.cuda.current_stream()

    # setup (untimed): tile autotuning for the shapes of the sweep
    if args.tune and not args.no_tune:
        Yt = Q.empty_block(N, K)
        aws = Q.workspace(max(Q.qtt_workspace_bytes(A, "fp64", K),
                              *[Q.qtt_workspace_bytes(Ai, DT(v), K) for v in variants]))
        Q.qtt_autotune(A, "fp64", F, Yt, aws)
        for v in variants:
            if v not in ("fp32s", "sched", "mixed"):          # pinned configuration: not tuned
                Q.qtt_autotune(Ai, v, F, Yt, aws)
        del Yt, aws
        torch.cuda.synchronize()

    def solver(v):
        """One refined solve of variant v (sched: the inverse's BF16 copy in the
        first pass, the split-product FP32 copy after it; mixed: sched with the
        late residual updates by A's split-product copy)."""
        Ah, dv = inv_h[v]
        if v in ("sched", "mixed"):
            sc = schedule(v)
            return lambda: Q.qtt_solve_schedule(A, Ah, dv, F, Sig, rtol=rtol, ws=ws, stream=stream, **sc)
        return lambda: Q.qtt_solve(A, Ah, dv, F, Sig, rtol=rtol, ws=ws, stream=stream)

    results = {}
    for v in variants:
        Ah, dv = inv_h[v]
        solve = solver(v)
        for _ in range(args.warmup):
            solve()
        torch.cuda.synchronize()
        # the timed solves replay each sweep from its captured graph (one
        # hipGraphLaunch per sweep); no per-launch events in this region
        lat = []
        infos = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            s0 = time.perf_counter()
            _, info, _ = solve()
            lat.append((time.perf_counter() - s0) * 1e3)
            infos.append(info)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        timing = (v == variants[0])
        if timing:
            # kernel figures for the roofline: a separate run of the same solve
            # with HIP events around every launch (direct launches, no graphs)
            Q.qtt_timing_reset()
            Q.qtt_timing_enable(True)
            for _ in range(max(2, min(args.steps, 8))):
                solve()
            torch.cuda.synchronize()
            Q.qtt_timing_enable(False)
            kt = {(dt, pos): Q.qtt_timing_read(dt, pos) for dt in ("fp64", dv) for pos in (0, 1, 2)}
            ks = {(dt, sh): Q.qtt_timing_read_shape(dt, sh)
                  for dt in ("fp64", dv)
                  for sh in Q.qtt_list_shapes(dt) + Q.PAIR_SHAPES + ([Q.F32_SPLIT] if dt == "fp32" else [])}
            Q.qtt_timing_reset()
        elapsed = t1 - t0
        if v == variants[0]:
            sigma0 = Sig[:, 0].cpu().numpy().copy()   # the headline solve's first solution
        iters = max(c[0] for c in infos[-1])
        worst = max(c[1] for inf in infos for c in inf)
        # untimed: the last solve's true residuals, A applied in FP64
        Rt = F - Q.qtt_apply(A, "fp64", Sig)
        true = float((torch.linalg.vector_norm(Rt, dim=0) / torch.linalg.vector_norm(F, dim=0)).max())
        del Rt
        results[v] = {"rhs_per_s": K * args.steps / elapsed, "ms_per_step": 1e3 * elapsed / args.steps,
                      "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
                      "passes": iters, "max_rel_residual": worst, "max_rel_residual_true": true}
        if timing:
            results[v]["kernels"] = kt
            results[v]["shapes"] = ks

    head = variants[0]
    r0 = results[head]

    # continuity: the same solves with the first-order inverse (the previous
    # headline inverse), fewer steps
    first_order = None
    if not args.first_order_inverse:
        first_order = {}
        for v in ("bf16", "fp64"):
            if v not in inv_dtypes:
                continue
            for _ in range(2):
                Q.qtt_solve(A, Ai0, v, F, Sig, rtol=rtol, ws=ws, stream=stream)
            torch.cuda.synchronize()
            n_fo = max(3, args.steps // 4)
            t0 = time.perf_counter()
            for _ in range(n_fo):
                _, info, _ = Q.qtt_solve(A, Ai0, v, F, Sig, rtol=rtol, ws=ws, stream=stream)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / n_fo
            first_order[v] = {"rhs_per_s": round(K / dt, 3), "passes": max(c[0] for c in info),
                              "max_rel_residual": max(c[1] for c in info)}

    def dominant(dt):
        """The kernel configuration that carries the most flops of dtype dt."""
        cand = [(r["flops"], sh, r) for (d, sh), r in r0["shapes"].items() if d == dt and r["launches"]]
        return max(cand, key=lambda c: c[0])[1:] if cand else (None, None)

    sh64, f64 = dominant("fp64")
    traffic, kname = measured_traffic("fp64", sh64)
    roof = None
    if f64 is not None:
        avg_ms = f64["ms"] / f64["launches"]
        per_launch_flops = f64["flops"] / f64["launches"]
        achieved = per_launch_flops / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                "traffic": (None if (traffic is None or args.tune) else traffic),
                "kernel": (f"FP64 core step, configuration {sh64}" + (f" ({kname})" if kname else "")
                           + ", the one carrying most of the FP64 residual apply's flops"),
                "launches": f64["launches"], "avg_launch_ms": round(avg_ms, 4),
                "flops_per_launch": per_launch_flops,
                "achieved_hbm_GBs": round(f64["bytes"] / f64["ms"] * 1e-6, 1)}
    roof_lo = None
    if head != "fp64":
        shlo, lo = dominant(DT(head))
        if lo is not None:
            gbs = lo["bytes"] / lo["ms"] * 1e-6
            tfs = lo["flops"] / lo["ms"] * 1e-9
            tlo, klo = measured_traffic(DT(head), shlo)
            roof_lo = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                       "frac": round(gbs / PEAK_HBM_GBS, 4), "tflops": round(tfs, 2),
                       # mixed: the configuration's launches include those of
                       # A's split copy, while the counters cover the inverse's
                       "traffic": (None if (tlo is None or args.tune or head == "mixed") else tlo),
                       "kernel": (f"{'fp32s' if head in ('sched', 'mixed') else head} core step, configuration {shlo}"
                                  + (f" ({klo})" if klo else "")
                                  + (", the one carrying most of the split-product applies' flops (the inverse's "
                                     "and, in the late residual updates, A's)" if head == "mixed" else
                                     ", the one carrying most of the inverse apply's flops")),
                       "launches": lo["launches"], "avg_launch_ms": round(lo["ms"] / lo["launches"], 4)}

    fg = None if args.no_fgmres else fgmres_run(Q, torch, A, inv_h[head][0], inv_h[head][1], F, K, N, rtol, args,
                                                label=head, sched=schedule(head))

    nti = None if args.no_nti else nti_run(Q, torch, Ac, F, K, N)
    cmv = None if args.no_compressed else compressed_run(Q, torch, Ac)

    batched = None if args.no_batched else batched_run(Q, torch)

    serving = None if args.no_serving else serving_run(Q, torch, args.serving_requests)
    qtt_solve_c = None if args.no_tt else qtt_solve_compressed_run(Q, torch, Aic)
    ns = inv_info

    cpu = None
    if not args.no_cpu_baseline:
        # one standalone inverse apply of the first right-hand side per dtype
        inv_applies = {}
        f0 = F[:, :1].contiguous()
        for v in sorted(set(variants) | {"fp64"}):
            inv_applies[v] = Q.qtt_apply(inv_h[v][0], inv_h[v][1], f0)[:, 0].cpu().numpy().copy()
        cpu = cpu_baseline(Ac, Aic, F_h[:, :1], r0["passes"], sigma0, head, inv_applies)

    line = {
        "metric": "QTT-inverse RHS/s at 1e-8 rel residual (refined solve), L=7 r=32, vs plain FP64",
        "value": round(r0["rhs_per_s"], 3),
        "unit": "RHS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r0["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("bf16,fp32s" if head in ("sched", "mixed") else head) + "+f64",
        "data": "synthetic",
        "config": {"workload": "refine_L7: refined QTT-inverse solve, L=7 (N=2097152), mode 8x8, "
                               "A ranks [1,24,32,32,32,32,24,1], inverse ranks <= 32 (computed on the GPU), "
                               "K=8 RHS per step, rtol 1e-8",
                   "inverse_dtype": head, "inverse_arithmetic": INV_ARITH.get(head, head),
                   "residual_dtype": ("fp64; below 1e-5 ||F||: updated with A's split-product FP32 copy, "
                                      "FP64 accumulation" if head == "mixed" else "fp64"), "rhs_per_step": K,
                   "N": N, "L": L, "ranks": ranks},
        "latency_ms": {"p50": round(r0["p50_ms"], 3), "p99": round(r0["p99_ms"], 3)},
        "launch_path": "timed solves replay each sweep from its captured hipGraph; the roofline "
                       "figures come from a separate run with HIP events around every launch",
        "passes": r0["passes"],
        "max_rel_residual": r0["max_rel_residual"],
        "max_rel_residual_true": r0["max_rel_residual_true"],
        # the value stands only if every column of the reported solve meets
        # rtol by its true residual (A applied in FP64 to the returned sigma)
        "true_residual_meets_rtol": bool(r0["max_rel_residual_true"] <= rtol),
        "variants": {v: {k: (float(f"{x:.5g}") if isinstance(x, float) else x) for k, x in r.items()
                         if k not in ("kernels", "shapes")}
                     for v, r in results.items()},
        "speedup_vs_plain_fp64": (round(r0["rhs_per_s"] / results["fp64"]["rhs_per_s"], 3)
                                  if "fp64" in results and head != "fp64" else None),
        "roofline": roof,
        "roofline_inverse": roof_lo,
        "fgmres": fg,
        "nti_apply_L7": nti,
        "compressed_matvec_L7": cmv,
        "batched_uneven_L7": batched,
        "serving": serving,
        "qtt_solve_compressed_L7": qtt_solve_c,
        "inverse": ns,
        "first_order_inverse": first_order,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    A.free()
    Ai.free()
    if Ai is not Ai0:
        Ai0.free()


def compressed_run(Q, torch, Ac, nvec=64, rank=8, reps=20):
    """The compressed matrix-vector product (section 4.2) of the L=7 operator
    with a batch of TT vectors of rank 8: vectors/s and HBM rate (algorithmic
    bytes = input and output cores plus the operator's cores, per call)."""
    from paper_1511_06029_amd import inputs as I
    d = len(Ac)
    rb = [1] + [rank] * (d - 1) + [1]
    g = I.rng(77)
    B = [torch.from_numpy(g.standard_normal((nvec, rb[k], 8, rb[k + 1]))).cuda() for k in range(d)]
    A = Q.qtt_matrix_load(Ac, dtypes=("fp64",))
    C = Q.qtt_matvec_compressed(A, B)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        Q.qtt_matvec_compressed(A, B, C)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = sum(x.numel() for x in B) * 8 + sum(x.numel() for x in C) * 8 + sum(G.size for G in Ac) * 8
    A.free()
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"vectors": nvec, "vector_rank": rank, "ms_per_call": round(ms, 4),
            "vectors_per_s": round(nvec / (ms * 1e-3), 1), "bytes_per_call": nbytes,
            "achieved_GBs": round(gbs, 1), "frac_of_hbm_peak": round(gbs / PEAK_HBM_GBS, 4),
            "config": "L=7 operator, ranks [1,24,32,32,32,32,24,1]; TT vectors of rank 8; FP64"}


def nti_run(Q, torch, Ac, F, K, N, reps=10):
    """FP64 apply of the L=7 operator as K alone and as a I + B K W C (the
    non-translation-invariant form of section 3, diagonals as elementwise
    passes around the sweep): the cost of the diagonals."""
    from paper_1511_06029_amd import inputs as I
    g = I.rng(2024)
    b, wc = 1.0 + g.random(N), 1.0 + g.random(N)
    A = Q.qtt_matrix_load(Ac, dtypes=("fp64",))
    out = {}
    for name, diag in (("plain_ms", None), ("nti_ms", (1.0, b, wc))):
        if diag:
            Q.qtt_matrix_set_diagonals(A, *diag)
        ws = Q.workspace(Q.qtt_workspace_bytes(A, "fp64", K))
        Y = Q.empty_block(N, K)
        for _ in range(2):
            Q.qtt_apply(A, "fp64", F, Y, ws=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            Q.qtt_apply(A, "fp64", F, Y, ws=ws)
        torch.cuda.synchronize()
        out[name] = round(1e3 * (time.perf_counter() - t0) / reps, 3)
        del ws, Y
    A.free()
    out["overhead"] = round(out["nti_ms"] / out["plain_ms"] - 1.0, 4)
    out["config"] = "L=7, ranks [1,24,32,32,32,32,24,1], K=8 vectors, FP64, a=1, b and wc in [1,2)"
    return out


def fgmres_run(Q, torch, A, Ai, inv, F, K, N, rtol, args, max_iter=12, label=None, sched=None):
    """The same solve by flexible GMRES (the compressed inverse as right
    preconditioner, section 5.3's outer solver): RHS/s, steps, and the true
    relative residual recomputed by an FP64 apply outside the timed region.
    sched: the schedule of qtt_solve_fgmres_schedule (first steps'
    preconditioner, w = A_lo z_j below lo_below), or None."""
    sc = sched or {}
    ws = Q.workspace(Q.qtt_fgmres_schedule_workspace_bytes(A, Ai, inv, K, max_iter, **sc))
    Sig = Q.empty_block(N, K)
    stream = torch.cuda.current_stream()

    def solve():
        return Q.qtt_solve_fgmres_schedule(A, Ai, inv, F, Sig, rtol=rtol, max_iter=max_iter, ws=ws, stream=stream,
                                           **sc)
    for _ in range(max(args.warmup, 1)):
        solve()
    torch.cuda.synchronize()
    lat, info = [], None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        _, info, _ = solve()
        lat.append((time.perf_counter() - s0) * 1e3)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    del ws
    AS = Q.qtt_apply(A, "fp64", Sig)
    true = ((F - AS).norm(dim=0) / F.norm(dim=0)).max().item()
    return {"inverse_dtype": label or inv, "rhs_per_s": round(K * args.steps / el, 3),
            "ms_per_step": round(1e3 * el / args.steps, 3),
            "p50_ms": round(percentile(lat, 50), 3), "p99_ms": round(percentile(lat, 99), 3),
            "steps": max(c[0] for c in info), "max_rel_residual_estimate": max(c[1] for c in info),
            "max_rel_residual_true": true}


INV_ARITH = {
    "fp32s": "FP32 cores and intermediates; each FP32 product formed from split BF16 operands "
             "(hi + lo, three BF16 matrix instructions), FP32 accumulation",
    "sched": "first pass: the inverse's BF16 copy (BF16 cores and intermediates, FP32 accumulation); "
             "later passes: its FP32 copy with split-BF16 products (as fp32s)",
    "mixed": "the inverse as in sched; residual r = F - A sigma in FP64 in the passes that start above "
             "1e-5 ||F||, r -= A dx with A's split-product FP32 copy (FP64 update) in the others",
    "fp32": "FP32 cores and intermediates, FP32 matrix instructions",
    "bf16": "BF16 cores and intermediates, FP32 accumulation",
    "fp64": "FP64 throughout",
}


def DT(variant):
    """Compute dtype of a solve variant's main inverse: fp32s (and sched and
    mixed after their first pass) is FP32 with split-operand products."""
    return "fp32" if variant in ("fp32s", "sched", "mixed") else variant


def measured_traffic(dtype, shape):
    """(HBM bytes per launch, kernel name) of configuration `shape` of `dtype`
    from the committed PMC summary (profiles/hbm_traffic_refine_L7.json:
    FETCH_SIZE and WRITE_SIZE scaled by the copy calibration).  The bytes are
    None when the library sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_refine_L7.json")
    h = hashlib.sha256()
    for f in kernel_sources():
        h.update(open(f, "rb").read())
    try:
        rec = json.load(open(path))
        b = rec["bytes_per_launch"][f"{dtype} shape {shape}"]
    except (OSError, KeyError, ValueError):
        return None, None
    if rec.get("sources_sha256") != h.hexdigest():
        return None, b.get("kernel")
    return round(b["fetch"] + b["write"]), b.get("kernel")


def copy_probe(torch):
    """A plain device copy of 1 GiB, five times: reads 1 GiB and writes 1 GiB
    per launch.  Its HBM counters calibrate those of the core-step kernels."""
    n = 2 ** 30 // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(5):
        y.copy_(x)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / 5
    print(json.dumps({"copy_bytes_each_way": 2 ** 30, "launches": 5, "ms_per_copy": round(ms, 4),
                      "GBs_read_plus_write": round(2 * 2 ** 30 / ms * 1e-6, 1)}), flush=True)


def sweep_flops(ranks, m, n):
    """Flops of one sweep for one vector: core k multiplies an (r_k m_k) x
    (r_{k-1} n_k) matrix by prod_{l<k} m_l prod_{l>k} n_l columns."""
    total = 0
    for k in range(len(m)):
        cols = int(np.prod(m[:k], dtype=np.int64) * np.prod(n[k + 1:], dtype=np.int64))
        total += 2 * ranks[k + 1] * m[k] * ranks[k] * n[k] * cols
    return total


def batched_run(Q, torch):
    """Uneven batching: 64 blocks of widths drawn from {1,2,4,8,16,32} applied
    to the L=7 operator in FP32 by one qtt_apply_batched call per repetition
    (each core is one persistent launch per workspace wave, replayed from a
    graph).  Tiles come from the autotuner, run first on this workload's
    vector count (its choices are keyed by core shape, so a vector's kernels,
    and its bits, do not depend on the batch it is part of)."""
    from paper_1511_06029_amd import inputs as I
    w = I.WORKLOADS["batched_L7"]
    Ac, _ = I.perturbed_identity_pair(w["ranks"], [8] * 7, seed=w["core_seed"])
    widths = I.uneven_widths(w["nblocks"], seed=w["width_seed"])
    A = Q.qtt_matrix_load(Ac, dtypes=("fp32",))
    N = 8 ** 7
    g = torch.Generator(device="cuda").manual_seed(w["rhs_seed"])
    Xs = [torch.randn((k, N), generator=g, device="cuda", dtype=torch.float64).t() for k in widths]
    Ys = [Q.empty_block(N, k) for k in widths]
    total = sum(widths)
    ws_bytes = min(Q.qtt_workspace_bytes(A, "fp32", total), 96 * 2 ** 30)
    ws = Q.workspace(ws_bytes)
    t_tune = time.perf_counter()
    tw = max(widths)
    Q.qtt_autotune(A, "fp32", Xs[int(np.argmax(widths))], Ys[int(np.argmax(widths))],
                   Q.workspace(Q.qtt_workspace_bytes(A, "fp32", tw)))
    t_tune = time.perf_counter() - t_tune
    for _ in range(2):
        Q.qtt_apply_batched(A, "fp32", Xs, Ys, ws=ws)
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        Q.qtt_apply_batched(A, "fp32", Xs, Ys, ws=ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    # launches per core position in one call (timing on: direct launches)
    Q.qtt_timing_reset()
    Q.qtt_timing_enable(True)
    Q.qtt_apply_batched(A, "fp32", Xs, Ys, ws=ws)
    torch.cuda.synchronize()
    Q.qtt_timing_enable(False)
    launches = {name: Q.qtt_timing_read("fp32", pos)["launches"]
                for name, pos in (("first_core", 1), ("interior", 0), ("last_core", 2))}
    Q.qtt_timing_reset()
    flops = sweep_flops(w["ranks"], [8] * 7, [8] * 7) * total
    A.free()
    return {"blocks": len(widths), "rhs": total, "ms_per_call": round(dt * 1e3, 2),
            "rhs_per_s": round(total / dt, 1), "tflops": round(flops / dt / 1e12, 2),
            "workspace_gb": round(ws_bytes / 2 ** 30, 1), "dtype": "fp32",
            "launches_per_call": launches,
            "launch_path": "each core one persistent launch per workspace wave, segment table in device "
                           "memory; the sweep of each wave replayed from its captured hipGraph",
            "autotune_s": round(t_tune, 1)}


def serving_run(Q, torch, n_requests):
    """The serving workload: 12 resident operators (L in {5,6,7,8}, ranks 16-32),
    a seeded Poisson trace at 200 requests/s with 1-16 vectors each, a 200 GB
    arena, three slots.  Run with the BF16 inverse (FP64 residuals), with
    the BF16 inverse and the late residual updates by an FP32 copy of A
    (columns that start a pass below 1e-4 of their right-hand side), and
    with the FP64 inverse (plain FP64), same operators and trace; then the
    BF16 server again at about 70% of its measured capacity (the knee)."""
    from paper_1511_06029_amd import serving as SV
    torch.cuda.empty_cache()      # the arena takes 200 GB: return the earlier legs' cached blocks
    ops, descs = SV.serving_operators()
    out = {"operators": [{"L": d["L"], "r": d["ranks"][1]} for d in descs], "requests": n_requests,
           "slots": 3, "budget_gb": 200}
    for key, inv, kw in (("bf16_inverse_200_per_s", "bf16", {}),
                         ("bf16_inverse_fp32_residual_updates_200_per_s", "bf16",
                          dict(residual_lo="fp32", lo_below=1e-4)),
                         ("fp64_inverse_200_per_s", "fp64", {})):
        srv = SV.SolveServer(ops, inv_dtype=inv, budget_bytes=200 * 10 ** 9, n_slots=3, **kw)
        st = SV.serving_trace(srv, descs, n_requests, 200.0, seed=51)
        srv.close()
        del srv
        torch.cuda.empty_cache()
        out[key] = _round_stats(st)
    b, f = out["bf16_inverse_200_per_s"], out["fp64_inverse_200_per_s"]
    out["served_speedup_vs_plain_fp64"] = round(b["rhs_per_s"] / f["rhs_per_s"], 3)
    out["served_speedup_with_residual_updates"] = round(
        out["bf16_inverse_fp32_residual_updates_200_per_s"]["rhs_per_s"] / f["rhs_per_s"], 3)
    # knee: about 70% of the saturated BF16 capacity, in requests per second
    mean_k = 8.5
    rate = round(0.7 * b["rhs_per_s"] / mean_k, 2)
    srv = SV.SolveServer(ops, inv_dtype="bf16", budget_bytes=200 * 10 ** 9, n_slots=3)
    st = SV.serving_trace(srv, descs, max(8, n_requests // 2), rate, seed=52)
    srv.close()
    del srv
    torch.cuda.empty_cache()
    out["bf16_inverse_knee"] = dict(_round_stats(st), rate_per_s=rate)
    return out


def qtt_solve_compressed_run(Q, torch, Aic, eps=1e-4, eps_round=1e-3, reps=3):
    """The "QTT solve" of section 5.2 at L=7 on the GPU: compress the right-hand
    side f = phi(x) phi(y) phi(z), phi(t) = diric(2 pi t, 10), into TT form,
    take the compressed product with the compressed inverse (ranks multiply),
    round the product; each step timed (median of reps), and the result
    compared with the full-vector apply of the inverse to f."""
    L = 7
    N = 8 ** L
    side = 1 << L
    # f on the cell centres in octree order (octant digit 4z + 2y + x per level)
    idx = np.arange(N, dtype=np.int64)
    coord = [np.zeros(N, dtype=np.int64) for _ in range(3)]
    for k in range(L):
        dig = (idx >> (3 * k)) & 7
        for a in range(3):
            coord[a] |= ((dig >> a) & 1) << k
    t = 2 * np.pi * (np.stack(coord, axis=1) + 0.5) / side
    with np.errstate(divide="ignore", invalid="ignore"):
        phi = np.sin(10 * t / 2) / (10 * np.sin(t / 2))     # no cell centre hits t = 2 pi k
    f = torch.from_numpy(np.ascontiguousarray(phi[:, 0] * phi[:, 1] * phi[:, 2])).cuda()
    Ai = Q.qtt_matrix_load(Aic, dtypes=("fp64",))
    times = {"compress_ms": [], "product_ms": [], "round_ms": []}
    out = None
    for rep in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fc, fr, _ = Q.qtt_tt_compress(f, [8] * L, eps, seed=3)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        C = Q.qtt_matvec_compressed(Ai, [G[None].contiguous() for G in fc])
        prod = [Cc[0].contiguous() for Cc in C]
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        cores, ranks, st = Q.qtt_tt_round(prod, eps_round, seed=4, raise_on_cap=False)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        if rep > 0:
            times["compress_ms"].append((t1 - t0) * 1e3)
            times["product_ms"].append((t2 - t1) * 1e3)
            times["round_ms"].append((t3 - t2) * 1e3)
        out = (fr, [1] + [int(P.shape[2]) for P in prod], ranks, st, cores)
    fr, pr, ranks, st, cores = out
    # expand the rounded TT on the device and compare with Ainv f (full-vector sweep)
    v = cores[0].reshape(8, -1)
    for G in cores[1:]:
        v = (v @ G.reshape(G.shape[0], -1)).reshape(-1, G.shape[2])
    v = v.reshape(-1)
    # the expansion's index is i_1 fastest only after reordering: v was built
    # with i_1 slowest, so reverse the digit order
    v = v.reshape([8] * L).permute(*reversed(range(L))).reshape(-1)
    y = Q.qtt_apply(Ai, "fp64", f.reshape(N, 1))[:, 0]
    err = float((v - y).norm() / y.norm())
    Ai.free()
    med = {k: round(float(np.median(x)), 2) for k, x in times.items()}
    return {"eps_compress": eps, "eps_round": eps_round, "rhs_ranks": fr, "product_ranks": pr, "rounded_ranks": ranks,
            "rank_cap_reached": st == 9, **med,
            "total_ms": round(sum(med.values()), 2),
            "rel_error_vs_full_apply": err,
            "config": "L=7 (N=2097152), diric RHS (section 5.2), inverse ranks [1,24,32,32,32,32,24,1]; "
                      "compress (eps_compress), compressed product, round (eps_round)"}


def _round_stats(st):
    keep = ("requests", "rhs", "wall_s", "rhs_per_s", "p50_ms", "p99_ms", "batches", "all_converged",
            "iters_max", "max_rel_residual", "max_rel_residual_recomputed", "latency_by_L_ms")
    r = {}
    for k in keep:
        v = st.get(k)
        r[k] = float(f"{v:.5g}") if isinstance(v, float) else v
    return r


def cpu_baseline(Ac, Aic, f, passes, sigma0, head, gpu_inv_applies):
    """The FP64 oracle on a bounded sample of the workload: one refined solve
    of one right-hand side (x += Ainv r, r = f - A x), each pass timed on its
    own; the median pass time times the passes the GPU solve needs gives
    seconds per right-hand side.  The same leg checks the headline solve's
    first solution (its FP64 residual by the oracle's A apply) and reports the
    standalone error of the GPU's compressed-inverse apply in each dtype
    against the oracle's (the first pass is exactly Ainv f)."""
    from oracle import qtt_oracle as O
    threads = None
    try:
        from threadpoolctl import threadpool_info
        threads = max((p.get("num_threads", 0) for p in threadpool_info()), default=None)
    except Exception:
        pass
    f0 = f[:, 0]
    x = np.zeros_like(f0)
    r = f0.copy()
    times = []
    first = None
    # at least 5 timed passes: past the GPU solve's pass count the refinement
    # simply continues (each pass costs the same)
    for t in range(max(passes, 5)):
        t0 = time.perf_counter()
        dx = O.qtt_apply_alg2(Aic, r)
        x = x + dx
        r = f0 - O.qtt_apply_alg2(Ac, x)
        times.append(time.perf_counter() - t0)
        if first is None:
            first = dx
    med = float(np.median(times))
    per_rhs = med * passes
    res = f0 - O.qtt_apply_alg2(Ac, sigma0)
    oracle_rel = float(np.linalg.norm(res) / np.linalg.norm(f0))
    apply_error = {}
    for dt, y in gpu_inv_applies.items():
        e = y - first
        apply_error[dt] = {"normwise": float(np.linalg.norm(e) / np.linalg.norm(first)),
                           "max_abs_over_max_ref": float(np.abs(e).max() / np.abs(first).max())}
    # the direct solve's own error (one FP64 inverse apply, sigma_0 = Ainv f),
    # against the refined solution: about the inverse's contraction rho
    direct = float(np.linalg.norm(first - sigma0) / np.linalg.norm(sigma0))
    return {"value": round(1.0 / per_rhs, 6), "unit": "RHS/s", "cores": threads or os.cpu_count(),
            "kind": "oracle",
            "sample": f"a refined solve of 1 RHS at L=7 by the numpy FP64 oracle, {len(times)} passes "
                      f"(Ainv apply + A apply) each timed: median {med:.2f} s over {len(times)} runs "
                      f"(min {min(times):.2f}, max {max(times):.2f}); x {passes} passes (the GPU solve's count)",
            "host_cpus": os.cpu_count(),
            "oracle_check": {"rhs": 0, "inverse_dtype": head, "rel_residual": oracle_rel,
                             "what": "||f - A sigma|| / ||f|| of the GPU solution, A applied by the FP64 oracle"},
            "apply_error": {"inverse_apply_vs_oracle": apply_error,
                            "direct_solve_error_fp64": direct,
                            "what": "error of one GPU Ainv apply (per dtype) against the oracle's FP64 Ainv "
                                    "apply of the same vector; direct_solve_error_fp64 = "
                                    "||Ainv f - sigma|| / ||sigma|| (one FP64 apply, no refinement)"}}


if __name__ == "__main__":
    main()
