#!/usr/bin/env python3
"""Throughput of the bbFMM matvec phi = K sigma on one MI355X.

Workload (the configuration the headline metric is quoted on): N = 2^20
points uniform in the unit cube, kernel 1/r, Chebyshev order 5, 6 levels,
one right-hand side, SVD tolerance 1e-5, FP32 path.  Inputs are seeded
synthetic data (the paper's experiments use uniform random clouds).

One step = one full matvec through the C ABI (gather, P2M, M2M, M2L,
decompression + L2L, L2P + P2P, scatter) on inputs already resident in HBM.
Prints one JSON line: throughput in points x RHS per second, per-step
latency percentiles, per-stage device time from HIP events recorded inside
the timed steps, the roofline of the dominant kernel, and the FP64 oracle
timed on the host cores on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "bbFMM matvec points x RHS/sec at rel err 1e-5 vs plain FP32; p99 latency"
PEAK_FP32_MFMA_TFLOPS = 157.3     # MI355X dense FP32 matrix
PEAK_FP32_VECTOR_TFLOPS = 157.3   # MI355X FP32 vector (counts packed FP32)
PEAK_HBM_GBS = 8000.0


def flops_per_pair_p2p(kernel_id: int, r: int) -> int:
    """Flop convention for one kernel evaluation + accumulation: 3 sub,
    3 mul + 2 add for r^2, 1 for the kernel (rsqrt) = 9 for 1/r; exp(-r/a)
    adds sqrt, mul and exp (11); the Gaussian adds mul and exp (10); plus
    2 per right-hand side."""
    base = {0: 9, 1: 11, 2: 10}.get(kernel_id, 20)
    return base + 2 * r


def cpu_baseline(w, gpu_phi_rows):
    """The oracle as it stands on this host: full upward pass and M2L, L2P
    and P2P on the sampled targets; P2P time scaled to all N targets."""
    import numpy as np
    from oracle import fmm as ofmm, operators as oops, tree as otree
    rows = w.sample_rows
    t0 = time.perf_counter()
    tr = otree.build_tree(w.points, fixed_depth=w.fixed_depth)
    ops = oops.precompute(tr, w.kernel_id, w.kernel_param, w.order, w.eps)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    ref = ofmm.matvec(tr, ops, w.points, w.sigma, w.kernel_id, w.kernel_param, rows=rows)
    t_sample = time.perf_counter() - t0
    t0 = time.perf_counter()
    ofmm.matvec(tr, ops, w.points, w.sigma, w.kernel_id, w.kernel_param, rows=rows, far=False)
    t_near = time.perf_counter() - t0
    est = t_sample + t_near * (w.n / len(rows) - 1.0)
    exact = ofmm.direct(w.points, w.sigma, w.kernel_id, w.kernel_param, rows=rows)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": w.n * w.r / est, "unit": "points*RHS/s", "cores": cores, "kind": "oracle",
        "sample": (f"FP64 oracle bbFMM on the same workload: upward pass and M2L over all "
                   f"cells plus L2P+P2P on {len(rows)} sampled targets took {t_sample:.2f} s; "
                   f"its P2P part ({t_near:.2f} s) scaled by N/{len(rows)} gives "
                   f"{est:.1f} s per matvec (tree + operator setup {t_setup:.1f} s excluded)"),
        "rel_err_gpu_vs_oracle": ofmm.rel_l2(gpu_phi_rows, ref),
        "rel_err_gpu_vs_direct": ofmm.rel_l2(gpu_phi_rows, exact),
        "rel_err_oracle_vs_direct": ofmm.rel_l2(ref, exact),
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the matvec runs on a single device).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import synth
    from paper_1903_02153_amd import bbfmm

    w = synth.cfg_uniform_1m()
    dev = torch.device("cuda:0")
    pts = torch.from_numpy(w.points).to(dev)
    sig = torch.from_numpy(w.sigma).to(dev)
    phi = torch.empty_like(sig)
    tree = bbfmm.build_tree(pts, w.kernel_id, w.kernel_param, cheb_order=w.order,
                            fixed_depth=w.fixed_depth)
    ops = bbfmm.precompute_operators(tree, w.eps, bbfmm.M2L_FP32)
    plan = bbfmm.Plan(tree, ops, w.r)
    info = tree.info()
    L = info.depth - 1

    for _ in range(args.warmup):
        plan.execute(sig, phi)
    torch.cuda.synchronize()

    K = args.steps
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    plan.set_timing(True)
    plan.stage_times(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        starts[i].record()
        plan.execute(sig, phi)
        ends[i].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stage_ms, nexec = plan.stage_times(reset=True)
    plan.set_timing(False)
    lat = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    ms_per_step = (t1 - t0) * 1e3 / K
    value = w.n * w.r / (ms_per_step / 1e3)
    stage_avg = {k: v / nexec for k, v in stage_ms.items()}

    # roofline of the dominant single-launch kernel
    ranks = {lvl: ops.rank(lvl) for lvl in range(2, info.depth)}
    m2l_flop = sum(info.pairs[lvl] * 2 * ranks[lvl] ** 2 * w.r for lvl in ranks)
    p2p_flop = info.near_pairs * flops_per_pair_p2p(w.kernel_id, w.r)
    if stage_avg["m2l"] >= stage_avg["p2p"]:
        kern, flop, peak, bound = "m2l", m2l_flop, PEAK_FP32_MFMA_TFLOPS, "mfma"
    else:
        kern, flop, peak, bound = "p2p", p2p_flop, PEAK_FP32_VECTOR_TFLOPS, "alu"
    achieved = flop / (stage_avg[kern] * 1e-3) / 1e12
    roofline = {"kernel": kern, "bound": bound, "achieved": round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                "flop_per_launch": flop,
                "other": {"m2l_tflops": round(m2l_flop / (stage_avg["m2l"] * 1e-3) / 1e12, 3),
                          "p2p_tflops": round(p2p_flop / (stage_avg["p2p"] * 1e-3) / 1e12, 3)}}

    out = {
        "metric": METRIC, "value": value, "unit": "points*RHS/s", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "N": w.n, "r": w.r, "kernel": "1/r", "order": w.order,
                   "depth": info.depth, "leaf_cells": info.cells[L], "svd_eps": w.eps,
                   "ranks": ranks, "m2l": "fp32-mfma", "parallelism": "single-gpu"},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(lat.mean())},
        "stage_ms": {k: round(v, 4) for k, v in stage_avg.items()},
        "roofline": roofline,
    }
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)   # 256 MiB
        for _ in range(3):
            dst = src.clone()
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 2 * src.numel() * 4
        del src, dst
    if not args.no_cpu_baseline:
        torch.cuda.synchronize()
        plan.execute(sig, phi)
        torch.cuda.synchronize()
        got = phi.cpu().numpy().astype(np.float64)[w.sample_rows]
        out["cpu_baseline"] = cpu_baseline(w, got)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
