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
timed on the host cores on a bounded sample of the same workload.  Beside
it: the batched mixed-precision forms against plain single-RHS FP32 on the
clustered 2M-point (r = 16) and slab 1M-point (r = 64) workloads, and the
8-tree serving mix (Poisson arrivals, p50/p99 latency, throughput).
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
PEAK_FP32_SCALAR_TFLOPS = 78.6    # the same without packed FP32 (this build issues none)
PEAK_16BIT_MFMA_TFLOPS = 2500.0   # MI355X dense BF16 / FP16 matrix
PEAK_HBM_GBS = 8000.0


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (rocprofv3 FETCH_SIZE and WRITE_SIZE, each scaled by what the counter
    reads for a plain device copy of known size), or None when the summary
    is for another kernel or workload or the kernel source has changed since
    the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    ent = rec.get("kernels", {}).get(kernel)
    if ent is None or rec.get("workload") != workload:
        return None
    with open(os.path.join(ROOT, rec["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
            return None
    return (ent["fetch_kib"] * rec["fetch_scale"] + ent["write_kib"] * rec["write_scale"]) * 1024.0


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden")


def rel_l2(approx, exact) -> float:
    """||approx - exact||_2 / ||exact||_2 over all entries."""
    import numpy as np
    return float(np.linalg.norm(approx - exact) / np.linalg.norm(exact))


def flops_per_pair_p2p(kernel_id: int, r: int) -> int:
    """Flop convention for one kernel evaluation + accumulation: 3 sub,
    3 mul + 2 add for r^2, 1 for the kernel (rsqrt) = 9 for 1/r; exp(-r/a)
    adds sqrt, mul and exp (11); the Gaussian adds mul and exp (10); plus
    2 per right-hand side."""
    base = {0: 9, 1: 11, 2: 10}.get(kernel_id, 20)
    return base + 2 * r


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_threads() -> int:
    """Threads the oracle's BLAS and OpenMP pools use right now."""
    from threadpoolctl import threadpool_info
    return max([int(p.get("num_threads", 1)) for p in threadpool_info()] or [1])


def pass_bytes(info, ranks, order: int, r: int, nsplit: int):
    """Algorithmic HBM bytes of the upward and downward passes (FP32
    operands): upward = points and weights read by P2M (12 + 4r per point),
    then per cell of levels >= 2 its multipoles written and read back by the
    compression (4 n^3 r each) and the compressed ones written (4 k r), plus
    the children's multipoles read by M2M (4 n^3 r per child); downward = per
    cell the M2L partials read (4 k r per partial) and the locals written
    (4 n^3 r), plus for levels >= 3 the parent's locals read by L2L and the
    locals read back by the decompression (4 n^3 r each)."""
    m = order ** 3
    L = info.depth - 1
    up = info.n_points * (12 + 4 * r)
    down = 0
    for lvl in range(2, L + 1):
        C, k = info.cells[lvl], ranks[lvl]
        up += C * r * (8 * m + 4 * k)
        if lvl < L:
            up += info.cells[lvl + 1] * r * 4 * m
        down += C * r * (4 * k * nsplit + 4 * m)
        if lvl > 2:
            down += C * r * 8 * m
    return up, down


def cpu_baseline(w, gpu_phi_rows, single_rows: int = 512):
    """The oracle as it stands on this host: full upward pass and M2L, L2P
    and P2P on the sampled targets; P2P time scaled to all N targets.  Run
    on all host threads (the value) and again on one thread (on the first
    `single_rows` sampled targets).  For a block of right-hand sides the
    oracle runs the first column only (the columns are independent) and the
    rate is per column."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import fmm as ofmm, operators as oops, tree as otree
    rows = w.sample_rows if w.r == 1 else w.sample_rows[::4]
    sig = w.sigma[:, :1]
    t0 = time.perf_counter()
    tr = otree.build_tree(w.points, leaf_size=w.leaf_size, max_depth=w.max_depth,
                          fixed_depth=w.fixed_depth)
    ops = oops.precompute(tr, w.kernel_id, w.kernel_param, w.order, w.eps)
    t_setup = time.perf_counter() - t0

    def timed(rws):
        t0 = time.perf_counter()
        ref = ofmm.matvec(tr, ops, w.points, sig, w.kernel_id, w.kernel_param, rows=rws)
        t_sample = time.perf_counter() - t0
        t0 = time.perf_counter()
        ofmm.matvec(tr, ops, w.points, sig, w.kernel_id, w.kernel_param, rows=rws, far=False)
        t_near = time.perf_counter() - t0
        return ref, t_sample, t_near, t_sample + t_near * (w.n / len(rws) - 1.0)

    threads = _oracle_threads()
    ref, t_sample, t_near, est = timed(rows)
    with threadpool_limits(limits=1):
        one_threads = _oracle_threads()
        _, t1_sample, t1_near, est1 = timed(rows[:single_rows])
    exact = ofmm.direct(w.points, sig, w.kernel_id, w.kernel_param, rows=rows)
    got = gpu_phi_rows[:len(rows)] if w.r == 1 else gpu_phi_rows[::4][:, :1]
    return {
        "value": w.n / est, "unit": "points*RHS/s", "cores": threads, "kind": "oracle",
        "cpu_model": _cpu_model(), "host_logical_cpus": os.cpu_count(),
        "sample": (f"FP64 oracle bbFMM on the same workload (first right-hand side), "
                   f"{threads} threads: upward pass and M2L over all cells plus L2P+P2P on "
                   f"{len(rows)} sampled targets took {t_sample:.2f} s; its P2P part "
                   f"({t_near:.2f} s) scaled by N/{len(rows)} gives {est:.1f} s per matvec "
                   f"(tree + operator setup {t_setup:.1f} s excluded)"),
        "single_thread": {
            "value": w.n / est1, "unit": "points*RHS/s", "cores": one_threads,
            "sample": (f"same, one thread, L2P+P2P on {min(single_rows, len(rows))} sampled "
                       f"targets: {t1_sample:.2f} s, P2P part {t1_near:.2f} s, {est1:.1f} s "
                       f"per matvec")},
        "rel_err_gpu_vs_oracle": ofmm.rel_l2(got, ref),
        "rel_err_gpu_vs_direct": ofmm.rel_l2(got, exact),
        "rel_err_oracle_vs_direct": ofmm.rel_l2(ref, exact),
    }


def fft_m2l_section(w, sig, steps: int = 20):
    """The second M2L variant (Section 2.5): equally spaced nodes with the
    block-Toeplitz M2L applied by the FFT, on the same workload and order as
    the headline, beside the Chebyshev/SVD form; error against the direct
    sum on the workload's sampled rows for both."""
    import numpy as np
    import torch

    from paper_1903_02153_amd import bbfmm
    pts = torch.from_numpy(w.points).cuda()
    tree = bbfmm.build_tree(pts, w.kernel_id, w.kernel_param, cheb_order=w.order,
                            leaf_size=w.leaf_size, max_depth=w.max_depth,
                            fixed_depth=w.fixed_depth)
    stored = np.load(os.path.join(GOLDEN, "bench_ref_uniform.npz"))
    assert np.array_equal(stored["rows"], w.sample_rows)
    exact = stored["direct"]
    out = {"workload": w.name, "order": w.order}
    for tag, prec in (("svd_fp32", bbfmm.M2L_FP32), ("fft_uniform", bbfmm.M2L_FFT)):
        ops = bbfmm.precompute_operators(tree, w.eps, prec)
        plan = bbfmm.Plan(tree, ops, w.r)
        phi = torch.empty_like(sig)
        lat = time_plan(plan, sig, phi, steps, 3)
        plan.set_timing(True)
        plan.stage_times(reset=True)
        for _ in range(5):
            plan.execute(sig, phi)
        torch.cuda.synchronize()
        st, ne = plan.stage_times(reset=True)
        got = phi.cpu().numpy().astype(np.float64)[w.sample_rows]
        med = float(np.median(lat))
        out[tag] = {"ms_median": round(med, 4), "points_rhs_per_s": w.n * w.r / (med * 1e-3),
                    "m2l_ms": round(st["m2l"] / ne, 4),
                    "up_ms": round((st["p2m"] + st["m2m"]) / ne, 4),
                    "down_ms": round(st["down"] / ne, 4),
                    "rel_err_vs_direct": rel_l2(got, exact)}
        if tag == "fft_uniform":
            # algorithmic work of the pointwise products: a complex
            # multiply-add (8 flop) per frequency per interaction pair
            info = tree.info()
            q = (w.order + 1) * (2 * w.order) ** 2
            flop = sum(info.pairs[lvl] for lvl in range(2, info.depth)) * q * 8 * w.r
            tf = flop / (st["m2l"] / ne * 1e-3) / 1e12
            out[tag]["m2l_tflops"] = round(tf, 2)
            out[tag]["m2l_frac_of_non_packed_fp32"] = round(tf / PEAK_FP32_SCALAR_TFLOPS, 4)
        plan.close()
        ops.close()
    return out


def order_study():
    """Error against the direct sum per Chebyshev order (the error-versus-
    order study of the paper's accuracy section) on the small uniform
    workload (4096 points, 1/r, 3 levels): the GPU FP32 matvec at each
    order, with SVD tolerance 1e-5 and without compression, against the
    stored direct sum and FP64 oracle bbFMM (tests/golden/make_bench_refs.py)."""
    import numpy as np
    import torch

    import synth
    from paper_1903_02153_amd import bbfmm
    w = synth.cfg_small()
    stored = np.load(os.path.join(GOLDEN, "bench_ref_orders.npz"))
    exact = stored["direct"]
    orders = [int(v) for v in stored["orders"]]
    epss = [float(v) for v in stored["eps"]]
    pts = torch.from_numpy(w.points).cuda()
    sig = torch.from_numpy(np.ascontiguousarray(w.sigma, dtype=np.float32)).cuda()
    if sig.dim() == 1:
        sig = sig[:, None].contiguous()
    out = []
    for i, n in enumerate(orders):
        tree = bbfmm.build_tree(pts, w.kernel_id, w.kernel_param, cheb_order=n,
                                fixed_depth=w.fixed_depth)
        for j, eps in enumerate(epss):
            ops = bbfmm.precompute_operators(tree, eps)
            got = bbfmm.matvec(tree, ops, sig)
            torch.cuda.synchronize()
            g = got.cpu().numpy().astype(np.float64)
            ref = stored["bbfmm"][i, j]
            out.append({"n": n, "svd_eps": eps,
                        "gpu_vs_direct": rel_l2(g, exact),
                        "gpu_vs_oracle": rel_l2(g, ref),
                        "oracle_vs_direct": rel_l2(ref, exact)})
            ops.close()
        tree.close()
    return {"workload": w.name, "N": w.n, "kernel": "1/r", "depth": w.fixed_depth,
            "rows": "all", "per_order": out}


def time_plan(plan, sig, phi, steps: int, warmup: int):
    """Per-execution device time (ms, HIP events on the launching stream)."""
    import numpy as np
    import torch
    for _ in range(warmup):
        plan.execute(sig, phi)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    for a, b in ev:
        a.record()
        plan.execute(sig, phi)
        b.record()
    torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) for a, b in ev])


def batched_variants(steps: int, warmup: int, tune: bool):
    """Batched mixed-precision forms against plain single-RHS FP32 on the
    two batched workloads: points x RHS/s of the single-RHS FP32 form, the
    r-column FP32 form and the r-column low-precision forms (HIP-graph
    replay), with each form's largest per-column relative difference from
    the r-column FP32 result and its largest per-column relative error
    against the stored FP64 oracle bbFMM on the workload's 4096 sampled rows
    (tests/golden/make_fullsize_refs.py)."""
    import numpy as np
    import torch

    import synth
    from paper_1903_02153_amd import bbfmm
    out = []
    for make, precs in ((synth.cfg_clustered_2m, (bbfmm.M2L_BF16X3, bbfmm.M2L_FP16_SCALED)),
                        (synth.cfg_slab_1m, (bbfmm.M2L_BF16X3, bbfmm.M2L_FP16_SCALED))):
        w = make()
        dev = torch.device("cuda:0")
        pts = torch.from_numpy(w.points).to(dev)
        sig = torch.from_numpy(w.sigma).to(dev)
        tree = bbfmm.build_tree(pts, w.kernel_id, w.kernel_param, cheb_order=w.order,
                                leaf_size=w.leaf_size, max_depth=w.max_depth,
                                fixed_depth=w.fixed_depth)
        info = tree.info()
        rec = {"workload": w.name, "N": w.n, "r": w.r, "depth": info.depth,
               "near_pairs": info.near_pairs, "forms": {}}

        def run(tag, prec, r):
            ops = bbfmm.precompute_operators(tree, w.eps, prec)
            s = sig[:, :r].contiguous()
            phi = torch.empty_like(s)
            opts = bbfmm.autotune(tree, ops, s, phi, reps=3)[0] if tune else {}
            plan = bbfmm.Plan(tree, ops, r, **opts)
            plan.set_graph(True)
            n_steps = steps if r > 1 else max(steps, 10)
            lat = time_plan(plan, s, phi, n_steps, warmup)
            med = float(np.median(lat))
            rec["forms"][tag] = {"precision": ("fp32", "bf16x3", "fp16-scaled")[prec], "r": r,
                                 "ms_median": round(med, 4),
                                 "ms_p99": round(float(np.percentile(lat, 99)), 4),
                                 "points_rhs_per_s": w.n * r / (med * 1e-3),
                                 "plan_options": opts or "heuristic",
                                 "ranks": {lvl: ops.rank(lvl) for lvl in range(2, info.depth)}}
            plan.close()
            return phi

        stored = np.load(os.path.join(GOLDEN, f"fullsize_ref_{w.name}.npz"))
        assert np.array_equal(stored["rows"], w.sample_rows)
        oref = stored["phi"].astype(np.float64)

        def vs_oracle(phi, r):
            got = phi.cpu().numpy().astype(np.float64)[w.sample_rows]
            return float((np.linalg.norm(got - oref[:, :r], axis=0)
                          / np.linalg.norm(oref[:, :r], axis=0)).max())

        r1 = run("fp32_r1", bbfmm.M2L_FP32, 1)
        rec["forms"]["fp32_r1"]["max_col_rel_err_vs_oracle"] = vs_oracle(r1, 1)
        ref = run(f"fp32_r{w.r}", bbfmm.M2L_FP32, w.r)
        rec["forms"][f"fp32_r{w.r}"]["max_col_rel_err_vs_oracle"] = vs_oracle(ref, w.r)
        for prec in precs:
            tag = ("fp32", "bf16x3", "fp16s")[prec] + f"_r{w.r}"
            got = run(tag, prec, w.r)
            d = ((got - ref).norm(dim=0) / ref.norm(dim=0)).max().item()
            rec["forms"][tag]["max_col_rel_diff_vs_fp32"] = d
            rec["forms"][tag]["max_col_rel_err_vs_oracle"] = vs_oracle(got, w.r)
            del got
        base = rec["forms"]["fp32_r1"]["points_rhs_per_s"]
        for f in rec["forms"].values():
            f["speedup_vs_fp32_r1"] = round(f["points_rhs_per_s"] / base, 3)
        out.append(rec)
        del ref, sig, pts, tree
        torch.cuda.empty_cache()
    return out


def adaptive_section(steps: int = 10):
    """The level-adaptive tree (Section 2.1 on adaptive subdivision) on the
    clustered 2M-point workload (64 tight clusters, exp(-r/0.1), n = 6,
    r = 16, split-BF16 M2L, leaf size 64, at most 7 levels, then 8) beside
    the uniform tree of the same depth rule: cells, near-field pairs, time
    per product (HIP-graph replay) and the error against the stored direct
    sum on 1024 sampled rows (tests/golden/make_bench_refs.py)."""
    import numpy as np
    import torch

    import synth
    from paper_1903_02153_amd import bbfmm
    w = synth.cfg_clustered_2m()
    stored = np.load(os.path.join(GOLDEN, "bench_ref_clustered.npz"))
    rows = stored["rows"]
    assert np.array_equal(rows, w.sample_rows[:len(rows)])
    exact = stored["direct"]
    pts = torch.from_numpy(w.points).cuda()
    sig = torch.from_numpy(w.sigma).cuda()
    out = {"workload": w.name, "precision": "bf16x3"}
    # the workload's 7-level cap, then both trees with one more level (the
    # adaptive tree refines only the dense clusters)
    for tag, adaptive, md in (("uniform", False, w.max_depth), ("adaptive", True, w.max_depth),
                              ("uniform_d8", False, w.max_depth + 1),
                              ("adaptive_d8", True, w.max_depth + 1)):
        t0 = time.perf_counter()
        tree = bbfmm.build_tree(pts, w.kernel_id, w.kernel_param, cheb_order=w.order,
                                leaf_size=w.leaf_size, max_depth=md,
                                fixed_depth=w.fixed_depth, adaptive=adaptive)
        torch.cuda.synchronize()
        t_tree = time.perf_counter() - t0
        ops = bbfmm.precompute_operators(tree, w.eps, w.precision)
        phi = torch.empty_like(sig)
        plan = bbfmm.Plan(tree, ops, w.r)
        plan.set_graph(True)
        lat = time_plan(plan, sig, phi, steps, 2)
        plan.set_graph(False)
        plan.set_timing(True)
        plan.stage_times(reset=True)
        for _ in range(3):
            plan.execute(sig, phi)
        torch.cuda.synchronize()
        st, ne = plan.stage_times(reset=True)
        info = tree.info()
        got = phi.cpu().numpy().astype(np.float64)[rows]
        med = float(np.median(lat))
        out[tag] = {"cells": int(sum(info.cells[:info.depth])), "leaves": int(info.n_leaves),
                    "depth": int(info.depth), "near_pairs": int(info.near_pairs),
                    "w_entries": int(info.w_entries), "tree_build_s": round(t_tree, 3),
                    "ms_median": round(med, 4), "points_rhs_per_s": w.n * w.r / (med * 1e-3),
                    "stage_ms": {k: round(v / ne, 4) for k, v in st.items()},
                    "max_col_rel_err_vs_direct": float(
                        (np.linalg.norm(got - exact, axis=0) / np.linalg.norm(exact, axis=0)).max())}
        plan.close()
        ops.close()
        tree.close()
    return out


# wall-clock seconds of the paper's 32-core run for the rows of its
# strong-scaling table (Section 4, Table 1; another machine: context only)
PAPER_32CORE_S = (0.444, 3.49, 21.3)


def paper_scaling_section(steps: int, warmup: int, tune: bool):
    """The workloads of the paper's strong-scaling table (1/r, order 4,
    uniform points, N = 6.4e5 / 5.12e6 / 4.096e7 with 5 / 6 / 7 levels,
    non-negative weights): one GPU's matvec (graph replay, median of
    `steps`, launch shapes autotuned outside the timing), the tree build and
    operator set-up times, and the relative L2 error against the stored FP64
    direct sum on 256 sampled rows (tests/golden/make_paper_scaling_refs.py),
    beside the paper's 32-core wall clock."""
    import numpy as np
    import torch

    import synth
    from paper_1903_02153_amd import bbfmm
    ref = np.load(os.path.join(GOLDEN, "paper_scaling_ref.npz"))
    out = []
    for i in range(len(synth.PAPER_SCALING)):
        w = synth.cfg_paper_scaling(i)
        assert np.array_equal(ref[f"rows_{i}"], w.sample_rows)
        dev = torch.device("cuda:0")
        pts = torch.from_numpy(w.points).to(dev)
        sig = torch.from_numpy(w.sigma).to(dev)
        phi = torch.empty_like(sig)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tree = bbfmm.build_tree(pts, w.kernel_id, w.kernel_param, cheb_order=w.order,
                                fixed_depth=w.fixed_depth)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ops = bbfmm.precompute_operators(tree, w.eps)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        opts = bbfmm.autotune(tree, ops, sig, phi, reps=3)[0] if tune else {}
        plan = bbfmm.Plan(tree, ops, 1, **opts)
        plan.set_graph(True)
        med = float(np.median(time_plan(plan, sig, phi, steps, warmup)))
        got = phi.cpu().numpy().astype(np.float64)[w.sample_rows]
        plan.close()
        out.append({"N": w.n, "levels": w.fixed_depth, "order": w.order,
                    "ms_median": round(med, 4), "points_rhs_per_s": w.n / (med * 1e-3),
                    "tree_build_ms": round((t1 - t0) * 1e3, 2),
                    "operators_ms": round((t2 - t1) * 1e3, 2),
                    "rel_err_vs_direct": rel_l2(got, ref[f"phi_{i}"]),
                    "paper_32core_s": PAPER_32CORE_S[i],
                    "plan_options": opts})
        progress(f"paper scaling row {i}: N {w.n}, {med:.3f} ms")
        del plan, ops, tree, pts, sig, phi, w
        torch.cuda.empty_cache()
    return {"rows": out,
            "note": "the paper's times are FP64 on 2 x 28-core CPUs (32 threads), the same "
                    "workload shape; not the benchmark metric's configuration"}


def pca_section(n: int = 80_000, k: int = 100, l: int = 120):
    """The geostatistics application: top-k eigenpairs of the exp(-r)
    covariance of n uniform points (p = 4, 4 levels as in the paper's
    N = 8e4 run) from two block products with l random right-hand sides."""
    import numpy as np
    import torch

    from paper_1903_02153_amd import bbfmm, pca
    rng = np.random.default_rng(150)
    pts = torch.from_numpy(rng.random((n, 3)).astype(np.float32)).cuda()
    omega = torch.from_numpy(rng.standard_normal((n, l)).astype(np.float32)).cuda()
    tree = bbfmm.build_tree(pts, bbfmm.K_EXP, 1.0, cheb_order=4, fixed_depth=4)
    ops = bbfmm.precompute_operators(tree, 1e-5)
    plan = bbfmm.Plan(tree, ops, l)
    pca.randomized_eigh(tree, ops, omega, k, plan)          # warm-up
    torch.cuda.synchronize()
    times = []
    for _ in range(5):
        t0 = time.perf_counter()
        lam, _ = pca.randomized_eigh(tree, ops, omega, k, plan)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    return {"N": n, "k": k, "l": l, "kernel": "exp(-r)", "order": 4, "depth": 4,
            "ms_median": round(float(np.median(times)) * 1e3, 3),
            "lambda_1": float(lam[0]), "lambda_k": float(lam[-1]),
            "note": "two block products of l columns + CholeskyQR2 + l x l eigensolver, "
                    "wall clock per call"}


def serving_mix(n_requests: int, budget_gib: float, load: float):
    """The 8-tree serving mix: calibrate capacity with closed-loop bursts,
    then replay a Poisson stream at `load` x capacity and report latency
    percentiles (submit to completion, server clock) and throughput."""
    import numpy as np
    import torch

    import synth
    from paper_1903_02153_amd import bbfmm
    dev = torch.device("cuda:0")
    models, ids, classes = [], [], {}
    srv = bbfmm.Server(hbm_budget_bytes=int(budget_gib * (1 << 30)), max_inflight=8, r_max=32)
    rng = np.random.default_rng(5)
    ring = 8
    for i in range(len(synth.SERVING_SIZES)):
        w = synth.serving_tree(i)
        t = bbfmm.build_tree(torch.from_numpy(w.points).to(dev), w.kernel_id, w.kernel_param,
                             cheb_order=w.order, leaf_size=w.leaf_size, max_depth=w.max_depth)
        o = bbfmm.precompute_operators(t, w.eps)
        models.append((t, o, w.n))
        ids.append(srv.add(t, o))
        for r in synth.SERVING_R:
            s = torch.from_numpy(rng.standard_normal((w.n, r)).astype(np.float32)).to(dev)
            classes[(i, r)] = (s, [torch.empty_like(s) for _ in range(ring)])
    torch.cuda.synchronize()
    counter = {}

    def submit(i, r):
        s, outs = classes[(i, r)]
        c = counter.get((i, r), 0)
        counter[(i, r)] = c + 1
        # outputs rotate over a ring per (tree, r) class; they are not inspected
        return srv.submit(ids[i], s, outs[c % ring])

    tree_ix, rs, gaps = synth.serving_requests(n_requests, seed=5)

    def burst(lo, hi):
        t0 = time.perf_counter()
        rids = [submit(int(tree_ix[q]), int(rs[q])) for q in range(lo, hi)]
        st = [srv.wait(q) for q in rids]
        return time.perf_counter() - t0, st

    nb = min(200, n_requests)
    burst(0, nb)                       # creates and captures the plans
    t_burst, st = burst(0, nb)
    work = float(sum(models[int(tree_ix[q])][2] * int(rs[q]) for q in range(nb)))
    capacity = nb / t_burst
    lam = load * capacity
    arrivals = np.cumsum(gaps) / lam
    t0 = time.perf_counter()
    rids = []
    for q in range(n_requests):
        dt = arrivals[q] - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        rids.append(submit(int(tree_ix[q]), int(rs[q])))
    stats = [srv.wait(q) for q in rids]
    counters = srv.stats()
    srv.close()
    lat = np.array([s["t_done"] - s["t_submit"] for s in stats]) * 1e3
    queue = np.array([s["t_admit"] - s["t_submit"] for s in stats]) * 1e3
    span = max(s["t_done"] for s in stats) - min(s["t_submit"] for s in stats)
    total = float(sum(models[int(tree_ix[q])][2] * int(rs[q]) for q in range(n_requests)))
    batched = np.array([s["batch_r"] for s in stats]) > rs
    out = {"trees": [m[2] for m in models], "requests": n_requests, "r_choices": list(synth.SERVING_R),
           "hbm_budget_gib": budget_gib, "max_inflight": 8, "r_max": 32,
           "capacity_req_per_s": round(capacity, 2),
           "capacity_points_rhs_per_s": work / t_burst,
           "arrival_rate_req_per_s": round(lam, 2), "load": load,
           "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                          "mean": float(lat.mean()), "max": float(lat.max())},
           "queue_ms": {"p50": float(np.percentile(queue, 50)), "p99": float(np.percentile(queue, 99))},
           "throughput_points_rhs_per_s": total / span,
           "throughput_req_per_s": n_requests / span,
           "batched_fraction": float(batched.mean()),
           "server_counters": counters}
    del classes
    torch.cuda.empty_cache()
    return out


def progress(msg: str) -> None:
    """One line on stderr per finished phase (the JSON line stays alone on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="uniform-1M",
                    choices=["uniform-1M", "clustered-2M", "slab-1M"],
                    help="uniform-1M: the headline plain FP32 single-RHS workload; the other two "
                         "are the batched workloads (r = 16 and r = 64)")
    ap.add_argument("--precision", default=None, choices=["fp32", "bf16x3", "fp16s"],
                    help="M2L precision (default: fp32 for uniform-1M, else the workload's own)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the built-in launch-shape heuristic instead of bbfmm_plan_autotune")
    ap.add_argument("--plan-options", default=None,
                    help="JSON object of plan options to use instead of autotuning (for profiling "
                         "runs that repeat a configuration)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the batched mixed-precision comparison (clustered-2M, slab-1M)")
    ap.add_argument("--no-serving", action="store_true", help="skip the 8-tree serving mix")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the error-per-order study and the FFT M2L comparison")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--serving-budget-gib", type=float, default=96.0)
    ap.add_argument("--serving-load", type=float, default=0.7)
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

    w = {"uniform-1M": synth.cfg_uniform_1m, "clustered-2M": synth.cfg_clustered_2m,
         "slab-1M": synth.cfg_slab_1m}[args.workload]()
    prec_names = ("fp32", "bf16x3", "fp16s")
    prec = (prec_names.index(args.precision) if args.precision else
            (bbfmm.M2L_FP32 if args.workload == "uniform-1M" else w.precision))
    dev = torch.device("cuda:0")
    pts = torch.from_numpy(w.points).to(dev)
    sig = torch.from_numpy(w.sigma).to(dev)
    phi = torch.empty_like(sig)
    tree = bbfmm.build_tree(pts, w.kernel_id, w.kernel_param, cheb_order=w.order,
                            leaf_size=w.leaf_size, max_depth=w.max_depth,
                            fixed_depth=w.fixed_depth)
    ops = bbfmm.precompute_operators(tree, w.eps, prec)
    opts = {}
    if args.plan_options:
        opts = {k: int(v) for k, v in json.loads(args.plan_options).items()}
    elif not args.no_autotune:     # launch shapes only; outside the timed region
        opts, _ = bbfmm.autotune(tree, ops, sig, phi, reps=5)
    plan = bbfmm.Plan(tree, ops, w.r, **opts)
    info = tree.info()
    progress(f"{w.name}: tree, operators and plan ready ({opts or 'heuristic'})")
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
    progress(f"timed region: {K} steps, {(t1 - t0) * 1e3 / K:.3f} ms per step")
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
        kern, flop, bound = "m2l", m2l_flop, "mfma"
        peak = PEAK_FP32_MFMA_TFLOPS if prec == bbfmm.M2L_FP32 else PEAK_16BIT_MFMA_TFLOPS
    else:
        kern, flop, peak, bound = "p2p", p2p_flop, PEAK_FP32_VECTOR_TFLOPS, "alu"
    achieved = flop / (stage_avg[kern] * 1e-3) / 1e12
    # the same kernel alone: a short run with the one-stream schedule (the
    # timed region above may overlap the near field with the far field)
    isolated = None
    if opts.get("overlap", 1) == 2:
        solo = bbfmm.Plan(tree, ops, w.r, **dict(opts, overlap=1))
        for _ in range(3):
            solo.execute(sig, phi)
        solo.set_timing(True)
        solo.stage_times(reset=True)
        for _ in range(20):
            solo.execute(sig, phi)
        torch.cuda.synchronize()
        sms, sn = solo.stage_times(reset=True)
        solo.close()
        t_iso = sms[kern] / sn
        t_p2p = sms["p2p"] / sn
        isolated = {"ms": round(t_iso, 4), "achieved": round(flop / (t_iso * 1e-3) / 1e12, 3),
                    "frac": round(flop / (t_iso * 1e-3) / 1e12 / peak, 4),
                    "p2p_ms": round(t_p2p, 4),
                    "p2p_tflops": round(p2p_flop / (t_p2p * 1e-3) / 1e12, 3),
                    "p2p_frac_of_non_packed_fp32": round(p2p_flop / (t_p2p * 1e-3) / 1e12
                                                         / PEAK_FP32_SCALAR_TFLOPS, 4),
                    "note": "same plan options with the one-stream schedule, 20 launches; "
                            "p2p_* is the near-field stage alone (near field + L2P kernels) "
                            "against the 78.6 TFLOP/s FP32 vector rate without packed FP32"}
    # the same plan replayed as one HIP graph per product (after the timed
    # region; reported beside the metric, which is the eager timed region)
    plan.set_graph(True)
    for _ in range(3):
        plan.execute(sig, phi)
    torch.cuda.synchronize()
    tg0 = time.perf_counter()
    for _ in range(K):
        plan.execute(sig, phi)
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - tg0) * 1e3 / K
    plan.set_graph(False)
    up_b, down_b = pass_bytes(info, ranks, w.order, w.r, int(opts.get("m2l_split", 1)) if opts else 1)
    passes = {"up_gbs": round(up_b / ((stage_avg["p2m"] + stage_avg["m2m"]) * 1e-3) / 1e9, 1),
              "down_gbs": round(down_b / (stage_avg["down"] * 1e-3) / 1e9, 1),
              "up_bytes": up_b, "down_bytes": down_b, "peak_gbs": PEAK_HBM_GBS,
              "note": "algorithmic bytes (FP32 operands) over the stage times; the upward "
                      "chain may run beside the near field or the M2L"}
    roofline = {"kernel": kern, "bound": bound, "achieved": round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                "traffic": measured_traffic("k_m2l" if kern == "m2l" else "k_p2p", w.name),
                "flop_per_launch": flop,
                "other": {"m2l_tflops": round(m2l_flop / (stage_avg["m2l"] * 1e-3) / 1e12, 3),
                          "p2p_tflops": round(p2p_flop / (stage_avg["p2p"] * 1e-3) / 1e12, 3)},
                "isolated": isolated}

    out = {
        "metric": METRIC, "value": value, "unit": "points*RHS/s", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec == bbfmm.M2L_FP32 else ("f32+bf16x3" if prec == bbfmm.M2L_BF16X3
                                                       else "f32+f16"),
        "data": "synthetic",
        "config": {"workload": w.name, "N": w.n, "r": w.r,
                   "kernel": {0: "1/r", 1: f"exp(-r/{w.kernel_param})",
                              2: f"exp(-r^2/{w.kernel_param}^2)"}[w.kernel_id],
                   "order": w.order, "depth": info.depth, "leaf_cells": info.cells[L],
                   "svd_eps": w.eps, "ranks": ranks,
                   "m2l": ("fp32", "split-bf16x3", "scaled-fp16")[prec] + "-mfma",
                   "parallelism": "single-gpu",
                   "plan_options": opts or "heuristic"},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(lat.mean())},
        "graph_replay": {"ms_per_step": round(graph_ms, 4),
                         "points_rhs_per_s": w.n * w.r / (graph_ms / 1e3),
                         "note": "the same plan replayed as a HIP graph, K products after the "
                                 "timed region (the metric is the eager, stage-timed region)"},
        "stage_ms": {k: round(v, 4) for k, v in stage_avg.items()},
        "passes": passes,
        "roofline": roofline,
    }
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)   # 256 MiB
        for _ in range(3):
            dst = src.clone()
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 2 * src.numel() * 4
        del src, dst
    if args.workload != "uniform-1M":
        args.no_variants = args.no_serving = True     # sections of the headline run only
    if not args.no_variants:
        out["batched_variants"] = batched_variants(max(5, min(args.steps, 20)), 2,
                                                   not args.no_autotune)
        progress("batched variants done")
    if not args.no_serving:
        out["serving"] = serving_mix(args.serving_requests, args.serving_budget_gib,
                                     args.serving_load)
        progress("serving mix done")
    if not args.no_variants:
        out["pca"] = pca_section()
    if args.workload == "uniform-1M" and not args.no_extras:
        out["paper_scaling"] = paper_scaling_section(10, 3, not args.no_autotune)
        progress("randomized eigendecomposition done")
    if args.workload == "uniform-1M" and not args.no_extras:
        out["order_study"] = order_study()
        progress("error per order done")
        out["adaptive_tree"] = adaptive_section()
        progress("adaptive tree done")
        out["m2l_fft"] = fft_m2l_section(w, sig)
        progress("FFT M2L variant done")
    if not args.no_cpu_baseline:
        torch.cuda.synchronize()
        plan.execute(sig, phi)
        torch.cuda.synchronize()
        got = phi.cpu().numpy().astype(np.float64)[w.sample_rows]
        out["cpu_baseline"] = cpu_baseline(w, got)
        progress("CPU oracle baseline done")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
