"""Writes the stored FP64-oracle references that the benchmark's accuracy
sections compare the GPU against (the benchmark itself never runs the
oracle outside its CPU-baseline leg).

  bench_ref_orders.npz   the small uniform workload (4096 points, 1/r, three
                         levels): the direct sum (eq. (1)) on every row, and
                         the oracle bbFMM at Chebyshev orders 2..8 with SVD
                         tolerance 1e-5 and without compression
  bench_ref_uniform.npz  the uniform 1M-point workload: the direct sum on its
                         4096 sampled rows
  bench_ref_clustered.npz the clustered 2M-point workload (r = 16): the direct
                         sum on the first 1024 of its sampled rows, all columns

All values FP64.  Only ``oracle/`` and the seeded input generators are used.

    python tests/golden/make_bench_refs.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import fmm as ofmm, operators as oops, tree as otree  # noqa: E402

ORDERS = tuple(range(2, 9))
EPS = (1e-5, 0.0)


def main() -> None:
    w = synth.cfg_small()
    exact = ofmm.direct(w.points, w.sigma, w.kernel_id, w.kernel_param)
    ot = otree.build_tree(w.points, fixed_depth=w.fixed_depth)
    fmm = np.zeros((len(ORDERS), len(EPS)) + exact.shape)
    for i, n in enumerate(ORDERS):
        for j, eps in enumerate(EPS):
            oo = oops.precompute(ot, w.kernel_id, w.kernel_param, n, eps)
            fmm[i, j] = ofmm.matvec(ot, oo, w.points, w.sigma, w.kernel_id, w.kernel_param)
            print("order", n, "eps", eps, flush=True)
    np.savez_compressed(os.path.join(HERE, "bench_ref_orders.npz"), direct=exact, bbfmm=fmm,
                        orders=np.array(ORDERS), eps=np.array(EPS))
    u = synth.cfg_uniform_1m()
    ex = ofmm.direct(u.points, u.sigma, u.kernel_id, u.kernel_param, rows=u.sample_rows)
    np.savez_compressed(os.path.join(HERE, "bench_ref_uniform.npz"), direct=ex,
                        rows=u.sample_rows.astype(np.int64))
    print("uniform-1M sampled rows", ex.shape, flush=True)
    c = synth.cfg_clustered_2m()
    rows = c.sample_rows[:1024]
    ex = ofmm.direct(c.points, c.sigma, c.kernel_id, c.kernel_param, rows=rows)
    np.savez_compressed(os.path.join(HERE, "bench_ref_clustered.npz"), direct=ex,
                        rows=rows.astype(np.int64))
    print("clustered-2M sampled rows", ex.shape, flush=True)


if __name__ == "__main__":
    main()
