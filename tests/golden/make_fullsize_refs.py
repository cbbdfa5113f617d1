"""Writes the stored FP64-oracle references of the full-size parity tests.

For the clustered 2M-point workload (r = 16) and the slab 1M-point workload
(r = 64), the oracle bbFMM (same tree, order and SVD tolerance as the GPU
run) on the workload's 4096 sampled rows and every column, rounded to
float32 for storage (a relative perturbation of 6e-8, two orders of
magnitude below the parity bars).  Only ``oracle/`` and the seeded input
generators are used.  The tests recompute one column with the oracle and
compare it with the stored one before using the file.

    python tests/golden/make_fullsize_refs.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import fmm as ofmm, operators as oops, tree as otree  # noqa: E402


def reference(w):
    ot = otree.build_tree(w.points, leaf_size=w.leaf_size, max_depth=w.max_depth,
                          fixed_depth=w.fixed_depth)
    oo = oops.precompute(ot, w.kernel_id, w.kernel_param, w.order, w.eps)
    return ofmm.matvec(ot, oo, w.points, w.sigma, w.kernel_id, w.kernel_param,
                       rows=w.sample_rows)


def path(name: str) -> str:
    return os.path.join(HERE, f"fullsize_ref_{name}.npz")


def main() -> None:
    for make in (synth.cfg_clustered_2m, synth.cfg_slab_1m):
        w = make()
        ref = reference(w)
        np.savez_compressed(path(w.name), phi=ref.astype(np.float32),
                            rows=w.sample_rows.astype(np.int64))
        print(w.name, ref.shape, flush=True)


if __name__ == "__main__":
    main()
