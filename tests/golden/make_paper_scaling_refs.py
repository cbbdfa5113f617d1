"""Writes the stored FP64 direct sums (eq. (1), the oracle's pair loop) on
the sampled rows of the three workloads of the paper's strong-scaling
table (Section 4: 1/r, order 4, uniform points, N = 6.4e5 / 5.12e6 /
4.096e7 with 5 / 6 / 7 levels), which the benchmark's scaling section
compares the GPU against:

  paper_scaling_ref.npz   rows_<i>, phi_<i> for i = 0, 1, 2

Only ``oracle/`` and the seeded input generators are used.

    python tests/golden/make_paper_scaling_refs.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import fmm as ofmm  # noqa: E402


def main():
    out = {}
    for i in range(len(synth.PAPER_SCALING)):
        w = synth.cfg_paper_scaling(i)
        out[f"rows_{i}"] = w.sample_rows
        out[f"phi_{i}"] = ofmm.direct(w.points, w.sigma, w.kernel_id, w.kernel_param,
                                      rows=w.sample_rows)
        print(w.name, "done", flush=True)
        del w
    np.savez_compressed(os.path.join(HERE, "paper_scaling_ref.npz"), **out)


if __name__ == "__main__":
    main()
