"""Seeded synthetic inputs for the bbFMM matvec.

This module holds no part of the method's arithmetic: it only draws point
clouds and weight matrices.  Both the FP64 oracle and the HIP path consume
exactly the arrays produced here, so parity is checked on identical inputs.

Shapes follow the paper's experiments (Section 4): sources = targets, points
drawn uniformly in the unit cube (Section 4, "Parameters and notations"),
plus two non-uniform clouds standing in for the Gaussian-process workloads of
Section 4.3 (the FEniCS mesh of that section is not available).

Conventions shared by every generator:
  * a fresh ``numpy.random.default_rng(seed)`` (PCG64) per workload;
  * draw order: points first, then the weights;
  * points are drawn in float64 and rounded to float32; those float32 values
    are the input of both sides;
  * weights are float32 arrays of shape (N, r), row-major (r fastest).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

# kernel identifiers (same numbering as the C-ABI enum)
KERNEL_INV_R = 0
KERNEL_EXP = 1
KERNEL_GAUSS = 2
KERNEL_POLY_TEST = 100

PREC_FP32 = 0
PREC_BF16X3 = 1
PREC_FP16_SCALED = 2


@dataclasses.dataclass
class Workload:
    name: str
    points: np.ndarray            # (N, 3) float32, original order
    sigma: np.ndarray             # (N, r) float32
    kernel_id: int
    kernel_param: float
    order: int                    # Chebyshev nodes per axis (n)
    fixed_depth: int = 0          # >0: number of tree levels including the root
    leaf_size: int = 64
    max_depth: int = 22
    eps: float = 1e-5             # SVD truncation of the M2L operators
    precision: int = PREC_FP32
    sample_rows: Optional[np.ndarray] = None  # rows checked against the oracle

    @property
    def n(self) -> int:
        return self.points.shape[0]

    @property
    def r(self) -> int:
        return self.sigma.shape[1]


def uniform_points(rng: np.random.Generator, n: int) -> np.ndarray:
    """N iid points, uniform in [0,1)^3, rounded to float32."""
    return rng.random((n, 3)).astype(np.float32)


def clustered_points(rng: np.random.Generator, n: int, n_centers: int = 64,
                     std: float = 0.02) -> np.ndarray:
    """Gaussian clusters: centres uniform in the unit cube, labels uniform,
    isotropic normal offsets; not clipped to the cube."""
    centers = rng.random((n_centers, 3))
    labels = rng.integers(0, n_centers, size=n)
    offsets = rng.normal(0.0, std, size=(n, 3))
    return (centers[labels] + offsets).astype(np.float32)


def jittered_slab(rng: np.random.Generator, nx: int = 200, ny: int = 200,
                  nz: int = 25, h: float = 0.005) -> np.ndarray:
    """Points of an nx*ny*nz grid with spacing h, each moved by an
    independent uniform jitter of +-h/4 per axis (x fastest in the order)."""
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                          indexing="ij")
    idx = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64)
    jitter = rng.uniform(-0.25, 0.25, size=idx.shape)
    return ((idx + 0.5 + jitter) * h).astype(np.float32)


def cfg_small(seed: int = 1) -> Workload:
    """N=4096 uniform, 1/r, n=4, 3 levels, one RHS in U[-1,1]."""
    rng = np.random.default_rng(seed)
    pts = uniform_points(rng, 4096)
    sig = rng.uniform(-1.0, 1.0, size=(4096, 1)).astype(np.float32)
    return Workload("uniform-4k-invr-n4-d3", pts, sig, KERNEL_INV_R, 1.0, 4,
                    fixed_depth=3)


def cfg_uniform_1m(seed: int = 2, sample_seed: int = 1002,
                   n_sample: int = 4096) -> Workload:
    """N=2^20 uniform, 1/r, n=5, 6 levels, one RHS; 4096 rows sampled
    without replacement for the oracle comparison."""
    rng = np.random.default_rng(seed)
    n = 1 << 20
    pts = uniform_points(rng, n)
    sig = rng.uniform(-1.0, 1.0, size=(n, 1)).astype(np.float32)
    rows = np.sort(np.random.default_rng(sample_seed).choice(n, n_sample,
                                                             replace=False))
    return Workload("uniform-1M-invr-n5-d6", pts, sig, KERNEL_INV_R, 1.0, 5,
                    fixed_depth=6, sample_rows=rows)


# The paper's strong-scaling table (Section 4): uniform points in the unit
# cube, 1/r, Chebyshev order 4, tree levels 5 / 6 / 7 for N = 6.4e5 / 5.12e6
# / 4.096e7 (about 156 points per leaf).
PAPER_SCALING = ((640_000, 5), (5_120_000, 6), (40_960_000, 7))


def cfg_paper_scaling(i: int, n_sample: int = 256) -> Workload:
    """Row i of the paper's strong-scaling table: N uniform points, 1/r,
    n = 4, fixed depth, one RHS in U[0,1] (non-negative weights: the table
    does not print them, and these reproduce its errors); n_sample rows
    sampled without replacement for the comparison with the direct sum."""
    n, depth = PAPER_SCALING[i]
    rng = np.random.default_rng(60 + i)
    pts = uniform_points(rng, n)
    sig = rng.uniform(0.0, 1.0, size=(n, 1)).astype(np.float32)
    rows = np.sort(np.random.default_rng(1060 + i).choice(n, n_sample, replace=False))
    return Workload(f"uniform-{n}-invr-n4-d{depth}", pts, sig, KERNEL_INV_R, 1.0, 4,
                    fixed_depth=depth, sample_rows=rows)


def cfg_clustered_2m(seed: int = 3, r: int = 16,
                     precision: int = PREC_BF16X3) -> Workload:
    """N=2^21 in 64 Gaussian clusters (std 0.02), exp(-r/0.1), n=6, depth by
    the leaf-size rule capped at 7 levels, r=16 RHS ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    n = 1 << 21
    pts = clustered_points(rng, n)
    sig = rng.standard_normal((n, r)).astype(np.float32)
    rows = np.sort(np.random.default_rng(seed + 1000).choice(n, 4096,
                                                             replace=False))
    return Workload("clustered-2M-exp-n6-d7-r16", pts, sig, KERNEL_EXP, 0.1, 6,
                    leaf_size=64, max_depth=7, precision=precision,
                    sample_rows=rows)


def cfg_slab_1m(seed: int = 4, r: int = 64,
                precision: int = PREC_FP16_SCALED) -> Workload:
    """Jittered 200x200x25 grid in a 1x1x0.125 box, exp(-r^2/0.05^2), n=7,
    7 levels, r=64 RHS ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    pts = jittered_slab(rng)
    sig = rng.standard_normal((pts.shape[0], r)).astype(np.float32)
    rows = np.sort(np.random.default_rng(seed + 1000).choice(pts.shape[0],
                                                             4096,
                                                             replace=False))
    return Workload("slab-1M-gauss-n7-d7-r64", pts, sig, KERNEL_GAUSS, 0.05, 7,
                    fixed_depth=7, precision=precision, sample_rows=rows)


SERVING_SIZES = (16384, 65536, 262144, 524288, 1 << 20, 1 << 20, 1 << 21,
                 1 << 21)


def serving_tree(i: int) -> Workload:
    """Tree i of the 8-tree serving mix: uniform when floor(i/2) is even,
    clustered otherwise; 1/r for even i, exp(-r/0.1) for odd i; n = 4 + i%3;
    leaf-size 64 with at most 7 levels.  Weights are a single column (the
    request stream draws its own)."""
    rng = np.random.default_rng(50 + i)
    n = SERVING_SIZES[i]
    pts = uniform_points(rng, n) if (i // 2) % 2 == 0 else clustered_points(rng, n)
    sig = rng.standard_normal((n, 1)).astype(np.float32)
    kid, prm = (KERNEL_INV_R, 1.0) if i % 2 == 0 else (KERNEL_EXP, 0.1)
    return Workload(f"serve-{i}", pts, sig, kid, prm, 4 + i % 3, leaf_size=64,
                    max_depth=7)


SERVING_R = (1, 4, 16, 32)


def serving_requests(n_req: int = 2000, seed: int = 5):
    """Request stream of the serving mix: tree index uniform over the 8
    trees, r uniform over SERVING_R, and unit-rate exponential inter-arrival
    gaps (divide by the arrival rate lambda to get seconds).  Returns
    (tree (n_req,) int, r (n_req,) int, gap (n_req,) float64)."""
    rng = np.random.default_rng(seed)
    tree = rng.integers(0, len(SERVING_SIZES), n_req)
    r = np.asarray(SERVING_R)[rng.integers(0, len(SERVING_R), n_req)]
    gap = rng.exponential(1.0, n_req)
    return tree, r, gap


def random_cloud(n: int, seed: int, r: int = 1, kind: str = "uniform"):
    """Small generic clouds for tests: returns (points f32 (n,3), sigma f32 (n,r))."""
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        pts = uniform_points(rng, n)
    elif kind == "clustered":
        pts = clustered_points(rng, n, n_centers=8, std=0.05)
    elif kind == "slab":
        pts = rng.random((n, 3)) * np.array([1.0, 1.0, 0.125])
        pts = pts.astype(np.float32)
    else:
        raise ValueError(kind)
    sig = rng.uniform(-1.0, 1.0, size=(n, r)).astype(np.float32)
    return pts, sig
