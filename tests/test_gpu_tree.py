"""GPU octree and lists against the oracle, bit for bit (Section 2.1,
Definition 2.1): permutation, per-level keys / point ranges / parents /
children, leaf neighbour CSR and the M2L pair lists grouped by transfer
vector, for uniform, clustered and slab clouds, the leaf-size depth rule,
ragged sizes and degenerate inputs."""
import numpy as np
import pytest

import synth
from _helpers import compare_trees, gpu_tree, oracle_tree

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,seed,kind,depth", [
    (4096, 1, "uniform", 3), (20011, 2, "uniform", 5), (30000, 3, "clustered", 6),
    (12345, 4, "slab", 5), (777, 5, "clustered", 4), (1, 6, "uniform", 1),
    (50, 7, "uniform", 2), (3000, 8, "uniform", 7)])
def test_fixed_depth_tree_bit_exact(n, seed, kind, depth):
    pts, _ = synth.random_cloud(n, seed, kind=kind)
    compare_trees(gpu_tree(pts, 0, 1.0, 4, fixed_depth=depth),
                  oracle_tree(pts, fixed_depth=depth))


@pytest.mark.parametrize("n,seed,kind,leaf,cap", [
    (40000, 11, "clustered", 64, 7), (20000, 12, "uniform", 32, 22),
    (5000, 13, "slab", 16, 9), (100, 14, "uniform", 200, 22)])
def test_depth_rule_tree_bit_exact(n, seed, kind, leaf, cap):
    pts, _ = synth.random_cloud(n, seed, kind=kind)
    compare_trees(gpu_tree(pts, 1, 0.1, 5, leaf_size=leaf, max_depth=cap),
                  oracle_tree(pts, leaf_size=leaf, max_depth=cap))


def test_degenerate_clouds():
    same = np.full((300, 3), 0.25, np.float32)
    compare_trees(gpu_tree(same, 0, 1.0, 4, fixed_depth=4), oracle_tree(same, fixed_depth=4))
    line = np.zeros((500, 3), np.float32)
    line[:, 0] = np.linspace(-3, 5, 500, dtype=np.float32)
    compare_trees(gpu_tree(line, 0, 1.0, 4, fixed_depth=6), oracle_tree(line, fixed_depth=6))
    dup = np.repeat(synth.random_cloud(100, 3)[0], 7, axis=0)
    compare_trees(gpu_tree(dup, 0, 1.0, 4, leaf_size=10, max_depth=8),
                  oracle_tree(dup, leaf_size=10, max_depth=8))


def test_full_size_uniform_1m_tree_bit_exact():
    w = synth.cfg_uniform_1m()
    compare_trees(gpu_tree(w.points, 0, 1.0, 5, fixed_depth=6), oracle_tree(w.points, fixed_depth=6))


def test_nonfinite_points_rejected():
    from paper_1903_02153_amd import bbfmm
    pts, _ = synth.random_cloud(100, 1)
    pts[17, 1] = np.nan
    with pytest.raises(bbfmm.BBFMMError, match="non-finite"):
        gpu_tree(pts, 0, 1.0, 4, fixed_depth=3)
