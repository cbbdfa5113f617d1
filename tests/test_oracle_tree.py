"""Pins of the oracle's octree and lists (Section 2.1, Definition 2.1).

The lists built by ``oracle.tree`` (enumeration over offsets and transfer
vectors) are checked against a brute-force, set-based reading of Definition
2.1 over all cell pairs, against the counts the paper prints (27, 189, 316)
and against the coverage property of the figure in Section 2.3: every
source/target pair is handled exactly once, by P2P or by M2L on one level.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import tree as T

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")


def _counts():
    with open(GOLD) as f:
        return json.load(f)


def test_transfer_vectors():
    tv = T.transfer_vectors()
    assert len(tv) == _counts()["distinct_m2l_operators_per_level"] == 7 ** 3 - 3 ** 3
    assert len({tuple(t) for t in tv}) == 316
    assert np.all(np.abs(tv).max(axis=1) >= 2) and np.all(np.abs(tv) <= 3)
    idx = (tv[:, 0] + 3) + 7 * (tv[:, 1] + 3) + 49 * (tv[:, 2] + 3)
    assert np.all(np.diff(idx) > 0)


def test_morton_roundtrip_and_order():
    rng = np.random.default_rng(0)
    k = rng.integers(0, 1 << 7, (500, 3))
    key = T.morton(k, 7)
    assert np.array_equal(T.decode(key, 7), k)
    # bit layout: x -> bit 0, y -> bit 1, z -> bit 2
    assert T.morton(np.array([[1, 0, 0]]), 1)[0] == 1
    assert T.morton(np.array([[0, 1, 0]]), 1)[0] == 2
    assert T.morton(np.array([[0, 0, 1]]), 1)[0] == 4
    assert T.morton(np.array([[2, 0, 0]]), 2)[0] == 8


def _points_in_cells(tree, pts):
    """Each point lies in its leaf's box [lo + k w, lo + (k+1) w] up to the
    float32 binning error."""
    L = tree.leaf_level
    lev = tree.levels[L]
    w = float(tree.side) / 2 ** L
    Y = pts[tree.perm].astype(np.float64)
    leaf_of = np.repeat(np.arange(len(lev.keys)), lev.pe - lev.pb)
    lo = tree.lo.astype(np.float64) + lev.coords[leaf_of] * w
    tol = 4e-7 * float(tree.side) + 1e-30
    assert np.all(Y >= lo - tol) and np.all(Y <= lo + w + tol)


@pytest.mark.parametrize("kind", ["uniform", "clustered", "slab"])
def test_binning_sort_and_levels(kind):
    pts, _ = synth.random_cloud(3000, 7, kind=kind)
    tree = T.build_tree(pts, leaf_size=40, max_depth=8)
    _points_in_cells(tree, pts)
    L = tree.leaf_level
    # stable sort: keys ascending, ties in input order
    q = T.quantize(pts, tree.lo, tree.scale)
    key = T.morton(q >> (T.QBITS - L), L)[tree.perm]
    assert np.all(np.diff(key.astype(np.float64)) >= 0)
    same = key[1:] == key[:-1]
    assert np.all(tree.perm[1:][same] > tree.perm[:-1][same])
    # depth rule: smallest depth with every leaf <= leaf_size (cap 8)
    lev = tree.levels[L]
    assert (lev.pe - lev.pb).max() <= 40 or tree.depth == 8
    if tree.depth > 1:
        kp = T.morton(q >> (T.QBITS - (L - 1)), L - 1)
        assert np.unique(kp, return_counts=True)[1].max() > 40
    # parent / child / point ranges nest
    for lvl in range(1, tree.depth):
        ch, par = tree.levels[lvl], tree.levels[lvl - 1]
        assert np.array_equal(ch.keys >> np.uint64(3), par.keys[ch.parent])
        for p in range(len(par.keys)):
            c = np.arange(par.cb[p], par.ce[p])
            assert np.all(ch.parent[c] == p)
            assert par.pb[p] == ch.pb[c[0]] and par.pe[p] == ch.pe[c[-1]]
    assert tree.levels[0].pb[0] == 0 and tree.levels[0].pe[0] == len(pts)


def _adjacent(a, b):
    return max(abs(int(x) - int(y)) for x, y in zip(a, b)) <= 1


def _brute_lists(tree, lvl):
    """Definition 2.1 over every cell pair, written with sets."""
    lev = tree.levels[lvl]
    C = len(lev.keys)
    nbr = [{b for b in range(C) if _adjacent(lev.coords[a], lev.coords[b])}
           for a in range(C)]
    if lvl < 2:
        return nbr, [set() for _ in range(C)]
    par = tree.levels[lvl - 1]
    inter = []
    for a in range(C):
        pa = lev.parent[a]
        pn = {p for p in range(len(par.keys)) if _adjacent(par.coords[pa], par.coords[p])}
        children = {b for b in range(C) if lev.parent[b] in pn}
        inter.append(children - nbr[a])
    return nbr, inter


@pytest.mark.parametrize("seed,kind,depth", [(1, "uniform", 4), (2, "clustered", 5),
                                             (3, "slab", 4), (4, "uniform", 3)])
def test_lists_match_definition(seed, kind, depth):
    pts, _ = synth.random_cloud(600, seed, kind=kind)
    tree = T.build_tree(pts, fixed_depth=depth)
    counts = _counts()
    L = tree.leaf_level
    nbr, _ = _brute_lists(tree, L)
    for a in range(len(nbr)):
        row = tree.nbr_idx[tree.nbr_off[a]:tree.nbr_off[a + 1]]
        assert list(row) == sorted(nbr[a])
        assert a in row and len(row) <= counts["max_neighbors_3d"]
    tv = T.transfer_vectors()
    for lvl in range(2, tree.depth):
        _, inter = _brute_lists(tree, lvl)
        pr = tree.pairs[lvl]
        got = [set() for _ in inter]
        for t, a, b in zip(pr["t"], pr["tgt"], pr["src"]):
            got[a].add(b)
            lev = tree.levels[lvl]
            assert np.array_equal(lev.coords[b] - lev.coords[a], tv[t])
        assert got == inter
        assert max(len(s) for s in got) <= counts["max_interaction_list_3d"]
        # grouped by t, ascending target inside each group
        g = pr["group_off"]
        assert g[-1] == len(pr["t"])
        for ti in range(316):
            s, e = g[ti], g[ti + 1]
            assert np.all(pr["t"][s:e] == ti)
            assert np.all(np.diff(pr["tgt"][s:e]) > 0)


def test_full_tree_counts():
    """In a full tree, an interior cell has 27 neighbours and 189 cells in its
    interaction list (6^3 - 3^3)."""
    g = (np.arange(16) + 0.5) / 16
    pts = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3).astype(np.float32)
    tree = T.build_tree(pts, fixed_depth=5)
    L = tree.leaf_level
    deg = np.diff(tree.nbr_off)
    assert deg.max() == 27 and deg.min() == 8
    pr = tree.pairs[L]
    cnt = np.bincount(pr["tgt"], minlength=len(tree.levels[L].keys))
    assert cnt.max() == 189
    # each octant uses exactly the 189 transfer vectors whose parents touch
    oct_ = (tree.levels[L].keys & np.uint64(7)).astype(int)
    for o in range(8):
        ts = set(pr["t"][oct_[pr["tgt"]] == o])
        assert len(ts) == 189


@pytest.mark.parametrize("depth", [1, 2, 3, 4, 5])
def test_coverage_each_pair_exactly_once(depth):
    pts, _ = synth.random_cloud(250, 11 + depth, kind="clustered")
    tree = T.build_tree(pts, fixed_depth=depth)
    N = len(pts)
    cover = np.zeros((N, N), np.int64)
    pos_of = np.empty(N, np.int64)
    pos_of[tree.perm] = np.arange(N)
    L = tree.leaf_level
    leaf = tree.levels[L]
    for a in range(len(leaf.keys)):
        tg = tree.perm[leaf.pb[a]:leaf.pe[a]]
        for b in tree.nbr_idx[tree.nbr_off[a]:tree.nbr_off[a + 1]]:
            sr = tree.perm[leaf.pb[b]:leaf.pe[b]]
            cover[np.ix_(tg, sr)] += 1
    for lvl in range(2, tree.depth):
        lev = tree.levels[lvl]
        pr = tree.pairs[lvl]
        for a, b in zip(pr["tgt"], pr["src"]):
            tg = tree.perm[lev.pb[a]:lev.pe[a]]
            sr = tree.perm[lev.pb[b]:lev.pe[b]]
            cover[np.ix_(tg, sr)] += 1
    assert np.all(cover == 1)


def test_degenerate_inputs():
    one = T.build_tree(np.array([[0.25, 0.5, 0.75]], np.float32), leaf_size=4)
    assert one.depth == 1 and one.side == 1.0 and len(one.levels[0].keys) == 1
    same = T.build_tree(np.full((10, 3), 0.3, np.float32), fixed_depth=4)
    assert float(same.side) == 1.0
    assert len(same.levels[3].keys) == 1 and list(same.perm) == list(range(10))
    # the max face is clamped into the last cell
    pts = np.array([[0, 0, 0], [1, 1, 1]], np.float32)
    tr = T.build_tree(pts, fixed_depth=3)
    assert tr.levels[2].coords.tolist() == [[0, 0, 0], [3, 3, 3]]
    with pytest.raises(ValueError):
        T.build_tree(np.array([[0, np.nan, 0]], np.float32))
    with pytest.raises(ValueError):
        T.build_tree(np.zeros((0, 3), np.float32))
