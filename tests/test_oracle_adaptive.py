"""Pins of the oracle's level-adaptive tree and its U/V/W/X lists (Section
2.1 on adaptive subdivision; the list roles of the adaptive FMM).

* structure: leaves partition the points; a cell is split exactly when it
  holds more than leaf_size points (or sits above the finest level); every
  cell is a cell of the uniform tree with the same children;
* coverage: for every target leaf, U, W, and the V and X lists of the leaf
  and its ancestors reach every source leaf exactly once (brute force);
* duality: A in W(B) exactly when B in X(A);
* a cloud whose adaptive tree is the uniform tree has empty W and X lists
  and gives the uniform matvec;
* closed form: a kernel that is a polynomial of degree < n in each
  coordinate is interpolated exactly, so P2M/M2M/M2L/P2L/L2L/L2P/M2P are
  exact and the matvec is the direct sum;
* the 1/r error against the direct sum on a clustered cloud is at the level
  of the uniform tree's, with far fewer cells.
"""
import numpy as np
import pytest

import synth
from oracle import adaptive as A, fmm as F, operators as O, tree as T


def _cloud(n=3000, seed=11, r=2):
    rng = np.random.default_rng(seed)
    blob = rng.normal(0.3, 0.02, (2 * n // 3, 3))
    bg = rng.uniform(0.0, 1.0, (n - 2 * n // 3, 3))
    pts = np.concatenate([blob, bg]).astype(np.float32)
    sig = rng.uniform(-1.0, 1.0, (n, r)).astype(np.float32)
    return pts, sig


@pytest.fixture(scope="module")
def clustered():
    pts, sig = _cloud()
    return pts, sig, A.build_adaptive_tree(pts, leaf_size=32, max_depth=8)


def _leaves_under(tr, l, c):
    out, st = [], [(l, c)]
    while st:
        l, c = st.pop()
        lv = tr.levels[l]
        if lv.leaf[c]:
            out.append((l, c))
        else:
            st.extend((l + 1, k) for k in range(lv.cb[c], lv.ce[c]))
    return out


def test_structure(clustered):
    pts, _, tr = clustered
    ut = T.build_tree(pts, 32, 8)
    assert tr.depth == ut.depth
    # leaves partition the sorted points
    seen = np.zeros(len(pts), int)
    for l, c in tr.leaves:
        seen[tr.levels[l].pb[c]:tr.levels[l].pe[c]] += 1
    assert np.all(seen == 1)
    for l in range(tr.depth):
        lv = tr.levels[l]
        cnt = lv.pe - lv.pb
        assert np.all(cnt >= 1)
        if l < tr.depth - 1:
            assert np.array_equal(lv.leaf, cnt <= 32)
        else:
            assert lv.leaf.all()
        # every cell is a uniform-tree cell; non-leaves keep all their children
        pos = T.lookup(ut.levels[l].keys, lv.keys)
        assert np.all(pos >= 0)
        ul = ut.levels[l]
        for c in range(len(lv.keys)):
            if lv.leaf[c]:
                assert lv.cb[c] == lv.ce[c]
            else:
                u = pos[c]
                kids = ut.levels[l + 1].keys[ul.cb[u]:ul.ce[u]]
                assert np.array_equal(tr.levels[l + 1].keys[lv.cb[c]:lv.ce[c]], kids)
                assert np.all(tr.levels[l + 1].parent[lv.cb[c]:lv.ce[c]] == c)
    assert tr.n_cells() < sum(len(x.keys) for x in ut.levels) // 4
    assert sum(len(w) for w in tr.W) > 0 and len(tr.X) > 0


def test_lists_cover_every_source_leaf_once(clustered):
    _, _, tr = clustered
    every = sorted(map(tuple, tr.leaves.tolist()))
    for q, (l, c) in enumerate(tr.leaves):
        got = [tuple(a) for a in tr.U[q].tolist()]
        for a in tr.W[q].tolist():
            got += _leaves_under(tr, *a)
        L, C = int(l), int(c)
        while L >= 2:
            pr = tr.pairs[L]
            for s in pr["src"][pr["tgt"] == C]:
                got += _leaves_under(tr, L, int(s))
            got += [tuple(a) for a in tr.X.get((L, C), np.zeros((0, 2), int)).tolist()]
            C = int(tr.levels[L].parent[C])
            L -= 1
        assert sorted(got) == every, (l, c)


def test_w_and_x_are_dual(clustered):
    _, _, tr = clustered
    w_pairs = {(tuple(tr.leaves[q]), tuple(a)) for q in range(len(tr.leaves))
               for a in tr.W[q].tolist()}
    x_pairs = {(tuple(a), b) for b, xs in tr.X.items() for a in xs.tolist()}
    assert w_pairs == x_pairs
    # W entries lie strictly below the target's level, X entries strictly above
    for (b, a) in w_pairs:
        assert a[0] > b[0]


def test_full_tree_reduces_to_the_uniform_tree():
    pts, sig = synth.random_cloud(4096, 3, r=2)
    # leaf_size 1, four levels: every cell above the finest level is split
    tr = A.build_adaptive_tree(pts, leaf_size=1, fixed_depth=4)
    ut = T.build_tree(pts, fixed_depth=4)
    assert all(len(w) == 0 for w in tr.W) and len(tr.X) == 0
    for l in range(4):
        assert np.array_equal(tr.levels[l].keys, ut.levels[l].keys)
    ops = O.precompute(ut, 0, 1.0, 4, 1e-9)
    got = A.matvec(tr, ops, pts, sig, 0, 1.0)
    ref = F.matvec(ut, ops, pts, sig, 0, 1.0)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n", [4, 5])
def test_polynomial_kernel_is_exact(clustered, n):
    pts, sig, tr = clustered
    ops = O.precompute(tr, 100, 0.7, n, 0.0)
    got = A.matvec(tr, ops, pts, sig, 100, 0.7)
    ref = F.direct(pts, sig, 100, 0.7)
    assert F.rel_l2(got, ref) < 1e-12


def test_rows_subset(clustered):
    pts, sig, tr = clustered
    ops = O.precompute(tr, 0, 1.0, 4, 1e-6)
    rows = np.array([5, 17, 2999, 1000, 0])
    full = A.matvec(tr, ops, pts, sig, 0, 1.0)
    assert np.array_equal(A.matvec(tr, ops, pts, sig, 0, 1.0, rows=rows), full[rows])


def test_inv_r_error_matches_the_uniform_tree(clustered):
    pts, sig, tr = clustered
    ex = F.direct(pts, sig, 0, 1.0)
    ops = O.precompute(tr, 0, 1.0, 5, 1e-7)
    err = F.rel_l2(A.matvec(tr, ops, pts, sig, 0, 1.0), ex)
    ut = T.build_tree(pts, 32, 8)
    err_u = F.rel_l2(F.matvec(ut, O.precompute(ut, 0, 1.0, 5, 1e-7), pts, sig, 0, 1.0), ex)
    assert err < 2e-4 and err < 2.0 * err_u


def test_root_leaf_is_the_direct_sum():
    pts, sig = synth.random_cloud(50, 4, r=1)
    tr = A.build_adaptive_tree(pts, leaf_size=64, max_depth=5)
    assert tr.depth == 1 and len(tr.leaves) == 1
    got = A.matvec(tr, None, pts, sig, 0, 1.0)
    assert np.allclose(got, F.direct(pts, sig, 0, 1.0), rtol=1e-13, atol=1e-13)
