"""Octree, neighbour lists and interaction lists -- FP64/integer oracle.

Test infrastructure only.

Section 2.1: the cubical domain is split into eight children recursively; the
tree is uniform (all leaves on one level) and empty cells are skipped.
Definition 2.1: N(a) = same-level cells adjacent to a, a included;
I(a) = children of N(parent(a)) that are not in N(a).

Readings taken where the paper leaves the choice open:
  * domain = tight bounding cube anchored at the per-axis minimum, side =
    largest extent (1 when every point coincides);
  * binning in float32 exactly as the GPU does it: q_d = floor((x_d - lo_d) *
    scale) with scale = 2^21 / side computed once in float32, clamped to
    [0, 2^21 - 1]; the level-l cell coordinate is q_d >> (21 - l);
  * levels are counted from the root (level 0); "depth D" means levels
    0..D-1, leaf level L = D - 1;
  * depth rule: a fixed depth when one is given, else the smallest D whose
    largest leaf holds at most leaf_size points, capped by max_depth;
  * Morton key: bit b of k_x -> bit 3b, of k_y -> 3b+1, of k_z -> 3b+2;
    the child octant is key & 7;
  * points are ordered by a stable sort of the leaf key (ties keep the
    input order); cells of every level are stored in ascending key order;
  * transfer vector t = k(source) - k(target); the 316 vectors of
    {-3..3}^3 minus {-1..1}^3 (Section 2.3, memory footprint) are numbered
    by ascending (tx+3) + 7(ty+3) + 49(tz+3).
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List

import numpy as np

QBITS = 21
NQ = 1 << QBITS


def transfer_vectors() -> np.ndarray:
    """The 316 M2L transfer vectors, shape (316, 3), in compact-index order."""
    out = []
    for tz in range(-3, 4):
        for ty in range(-3, 4):
            for tx in range(-3, 4):
                if max(abs(tx), abs(ty), abs(tz)) >= 2:
                    out.append((tx, ty, tz))
    return np.array(out, dtype=np.int64)


def bounding_cube(points: np.ndarray):
    """(lo (3,) float32, side float32, scale float32)."""
    p = np.asarray(points, dtype=np.float32)
    lo = p.min(axis=0)
    hi = p.max(axis=0)
    ext = (hi - lo).astype(np.float32)
    side = np.float32(ext.max())
    if not side > 0:
        side = np.float32(1.0)
    scale = np.float32(np.float32(NQ) / side)
    return lo.astype(np.float32), side, scale


def quantize(points: np.ndarray, lo: np.ndarray, scale: np.float32) -> np.ndarray:
    """Integer coordinates q (N,3) in [0, 2^21): float32 subtract, float32
    multiply (each correctly rounded, no fused multiply-add), floor, clamp."""
    p = np.asarray(points, dtype=np.float32)
    d = (p - lo[None, :]).astype(np.float32)
    v = (d * np.float32(scale)).astype(np.float32)
    q = np.floor(v).astype(np.int64)
    return np.clip(q, 0, NQ - 1)


def morton(k: np.ndarray, bits: int) -> np.ndarray:
    """Interleave (k_x, k_y, k_z) (…,3) into a uint64 key."""
    k = np.asarray(k, dtype=np.uint64)
    key = np.zeros(k.shape[:-1], dtype=np.uint64)
    for b in range(bits):
        for d in range(3):
            bit = (k[..., d] >> np.uint64(b)) & np.uint64(1)
            key |= bit << np.uint64(3 * b + d)
    return key


def decode(keys: np.ndarray, bits: int) -> np.ndarray:
    """Inverse of ``morton``: (…,) uint64 -> (…,3) int64."""
    keys = np.asarray(keys, dtype=np.uint64)
    out = np.zeros(keys.shape + (3,), dtype=np.int64)
    for b in range(bits):
        for d in range(3):
            bit = (keys >> np.uint64(3 * b + d)) & np.uint64(1)
            out[..., d] |= bit.astype(np.int64) << b
    return out


def lookup(sorted_keys: np.ndarray, query: np.ndarray) -> np.ndarray:
    """Index of each query key in ``sorted_keys`` or -1 if absent."""
    pos = np.searchsorted(sorted_keys, query)
    pos_c = np.minimum(pos, max(len(sorted_keys) - 1, 0))
    hit = (pos < len(sorted_keys)) & (sorted_keys[pos_c] == query)
    return np.where(hit, pos_c, -1)


def depth_rule(q: np.ndarray, leaf_size: int, max_depth: int) -> int:
    for depth in range(1, max_depth + 1):
        lvl = depth - 1
        keys = morton(q >> (QBITS - lvl), lvl)
        _, counts = np.unique(keys, return_counts=True)
        if counts.max() <= leaf_size:
            return depth
    return max_depth


@dataclasses.dataclass
class Level:
    keys: np.ndarray     # uint64, ascending
    coords: np.ndarray   # (C,3) int64 cell coordinates at this level
    pb: np.ndarray       # first point (sorted order)
    pe: np.ndarray       # one past the last point
    parent: np.ndarray   # index into level-1 (-1 at the root)
    cb: np.ndarray       # first child (index into level+1), -1 on the leaf level
    ce: np.ndarray       # one past the last child


@dataclasses.dataclass
class Tree:
    lo: np.ndarray
    side: np.float32
    scale: np.float32
    depth: int
    perm: np.ndarray             # sorted position -> original index
    levels: List[Level]
    nbr_off: np.ndarray          # leaf neighbour CSR offsets (C_L + 1)
    nbr_idx: np.ndarray          # leaf neighbour indices (ascending per row)
    pairs: Dict[int, dict]       # level -> {t, tgt, src, group_off (317)}

    @property
    def leaf_level(self) -> int:
        return self.depth - 1

    def half_width(self, level: int) -> float:
        return float(self.side) / 2.0 ** (level + 1)

    def centers(self, level: int) -> np.ndarray:
        """Cell centres lo + (k + 1/2) * side / 2^level in float64."""
        w = float(self.side) / 2.0 ** level
        return self.lo.astype(np.float64)[None, :] + (self.levels[level].coords + 0.5) * w


def _unique_runs(keys: np.ndarray):
    """Start index and length of each run of equal values in a sorted array."""
    if len(keys) == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    head = np.ones(len(keys), dtype=bool)
    head[1:] = keys[1:] != keys[:-1]
    starts = np.nonzero(head)[0]
    ends = np.append(starts[1:], len(keys))
    return starts, ends - starts


def build_tree(points: np.ndarray, leaf_size: int = 64, max_depth: int = 22,
               fixed_depth: int = 0) -> Tree:
    points = np.asarray(points, dtype=np.float32)
    if points.ndim != 2 or points.shape[1] != 3 or points.shape[0] < 1:
        raise ValueError("points must be (N>=1, 3)")
    if not np.all(np.isfinite(points)):
        raise ValueError("non-finite coordinate")
    if not 1 <= max_depth <= 22:
        raise ValueError("max_depth must be in [1, 22]")
    lo, side, scale = bounding_cube(points)
    q = quantize(points, lo, scale)
    depth = fixed_depth if fixed_depth > 0 else depth_rule(q, leaf_size, max_depth)
    if not 1 <= depth <= 22:
        raise ValueError("depth must be in [1, 22]")
    L = depth - 1
    leaf_key = morton(q >> (QBITS - L), L)
    perm = np.argsort(leaf_key, kind="stable")
    skeys = leaf_key[perm]

    levels: List[Level] = [None] * depth  # type: ignore
    starts, counts = _unique_runs(skeys)
    keys_L = skeys[starts]
    levels[L] = Level(keys_L, decode(keys_L, L), starts, starts + counts,
                      np.full(len(keys_L), -1, np.int64),
                      np.full(len(keys_L), -1, np.int64),
                      np.full(len(keys_L), -1, np.int64))
    for lvl in range(L - 1, -1, -1):
        child = levels[lvl + 1]
        pk = child.keys >> np.uint64(3)
        cst, ccnt = _unique_runs(pk)
        keys = pk[cst]
        parent_of_child = np.repeat(np.arange(len(keys)), ccnt)
        child.parent = parent_of_child.astype(np.int64)
        cb = cst.astype(np.int64)
        ce = (cst + ccnt).astype(np.int64)
        levels[lvl] = Level(keys, decode(keys, lvl), child.pb[cb], child.pe[ce - 1],
                            np.full(len(keys), -1, np.int64), cb, ce)

    tree = Tree(lo, side, scale, depth, perm, levels, None, None, {})  # type: ignore
    tree.nbr_off, tree.nbr_idx = leaf_neighbors(tree)
    for lvl in range(2, depth):
        tree.pairs[lvl] = interaction_pairs(tree, lvl)
    return tree


def leaf_neighbors(tree: Tree):
    """CSR of N(a) on the leaf level: occupied leaves b with max|k_b - k_a| <= 1
    (a itself included), ascending cell index within each row."""
    L = tree.leaf_level
    lev = tree.levels[L]
    C = len(lev.keys)
    rows, cols = [], []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                kb = lev.coords + np.array([dx, dy, dz])
                ok = np.all((kb >= 0) & (kb < (1 << L)), axis=1)
                idx = np.full(C, -1, np.int64)
                idx[ok] = lookup(lev.keys, morton(kb[ok], L))
                hit = idx >= 0
                rows.append(np.nonzero(hit)[0])
                cols.append(idx[hit])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    off = np.zeros(C + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=C), out=off[1:])
    return off, cols.astype(np.int64)


def interaction_pairs(tree: Tree, lvl: int) -> dict:
    """Pairs (target a, source b, t) with b in I(a) at level ``lvl``, grouped by
    transfer vector (ascending compact index), ascending target within a group."""
    lev = tree.levels[lvl]
    T = transfer_vectors()
    tt, tg, sr = [], [], []
    off = np.zeros(len(T) + 1, np.int64)
    for ti, t in enumerate(T):
        kb = lev.coords + t[None, :]
        inb = np.all((kb >= 0) & (kb < (1 << lvl)), axis=1)
        padj = np.all(np.abs((kb >> 1) - (lev.coords >> 1)) <= 1, axis=1)
        cand = np.nonzero(inb & padj)[0]
        src = lookup(lev.keys, morton(kb[cand], lvl))
        hit = src >= 0
        tg.append(cand[hit])
        sr.append(src[hit])
        tt.append(np.full(hit.sum(), ti, np.int64))
        off[ti + 1] = off[ti] + hit.sum()
    return {"t": np.concatenate(tt), "tgt": np.concatenate(tg),
            "src": np.concatenate(sr), "group_off": off}
