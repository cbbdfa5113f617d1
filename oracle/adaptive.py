"""Level-adaptive octree, its U/V/W/X lists and the bbFMM matvec over it --
FP64/integer oracle.

Test infrastructure only.

Section 2.1 notes that the recursive subdivision (split a cell until it holds
no more than a prescribed number of points) generally gives a non-uniform
tree; the uniform tree trades that for simpler parallelism and pays for cells
holding few points.  This module is the adaptive form.

Readings taken:
  * The tree is the uniform tree of the same point set (same bounding cube,
    binning, depth rule and point order) with every cell that holds at most
    ``leaf_size`` points made a leaf and its descendants removed.  The
    finest level keeps the uniform tree's leaf level, so a cell on it is a
    leaf whatever its count; trailing levels left without cells are dropped.
    Every cell is a contiguous range of the sorted points, and the cells of
    each level stay in ascending key order.
  * Cells A and B are adjacent when their closed boxes touch or overlap (on
    any level pair).  The lists are the standard ones of the adaptive FMM
    (Greengard-Rokhlin / the kernel-independent FMM), stated for the
    interpolation-based expansions of Section 2.3:
      U(B), B a leaf : leaves A adjacent to B (B included)      -> P2P
      V(B), any cell : same-level cells A whose parent is adjacent to
                       parent(B) and that are not adjacent to B
                       (Definition 2.1's interaction list)        -> M2L
      W(B), B a leaf : cells A finer than B, not adjacent to B,
                       whose parent is adjacent to B              -> M2P
      X(B), any cell : leaves A coarser than B, not adjacent to B,
                       adjacent to parent(B)  (B in W(A))         -> P2L
  * M2P: phi(x) += sum_m K(x, y*_m) M_A[m] over the Chebyshev nodes y*_m of A
    (the multipole coefficients act as charges at the nodes, eq. (3)).
    P2L: F_B[m] += sum_{y_j in A} K(x*_m, y_j) sigma_j (the local
    coefficients are the field at B's nodes, eq. (3)).
  * Expansions (M, F) exist on levels >= 2 only, as in the uniform tree; a
    leaf on level 0 or 1 has only U and W lists, and no cell below level 2
    has V or X entries.
  * Adaptive trees take a single point set (targets = sources).
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import numpy as np

from . import cheb
from ._native import direct_sum
from .operators import Ops
from .tree import Tree, build_tree, interaction_pairs


@dataclasses.dataclass
class ALevel:
    keys: np.ndarray     # uint64, ascending
    coords: np.ndarray   # (C,3) int64
    pb: np.ndarray       # first point (sorted order)
    pe: np.ndarray       # one past the last point
    parent: np.ndarray   # index into the level above (-1 at the root)
    cb: np.ndarray       # first child on the level below (cb == ce for a leaf)
    ce: np.ndarray
    leaf: np.ndarray     # bool


@dataclasses.dataclass
class ATree:
    lo: np.ndarray
    side: np.float32
    depth: int                    # levels 0..depth-1
    perm: np.ndarray
    levels: List[ALevel]
    pairs: Dict[int, dict]        # V lists per level >= 2 (Tree.pairs layout)
    leaves: np.ndarray            # (NL, 2): (level, cell) of every leaf, by
                                  # level then cell index
    U: List[np.ndarray]           # per leaf: (k, 2) (level, cell), sorted
    W: List[np.ndarray]           # per leaf: (k, 2)
    X: Dict[tuple, np.ndarray]    # (level, cell) -> (k, 2) leaves, sorted

    def half_width(self, level: int) -> float:
        return float(self.side) / 2.0 ** (level + 1)

    def centers(self, level: int) -> np.ndarray:
        w = float(self.side) / 2.0 ** level
        return self.lo.astype(np.float64)[None, :] + (self.levels[level].coords + 0.5) * w

    def box(self, level: int, cell: int):
        """Integer box [lo, hi] (closed) of a cell in units of the finest level."""
        f = self.depth - 1
        lo = self.levels[level].coords[cell] << (f - level)
        return lo, lo + (1 << (f - level))

    def n_cells(self) -> int:
        return sum(len(lv.keys) for lv in self.levels)


def build_adaptive_tree(points: np.ndarray, leaf_size: int = 64, max_depth: int = 22,
                        fixed_depth: int = 0) -> ATree:
    ut: Tree = build_tree(points, leaf_size, max_depth, fixed_depth)
    D = ut.depth
    F = D - 1
    keep = [np.ones(1, bool)]
    leaf = []
    for lvl in range(D):
        lv = ut.levels[lvl]
        cnt = lv.pe - lv.pb
        lf = (cnt <= leaf_size) | (lvl == F)
        leaf.append(lf)
        if lvl < F:
            child = ut.levels[lvl + 1]
            keep.append(keep[lvl][child.parent] & ~lf[child.parent])
    # levels left without cells (every cell above them a leaf) are dropped
    while D > 1 and not keep[D - 1].any():
        D -= 1
    F = D - 1
    levels: List[ALevel] = []
    new_index = []
    for lvl in range(D):
        lv = ut.levels[lvl]
        idx = np.nonzero(keep[lvl])[0]
        m = np.full(len(lv.keys), -1, np.int64)
        m[idx] = np.arange(len(idx))
        new_index.append(m)
        levels.append(ALevel(lv.keys[idx], lv.coords[idx], lv.pb[idx], lv.pe[idx],
                             lv.parent[idx].copy(), np.zeros(len(idx), np.int64),
                             np.zeros(len(idx), np.int64), leaf[lvl][idx]))
    for lvl in range(1, D):
        levels[lvl].parent = new_index[lvl - 1][levels[lvl].parent]
    for lvl in range(D):
        a = levels[lvl]
        if lvl < F:
            ch = levels[lvl + 1]
            # children are a contiguous run on the level below (ascending keys)
            first = np.searchsorted(ch.parent, np.arange(len(a.keys)), side="left")
            last = np.searchsorted(ch.parent, np.arange(len(a.keys)), side="right")
            a.cb, a.ce = first.astype(np.int64), last.astype(np.int64)
        else:
            a.cb = np.zeros(len(a.keys), np.int64)
            a.ce = np.zeros(len(a.keys), np.int64)
    tr = ATree(ut.lo, ut.side, D, ut.perm, levels, {}, None, [], [], {})  # type: ignore
    for lvl in range(2, D):
        tr.pairs[lvl] = interaction_pairs(tr, lvl)  # same-level lists, Definition 2.1
    tr.leaves = np.array([(l, c) for l in range(D) for c in np.nonzero(levels[l].leaf)[0]],
                         dtype=np.int64).reshape(-1, 2)
    _build_lists(tr)
    return tr


def _build_lists(tr: ATree) -> None:
    """U, W per leaf and X per cell, straight from their definitions by
    testing every pair of cells (quadratic: small trees only)."""
    D = tr.depth
    lev = np.concatenate([np.full(len(tr.levels[l].keys), l, np.int64) for l in range(D)])
    idx = np.concatenate([np.arange(len(tr.levels[l].keys), dtype=np.int64) for l in range(D)])
    base = np.cumsum([0] + [len(tr.levels[l].keys) for l in range(D)])
    lo = np.array([tr.box(l, c)[0] for l, c in zip(lev, idx)]).reshape(-1, 3)
    hi = lo + (1 << (D - 1 - lev))[:, None]
    par = np.array([base[l - 1] + tr.levels[l].parent[c] if l > 0 else -1
                    for l, c in zip(lev, idx)], np.int64)
    is_leaf = np.concatenate([tr.levels[l].leaf for l in range(D)])

    def adj(g):            # every cell against cell g: closed boxes touch or overlap
        return np.all(lo <= hi[g], axis=1) & np.all(lo[g] <= hi, axis=1)

    def pairs(mask):
        sel = np.nonzero(mask)[0]
        return np.stack([lev[sel], idx[sel]], axis=1)

    for l, c in tr.leaves:
        g = base[l] + c
        a_b = adj(g)
        tr.U.append(pairs(is_leaf & a_b))
        # W: cells finer than b, not adjacent to b, with a parent adjacent to b
        p_adj = np.zeros(len(lev), bool)
        has_p = par >= 0
        p_adj[has_p] = a_b[par[has_p]]
        tr.W.append(pairs((lev > l) & ~a_b & p_adj))
    for g in range(len(lev)):
        if lev[g] == 0:
            continue
        m = is_leaf & (lev < lev[g]) & ~adj(g) & adj(par[g])
        if m.any():
            tr.X[(int(lev[g]), int(idx[g]))] = pairs(m)


def _nodes(tr: ATree, n: int, kind: str, level: int, cell: int) -> np.ndarray:
    return tr.centers(level)[cell] + tr.half_width(level) * cheb.grid_nodes(n, kind)


def _points(tr: ATree, level: int, cell: int) -> np.ndarray:
    lv = tr.levels[level]
    return np.arange(lv.pb[cell], lv.pe[cell])


def matvec(tr: ATree, ops: Optional[Ops], points: np.ndarray, sigma: np.ndarray,
           kernel_id: int, param: float, rows: Optional[np.ndarray] = None,
           near: bool = True, far: bool = True) -> np.ndarray:
    """phi ~ K sigma over the adaptive tree, FP64; (len(rows) or N, r).
    near / far: include the U-list direct sums / everything else."""
    pts = np.asarray(points, dtype=np.float32).astype(np.float64)
    sig = np.asarray(sigma, dtype=np.float64)
    sig = sig[:, None] if sig.ndim == 1 else sig
    N, r = len(pts), sig.shape[1]
    Y = pts[tr.perm]
    S = sig[tr.perm]
    D = tr.depth
    n = ops.n if ops is not None else 0
    kind = ops.nodes if ops is not None else "cheb"
    T3 = [cheb.m2m_matrix(n, o, kind) for o in range(8)] if n else []

    # upward: P2M at leaves, M2M at the other cells (Section 2.3)
    M: Dict[int, np.ndarray] = {}
    for lvl in range(D - 1, 1, -1):
        lv = tr.levels[lvl]
        Ml = np.zeros((len(lv.keys), n ** 3, r))
        c_l, h_l = tr.centers(lvl), tr.half_width(lvl)
        for a in range(len(lv.keys)):
            if lv.leaf[a]:
                j = _points(tr, lvl, a)
                Sa = cheb.lagrange_3d(n, (Y[j] - c_l[a]) / h_l, kind)
                Ml[a] = Sa.T @ S[j]
            else:
                ch = tr.levels[lvl + 1]
                for b in range(lv.cb[a], lv.ce[a]):
                    Ml[a] += T3[int(ch.keys[b] & np.uint64(7))] @ M[lvl + 1][b]
        M[lvl] = Ml

    # M2L over V (compressed, as on the uniform tree), then P2L over X
    Fl: Dict[int, np.ndarray] = {}
    for lvl in range(2, D):
        lv = tr.levels[lvl]
        op = ops.levels[lvl]
        Mh = np.einsum("ik,cir->ckr", op.V, M[lvl])
        Fh = np.zeros_like(Mh)
        pr = tr.pairs[lvl]
        g = pr["group_off"]
        for ti in range(len(g) - 1):
            for e in range(g[ti], g[ti + 1]):
                Fh[pr["tgt"][e]] += op.C[ti] @ Mh[pr["src"][e]]
        Fl[lvl] = np.einsum("ik,ckr->cir", op.U, Fh)
        for a in range(len(lv.keys)):
            for (la, ca) in tr.X.get((lvl, a), np.zeros((0, 2), np.int64)):
                j = _points(tr, int(la), int(ca))
                Fl[lvl][a] += direct_sum(_nodes(tr, n, kind, lvl, a), Y[j], S[j],
                                         kernel_id, param)
    # downward: L2L (levels >= 3)
    for lvl in range(3, D):
        lv = tr.levels[lvl]
        for a in range(len(lv.keys)):
            Fl[lvl][a] += T3[int(lv.keys[a] & np.uint64(7))].T @ Fl[lvl - 1][lv.parent[a]]

    # leaves: L2P, M2P over W, P2P over U
    out_sorted = np.zeros((N, r))
    for q, (lvl, b) in enumerate(tr.leaves):
        lvl, b = int(lvl), int(b)
        i = _points(tr, lvl, b)
        if len(i) == 0:
            continue
        if far and lvl >= 2:
            Sx = cheb.lagrange_3d(n, (Y[i] - tr.centers(lvl)[b]) / tr.half_width(lvl), kind)
            out_sorted[i] += Sx @ Fl[lvl][b]
        for (la, ca) in (tr.W[q] if far else []):
            out_sorted[i] += direct_sum(Y[i], _nodes(tr, n, kind, int(la), int(ca)),
                                        M[int(la)][int(ca)], kernel_id, param)
        if near:
            src = np.concatenate([_points(tr, int(la), int(ca)) for la, ca in tr.U[q]])
            out_sorted[i] += direct_sum(Y[i], Y[src], S[src], kernel_id, param)
    out = np.empty((N, r))
    out[tr.perm] = out_sorted
    return out if rows is None else out[np.asarray(rows)]
