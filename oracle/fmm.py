"""The bbFMM matvec and the direct sum -- FP64 oracle.

Test infrastructure only.

Stages follow Section 2.3, run level by level (the level-synchronous
traversal the paper names as the alternative to task-based traversal):

  P2M (leaves)   M_a[i] = sum_{y_j in a} L_p(y*_i, y_j) sigma_j
  M2M (upward)   M_a[i] = sum_{b in C(a)} sum_j L_p(y*_i, y*_j) M_b[j]
  M2L            F_a[i] = sum_{b in I(a)} sum_j K(x*_i, y*_j) M_b[j]
                 applied in the compressed form  F_a += U sum_b C_t (V^T M_b)
  L2L (downward) F_a[i] += sum_j F_parent[j] L_p(x*_j, x*_i)
  L2P (leaves)   phi_i = sum_j F_a[j] L_p(x*_j, x_i)
  P2P (leaves)   phi_i += sum_{b in N(a)} sum_{y_j in b} K(x_i, y_j) sigma_j

Interpolation coordinates: xi = (x - c)/h with c the FP64 cell centre and h
the half-width.  M2L runs on levels >= 2 (I(.) is empty on levels 0 and 1).
With fewer than three levels everything is near field and the result is the
direct sum.

``rows`` restricts the output to a subset of targets (original indices): the
upward pass and M2L still run over every cell, while L2P and P2P are only
evaluated for the requested targets.

Separate target and source sets (eq. (1) distinguishes targets x_i from
sources y_j): the tree is built over the union of both sets, targets first
(``n_targets`` of them), and each stage sums over sources only (P2M and the
near field) and evaluates at targets only (L2P and the near field).
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import cheb
from ._native import direct_sum
from .operators import Ops
from .tree import Tree


def direct(points: np.ndarray, sigma: np.ndarray, kernel_id: int,
           param: float, rows: Optional[np.ndarray] = None,
           sources: Optional[np.ndarray] = None) -> np.ndarray:
    """Exact phi = K sigma (eq. (2)) in FP64, for all rows or a subset.
    With ``sources`` given, ``points`` are the targets and sigma belongs to
    the sources (eq. (1) with separate sets)."""
    pts = np.asarray(points, dtype=np.float32).astype(np.float64)
    src = pts if sources is None else np.asarray(sources, np.float32).astype(np.float64)
    sig = _as_2d(sigma)
    tgt = pts if rows is None else pts[np.asarray(rows)]
    return direct_sum(tgt, src, sig, kernel_id, param)


def _left(A: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Y[c, i, r] = sum_j A[i, j] X[c, j, r], evaluated as one matrix product."""
    c, j, r = X.shape
    Y = A @ X.transpose(1, 0, 2).reshape(j, c * r)
    return np.ascontiguousarray(Y.reshape(A.shape[0], c, r).transpose(1, 0, 2))


def _as_2d(sigma) -> np.ndarray:
    s = np.asarray(sigma, dtype=np.float64)
    return s[:, None] if s.ndim == 1 else s


def upward(tree: Tree, ops: Ops, Y: np.ndarray, S: np.ndarray,
           is_src: Optional[np.ndarray] = None) -> dict:
    """Multipole coefficients M[level] of shape (cells, n^3, r), levels >= 2,
    from the sources (``is_src``: which sorted points are sources; all by
    default)."""
    n = ops.n
    L = tree.leaf_level
    leaf = tree.levels[L]
    cL = tree.centers(L)
    hL = tree.half_width(L)
    M = {}
    ML = np.zeros((len(leaf.keys), n ** 3, S.shape[1]))
    for a in range(len(leaf.keys)):
        j = np.arange(leaf.pb[a], leaf.pe[a])
        if is_src is not None:
            j = j[is_src[j]]
        Sa = cheb.lagrange_3d(n, (Y[j] - cL[a]) / hL, ops.nodes)   # (sources, n^3)
        ML[a] = Sa.T @ S[j]
    M[L] = ML
    T3 = [cheb.m2m_matrix(n, o, ops.nodes) for o in range(8)]
    for lvl in range(L - 1, 1, -1):
        child = tree.levels[lvl + 1]
        Mp = np.zeros((len(tree.levels[lvl].keys), n ** 3, S.shape[1]))
        octant = (child.keys & np.uint64(7)).astype(np.int64)
        for o in range(8):
            sel = np.nonzero(octant == o)[0]
            # a parent has at most one child per octant: no repeated index
            Mp[child.parent[sel]] += _left(T3[o], M[lvl + 1][sel])
        M[lvl] = Mp
    return M


def m2l(tree: Tree, ops: Ops, M: dict) -> dict:
    """Local coefficients from the interaction lists, F[level] (cells, n^3, r)."""
    F = {}
    for lvl in range(2, tree.depth):
        op = ops.levels[lvl]
        Mh = _left(op.V.T, M[lvl])
        Fh = np.zeros_like(Mh)
        pr = tree.pairs[lvl]
        g = pr["group_off"]
        for ti in range(len(g) - 1):
            s, e = g[ti], g[ti + 1]
            if s == e:
                continue
            # within one transfer vector each target occurs at most once
            Fh[pr["tgt"][s:e]] += _left(op.C[ti], Mh[pr["src"][s:e]])
        F[lvl] = _left(op.U, Fh)
    return F


def downward(tree: Tree, ops: Ops, F: dict) -> dict:
    """Adds the parents' local coefficients into every level >= 3 (L2L)."""
    n = ops.n
    T3 = [cheb.m2m_matrix(n, o, ops.nodes) for o in range(8)]
    for lvl in range(3, tree.depth):
        child = tree.levels[lvl]
        octant = (child.keys & np.uint64(7)).astype(np.int64)
        for o in range(8):
            sel = np.nonzero(octant == o)[0]
            F[lvl][sel] += _left(T3[o].T, F[lvl - 1][child.parent[sel]])
    return F


def matvec(tree: Tree, ops: Optional[Ops], points: np.ndarray,
           sigma: np.ndarray, kernel_id: int, param: float,
           rows: Optional[np.ndarray] = None, near: bool = True,
           far: bool = True, n_targets: Optional[int] = None) -> np.ndarray:
    """phi ~ K sigma by the bbFMM; returns (len(rows) or N, r) in FP64.

    n_targets: the tree was built over [targets; sources] and the first
    n_targets points are the targets; sigma then has one row per source
    and the result one row per target (rows index the targets)."""
    pts = np.asarray(points, dtype=np.float32).astype(np.float64)
    sig = _as_2d(sigma)
    N = len(pts)
    r = sig.shape[1]
    nt = N if n_targets is None else int(n_targets)
    is_src = np.ones(N, bool) if n_targets is None else np.arange(N) >= nt
    if n_targets is None:
        assert sig.shape[0] == N
        sig_all = sig
    else:
        assert sig.shape[0] == N - nt
        sig_all = np.zeros((N, r))
        sig_all[nt:] = sig          # the sources' weights; targets carry none
    L = tree.leaf_level
    Y = pts[tree.perm]
    S = sig_all[tree.perm]
    src_sorted = is_src[tree.perm]
    leaf = tree.levels[L]

    inv = np.empty(N, np.int64)
    inv[tree.perm] = np.arange(N)
    want = np.arange(nt) if rows is None else np.asarray(rows)
    assert np.all(want < nt)
    want_pos = inv[want]
    leaf_of = np.searchsorted(leaf.pb, want_pos, side="right") - 1
    out = np.zeros((len(want_pos), r))

    if far and L >= 2:
        n = ops.n
        M = upward(tree, ops, Y, S, src_sorted)
        F = downward(tree, ops, m2l(tree, ops, M))
        cL = tree.centers(L)
        hL = tree.half_width(L)
        xi = (Y[want_pos] - cL[leaf_of]) / hL
        Sx = cheb.lagrange_3d(n, xi, ops.nodes)            # (targets, n^3)
        out += np.matmul(Sx[:, None, :], F[L][leaf_of])[:, 0, :]

    if near:
        order = np.argsort(leaf_of, kind="stable")
        lo_s = leaf_of[order]
        starts = np.nonzero(np.r_[True, lo_s[1:] != lo_s[:-1]])[0]
        ends = np.r_[starts[1:], len(lo_s)]
        for s, e in zip(starts, ends):
            a = lo_s[s]
            nb = tree.nbr_idx[tree.nbr_off[a]:tree.nbr_off[a + 1]]
            src = np.concatenate([np.arange(leaf.pb[b], leaf.pe[b]) for b in nb])
            src = src[src_sorted[src]]
            sel = order[s:e]
            out[sel] += direct_sum(Y[want_pos[sel]], Y[src], S[src], kernel_id,
                                   param)
    return out


def rel_l2(approx: np.ndarray, exact: np.ndarray) -> float:
    """||approx - exact||_2 / ||exact||_2 (Section 4.1), over all entries."""
    return float(np.linalg.norm(approx - exact) / np.linalg.norm(exact))


def rel_l2_cols(approx: np.ndarray, exact: np.ndarray) -> np.ndarray:
    """The same error per right-hand side (column)."""
    return np.linalg.norm(approx - exact, axis=0) / np.linalg.norm(exact, axis=0)
