"""M2L operators and their SVD compression -- FP64 oracle.

Test infrastructure only.

Section 2.3 (M2L) and eq. (3): the far-field interaction of cells a and b uses
the kernel sampled at their Chebyshev nodes, K(x*_i, y*_j).  By translation
invariance only the transfer vector t = k(b) - k(a) matters, so each level
has 316 operators (Section 2.3, memory footprint):

    K_t[i, j] = K(h s_i, h (2 t + s_j)),   h = half-width of the level,

with s_i the 3D Chebyshev node i of [-1,1]^3 (target cell centred at 0,
source cell centred at 2 h t).

Homogeneous kernels (Section 2.5): K(c x, c y) = c^m K(x, y); the operators
are built once for h = 1 and scaled by h^m on each level (1/r: m = -1; the
dipole kernel (x_1 - y_1)/|x - y|^3: m = -2).

Symmetry and skew-symmetry (Section 2.5): K(y, x) = +K(x, y) or -K(x, y).
Then K_{-t} = +K_t^T or -K_t^T, and the compressed operators obey the same
relation in the reconstructed form U C_{-t} V^T = +-(U C_t V^T)^T.

SVD compression (Section 2.5, "Fast M2L translation"; details follow the
Fong-Darve construction the paper cites).  Reading taken here:
  K_fat  = [K_t1, K_t2, ...]     (n^3 x 316 n^3)
  K_thin = [K_t1; K_t2; ...]     (316 n^3 x n^3)
  k      = max(#{s_i(K_fat)  > eps s_1(K_fat)},
               #{s_i(K_thin) > eps s_1(K_thin)}),  at least 1
  U      = leading k left singular vectors of K_fat
  V      = leading k right singular vectors of K_thin
  C_t    = U^T K_t V      (k x k)
so that K_t ~ U C_t V^T.  eps = 0 disables compression (U = V = I, C_t = K_t).
The SVD itself is LAPACK's (numpy.linalg.svd), used as a library step.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Optional

import numpy as np

from . import cheb
from ._native import kernel_values
from .tree import Tree, transfer_vectors

HOMOGENEOUS_DEGREE = {0: -1, 3: -2}     # 1/r: -1, dipole (x_1 - y_1)/r^3: -2
# K(y, x) = SYMMETRY * K(x, y): +1 symmetric, -1 skew-symmetric, 0 neither
SYMMETRY = {0: 1, 1: 1, 2: 1, 3: -1, 100: 0}


@dataclasses.dataclass
class LevelOps:
    k: int
    U: np.ndarray        # (m, k)
    V: np.ndarray        # (m, k)
    C: np.ndarray        # (316, k, k), already scaled for this level
    sv_fat: Optional[np.ndarray] = None
    sv_thin: Optional[np.ndarray] = None


@dataclasses.dataclass
class Ops:
    n: int
    eps: float
    kernel_id: int
    kernel_param: float
    levels: Dict[int, LevelOps]
    nodes: str = "cheb"          # interpolation nodes: "cheb" or "uniform"


def sample_m2l(kernel_id: int, param: float, n: int, h: float,
               nodes: str = "cheb") -> np.ndarray:
    """All 316 K_t at half-width h: array (316, n^3, n^3)."""
    g = cheb.grid_nodes(n, nodes)
    T = transfer_vectors().astype(np.float64)
    tgt = h * g                                        # (m, 3)
    src = h * (2.0 * T[:, None, :] + g[None, :, :])    # (316, m, 3)
    diff = tgt[None, :, None, :] - src[:, None, :, :]  # (316, m, m, 3)
    return kernel_values(diff, kernel_id, param)


def compress(K: np.ndarray, eps: float) -> LevelOps:
    nt, m, _ = K.shape
    if eps == 0.0:
        eye = np.eye(m)
        return LevelOps(m, eye, eye.copy(), K.copy())
    k_fat = K.transpose(1, 0, 2).reshape(m, nt * m)
    k_thin = K.reshape(nt * m, m)
    uf, sf, _ = np.linalg.svd(k_fat, full_matrices=False)
    _, st, vth = np.linalg.svd(k_thin, full_matrices=False)
    kf = int(np.count_nonzero(sf > eps * sf[0])) if sf[0] > 0 else 0
    kt = int(np.count_nonzero(st > eps * st[0])) if st[0] > 0 else 0
    k = max(kf, kt, 1)
    U = uf[:, :k].copy()
    V = vth[:k, :].T.copy()
    C = np.einsum("ia,tij,jb->tab", U, K, V, optimize=True)
    return LevelOps(k, U, V, C, sf, st)


def precompute(tree: Tree, kernel_id: int, param: float, n: int,
               eps: float, nodes: str = "cheb") -> Ops:
    """Operators of every level >= 2.  With equally spaced nodes ("uniform",
    Section 2.5 "Fast M2L translation") the operators stay uncompressed
    (eps is ignored): K_t is the block-Toeplitz matrix a fast method applies
    with the FFT, and the oracle applies it as the dense product."""
    levels: Dict[int, LevelOps] = {}
    if nodes == "uniform":
        eps = 0.0
    deg = HOMOGENEOUS_DEGREE.get(kernel_id)
    if deg is not None:
        base = compress(sample_m2l(kernel_id, param, n, 1.0, nodes), eps)
        for lvl in range(2, tree.depth):
            s = tree.half_width(lvl) ** deg
            levels[lvl] = LevelOps(base.k, base.U, base.V, base.C * s,
                                   base.sv_fat, base.sv_thin)
    else:
        for lvl in range(2, tree.depth):
            K = sample_m2l(kernel_id, param, n, tree.half_width(lvl), nodes)
            levels[lvl] = compress(K, eps)
    return Ops(n, eps, kernel_id, param, levels, nodes)
