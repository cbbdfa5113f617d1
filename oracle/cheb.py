"""Interpolation nodes and Lagrange bases (Section 2.2) -- FP64 oracle.

Test infrastructure only.

* Nodes ("cheb", the default): the Chebyshev points cos((2k-1)pi/(2p)),
  k = 1..p (Section 2.2), indexed here from 0: s_m = cos((2m+1)pi/(2n)),
  m = 0..n-1.
* Nodes ("uniform"): the equally spaced points (k-1)/(p-1), k = 1..p, of
  Section 2.2, on the cell's [-1, 1] frame: s_m = -1 + 2m/(n-1) (both ends
  of the interval are nodes).
* 1D basis (Definition 2.2): l_m(x) = prod_{k != m} (x - s_k)/(s_m - s_k),
  evaluated in this product form.
* 3D basis (Definition 2.2): the product of three 1D factors.  Node i of the
  n x n x n grid has 3D index (i1, i2, i3) with i = i1 + n*i2 + n^2*i3
  (x fastest) -- the reading taken of the garbled index map in Section 2.2.
"""
from __future__ import annotations

import numpy as np


def nodes(n: int, kind: str = "cheb") -> np.ndarray:
    m = np.arange(n, dtype=np.float64)
    if kind == "uniform":
        return -1.0 + 2.0 * m / (n - 1)
    if kind != "cheb":
        raise ValueError(f"unknown node kind {kind!r}")
    return np.cos((2.0 * m + 1.0) * np.pi / (2.0 * n))


def lagrange_1d(n: int, x, kind: str = "cheb") -> np.ndarray:
    """Array of shape x.shape + (n,) holding l_m(x) for m = 0..n-1."""
    s = nodes(n, kind)
    x = np.asarray(x, dtype=np.float64)
    out = np.ones(x.shape + (n,), dtype=np.float64)
    for m in range(n):
        for k in range(n):
            if k != m:
                out[..., m] *= (x - s[k]) / (s[m] - s[k])
    return out


def grid_nodes(n: int, kind: str = "cheb") -> np.ndarray:
    """The n^3 tensor nodes (x*_{i1}, x*_{i2}, x*_{i3}) as an (n^3, 3) array,
    row i = i1 + n*i2 + n^2*i3."""
    s = nodes(n, kind)
    i = np.arange(n ** 3)
    return np.stack([s[i % n], s[(i // n) % n], s[i // (n * n)]], axis=1)


def lagrange_3d(n: int, xi, kind: str = "cheb") -> np.ndarray:
    """L_p(x*_i, xi) for every node i: shape xi.shape[:-1] + (n^3,)."""
    xi = np.asarray(xi, dtype=np.float64)
    lx = lagrange_1d(n, xi[..., 0], kind)
    ly = lagrange_1d(n, xi[..., 1], kind)
    lz = lagrange_1d(n, xi[..., 2], kind)
    prod = (lz[..., :, None, None] * ly[..., None, :, None]
            * lx[..., None, None, :])
    return prod.reshape(xi.shape[:-1] + (n ** 3,))


def child_node_positions(n: int, octant: int, kind: str = "cheb") -> np.ndarray:
    """Nodes of child ``octant`` expressed in its parent's [-1,1]^3 frame.

    A child of half-width h/2 is centred at the parent centre shifted by
    -h/2 (bit 0) or +h/2 (bit 1) on each axis, so its node s_j sits at
    (2*bit - 1)/2 + s_j/2 in parent coordinates.  Octant bits: x = bit 0,
    y = bit 1, z = bit 2 (the Morton order of the tree)."""
    g = grid_nodes(n, kind)
    shift = np.array([(octant >> d) & 1 for d in range(3)], dtype=np.float64)
    return (2.0 * shift - 1.0) / 2.0 + g / 2.0


def m2m_matrix(n: int, octant: int, kind: str = "cheb") -> np.ndarray:
    """Dense n^3 x n^3 M2M operator of child ``octant`` (Section 2.3, upward
    pass): entry [i, j] = L_p(y*_i of the parent, y*_j of the child), i.e.
    the parent's 3D Lagrange basis evaluated at the child's nodes."""
    return lagrange_3d(n, child_node_positions(n, octant, kind), kind).T.copy()
