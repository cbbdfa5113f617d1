"""Truncated eigendecomposition of a kernel (covariance) matrix with the
randomized algorithm the paper accelerates in its geostatistics application
(Section 4: the top-k eigenpairs from two block products with l = k +
oversampling random right-hand sides; the method is the "direct eigenvalue
decomposition" of Halko, Martinsson and Tropp, their Algorithm 5.3, on a
range basis from their randomized range finder).

Both block products K Omega and K Q run through a bbFMM plan (one launch
sequence for all l columns).  The dense steps are small: Q is the
orthonormal factor of Y = K Omega by CholeskyQR2 (the Gram matrices Q^T Q
and the products Q R^-1 on the GPU with the library's FP64-accumulating
kernels, bbfmm_dense_atb / bbfmm_dense_ab; the l x l Cholesky factors and
their inverses on the host in FP64), B = Q^T (K Q) is formed on the GPU the
same way, and B's eigendecomposition (l x l) is done on the host in FP64.
The random matrix Omega is an input, so a caller (or a test) can repeat the
algorithm with exact products on the same Omega.
"""
from typing import Optional

import numpy as np

from . import bbfmm


def _to_host(C, stream):
    """Host copy of a result written on `stream` (torch copies on its
    current stream)."""
    import torch
    if stream is not None:
        torch.cuda.synchronize()
    return C.cpu().numpy()


def _to_device(a, device, stream):
    """Device copy of a host array, complete before work on `stream` uses it."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).to(device)
    if stream is not None:
        torch.cuda.synchronize()
    return t


def _orthonormalize(Y, stream=None):
    """CholeskyQR2: Q = Y R^-1 with R from the Cholesky factor of Y^T Y
    (accumulated in FP64), applied twice (the second pass restores
    orthogonality to the round-off of the FP32 basis the next block product
    uses)."""
    Q = Y
    for _ in range(2):
        G = _to_host(bbfmm.dense_atb(Q, Q, stream=stream), stream)
        R = np.linalg.cholesky(0.5 * (G + G.T)).T          # G = R^T R, R upper triangular
        Rinv = np.linalg.solve(R, np.eye(R.shape[0]))
        Q = bbfmm.dense_ab(Q, _to_device(Rinv, Q.device, stream), stream=stream)
    return Q


def randomized_eigh(tree: "bbfmm.Tree", ops: "bbfmm.Ops", omega, k: int,
                    plan: Optional["bbfmm.Plan"] = None, stream=None):
    """Top-k eigenpairs of the kernel matrix K of `tree` (symmetric kernel).

    omega: (N, l) float32 CUDA tensor of independent N(0, 1) entries, l >= k
           (in the points' original order, like sigma).
    Returns (eigenvalues (k,) float64 numpy, descending; eigenvectors (N, k)
    float32 CUDA tensor, orthonormal columns, original point order).
    """
    import torch
    n, l = omega.shape
    if not 1 <= k <= l:
        raise ValueError("need 1 <= k <= number of columns of omega")
    if plan is None:
        plan = bbfmm.Plan(tree, ops, l)
    Y = torch.empty_like(omega)
    plan.execute(omega, Y, stream)                    # first block product
    Q = _orthonormalize(Y, stream)
    Z = torch.empty_like(Q)
    plan.execute(Q, Z, stream)                        # second block product
    B = _to_host(bbfmm.dense_atb(Q, Z, stream=stream), stream)
    B = 0.5 * (B + B.T)
    lam, V = np.linalg.eigh(B)
    order = np.argsort(lam)[::-1][:k]
    lam, V = lam[order], V[:, order]
    U = bbfmm.dense_ab(Q, _to_device(V, Q.device, stream), stream=stream)
    return lam, U
