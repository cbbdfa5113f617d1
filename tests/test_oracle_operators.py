"""Pins of the oracle's M2L operators and SVD compression (Sections 2.3, 2.5).

Checks use independent routes: the symmetric eigensolver on Gram matrices
summed operator by operator (not the concatenated matrices the oracle feeds
to the SVD), direct kernel evaluation at the nodes, the homogeneity identity
of Section 2.5, and the symmetry identities that a symmetric kernel implies.
"""
import numpy as np
import pytest

import synth
from oracle import cheb, operators as O, tree as T
from oracle._native import kernel_values


def test_sampled_operator_matches_pointwise_kernel():
    n, h = 3, 0.125
    K = O.sample_m2l(0, 1.0, n, h)
    tv = T.transfer_vectors()
    s = cheb.nodes(n)
    ti = 100
    i, j = 5, 17           # i = i1 + n i2 + n^2 i3
    xi = h * np.array([s[i % n], s[(i // n) % n], s[i // n ** 2]])
    yj = h * (2 * tv[ti] + np.array([s[j % n], s[(j // n) % n], s[j // n ** 2]]))
    assert np.isclose(K[ti, i, j], 1.0 / np.linalg.norm(xi - yj), rtol=1e-14)


def test_kernel_values_closed_forms():
    d = np.array([[3.0, 4.0, 0.0], [0.0, 0.0, 0.0]])
    assert np.allclose(kernel_values(d, 0, 1.0), [0.2, 0.0])
    assert np.allclose(kernel_values(d, 1, 2.0), [np.exp(-2.5), 1.0])
    assert np.allclose(kernel_values(d, 2, 5.0), [np.exp(-1.0), 1.0])
    u = np.array([[0.5, -1.0, 2.0]])
    g = lambda x: 1 + x / 2 - x * x / 3 + x ** 3 / 5
    assert np.allclose(kernel_values(u, 100, 1.0), g(0.5) * g(-1.0) * g(2.0))


@pytest.mark.parametrize("kid,param", [(0, 1.0), (1, 0.1), (2, 0.05)])
def test_symmetric_kernel_operator_identities(kid, param):
    n = 4
    K = O.sample_m2l(kid, param, n, 0.03125)
    tv = T.transfer_vectors()
    neg = {tuple(t): i for i, t in enumerate(tv)}
    for ti, t in enumerate(tv):
        assert np.allclose(K[neg[tuple(-t)]], K[ti].T, rtol=1e-13, atol=0)
    op = O.compress(K, 1e-5)
    # U U^T = V V^T for a symmetric kernel, and C_{-t} = C_t^T
    assert np.allclose(op.U @ op.U.T, op.V @ op.V.T, atol=1e-8)
    R = op.V.T @ op.U          # rotation between the two bases (near orthogonal)
    for ti, t in enumerate(tv[:40]):
        a = R @ op.C[neg[tuple(-t)]] @ R
        assert np.allclose(a, op.C[ti].T, atol=1e-8 * np.abs(op.C).max())


@pytest.mark.parametrize("kid,param,h", [(0, 1.0, 0.25), (1, 0.1, 0.0625), (100, 1.0, 0.5)])
def test_svd_against_gram_eigenvalues_and_truncation(kid, param, h):
    n = 4
    eps = 1e-5
    K = O.sample_m2l(kid, param, n, h)
    op = O.compress(K, eps)
    g_fat = sum(Kt @ Kt.T for Kt in K)
    g_thin = sum(Kt.T @ Kt for Kt in K)
    ev_f = np.sort(np.linalg.eigvalsh(g_fat))[::-1]
    ev_t = np.sort(np.linalg.eigvalsh(g_thin))[::-1]
    assert np.allclose(op.sv_fat ** 2, ev_f, atol=1e-12 * ev_f[0])
    assert np.allclose(op.sv_thin ** 2, ev_t, atol=1e-12 * ev_t[0])
    k_ref = max(np.count_nonzero(ev_f > eps ** 2 * ev_f[0]),
                np.count_nonzero(ev_t > eps ** 2 * ev_t[0]))
    assert op.k == k_ref
    # reconstruction error bounded by the discarded singular values
    tail = np.sqrt(np.sum(op.sv_fat[op.k:] ** 2) + np.sum(op.sv_thin[op.k:] ** 2))
    err = np.sqrt(sum(np.linalg.norm(K[t] - op.U @ op.C[t] @ op.V.T) ** 2 for t in range(316)))
    assert err <= 1.01 * tail + 1e-14 * op.sv_fat[0]
    assert err <= 2 * eps * op.sv_fat[0] * np.sqrt(len(op.sv_fat))
    # U, V orthonormal
    assert np.allclose(op.U.T @ op.U, np.eye(op.k), atol=1e-12)
    assert np.allclose(op.V.T @ op.V, np.eye(op.k), atol=1e-12)


def test_rank_monotone_in_eps_and_eps_zero_is_identity():
    K = O.sample_m2l(1, 0.1, 4, 0.05)
    ks = [O.compress(K, e).k for e in (1e-2, 1e-4, 1e-6, 1e-8)]
    assert ks == sorted(ks) and ks[0] < ks[-1] <= 64
    op0 = O.compress(K, 0.0)
    assert op0.k == 64 and np.array_equal(op0.C, K)
    assert np.array_equal(op0.U, np.eye(64))


def test_homogeneous_scaling_matches_direct_sampling():
    """Section 2.5: K(c x, c y) = c^-1 K(x, y) for 1/r, so the level-l
    operators are the unit ones times h_l^-1."""
    pts, _ = synth.random_cloud(500, 3)
    tree = T.build_tree(pts, fixed_depth=5)
    ops = O.precompute(tree, 0, 1.0, 4, 1e-5)
    for lvl in range(2, 5):
        h = tree.half_width(lvl)
        direct = O.compress(O.sample_m2l(0, 1.0, 4, h), 1e-5)
        op = ops.levels[lvl]
        assert op.k == direct.k
        for ti in (0, 57, 200, 315):
            a = op.U @ op.C[ti] @ op.V.T
            b = direct.U @ direct.C[ti] @ direct.V.T
            assert np.allclose(a, b, rtol=0, atol=1e-9 * np.abs(b).max())


@pytest.mark.parametrize("n", [2, 4, 5])
def test_uniform_node_operator_is_block_toeplitz(n):
    """With equally spaced nodes K_t[i, j] depends only on the per-axis
    index differences i_d - j_d (Section 2.5, fast M2L translation): a
    p^3 x p^3 operator with only (2p - 1)^3 distinct entries."""
    K = O.sample_m2l(1, 0.7, n, 0.3, nodes="uniform")
    idx = np.arange(n ** 3)
    i3 = np.stack([idx % n, (idx // n) % n, idx // (n * n)], axis=1)
    diff = i3[:, None, :] - i3[None, :, :] + (n - 1)           # in [0, 2n-2]
    code = diff[..., 0] + (2 * n - 1) * (diff[..., 1] + (2 * n - 1) * diff[..., 2])
    for t in (0, 150, 315):
        vals = {}
        for c, v in zip(code.ravel(), K[t].ravel()):
            vals.setdefault(int(c), []).append(v)
        assert len(vals) == (2 * n - 1) ** 3
        assert max(np.ptp(v) for v in vals.values()) <= 1e-15 * np.abs(K[t]).max()
    # Chebyshev nodes have no such structure (from n = 3 on; two nodes are
    # symmetric about 0 and so equally spaced)
    if n > 2:
        Kc = O.sample_m2l(1, 0.7, n, 0.3)[150].ravel()
        spread = max(np.ptp(Kc[code.ravel() == c]) for c in np.unique(code))
        assert spread > 1e-6 * np.abs(Kc).max()
