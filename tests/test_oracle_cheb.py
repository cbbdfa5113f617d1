"""Pins of the oracle's interpolation layer (Section 2.2, Definition 2.2).

Each check compares against something other than the oracle's own formula:
roots of T_n from numpy's Chebyshev module, monomials evaluated by numpy's
polynomial module, and the discrete-orthogonality form of the Chebyshev
Lagrange basis.
"""
import numpy as np
import numpy.polynomial.chebyshev as npcheb
import numpy.polynomial.polynomial as nppoly
import pytest

from oracle import cheb


@pytest.mark.parametrize("n", range(2, 9))
def test_nodes_are_roots_of_Tn(n):
    s = cheb.nodes(n)
    coef = np.zeros(n + 1)
    coef[n] = 1.0
    assert np.allclose(npcheb.chebval(s, coef), 0.0, atol=1e-13)
    assert len(np.unique(np.round(s, 12))) == n
    assert np.all(np.abs(s) < 1.0)
    # descending order for the 0-based index m: cos((2m+1) pi / 2n)
    assert np.all(np.diff(s) < 0)


@pytest.mark.parametrize("n", range(2, 9))
def test_lagrange_kronecker_delta_and_partition_of_unity(n):
    s = cheb.nodes(n)
    assert np.allclose(cheb.lagrange_1d(n, s), np.eye(n), atol=1e-13)
    x = np.random.default_rng(n).uniform(-1, 1, 200)
    assert np.allclose(cheb.lagrange_1d(n, x).sum(axis=1), 1.0, atol=1e-12)


@pytest.mark.parametrize("n", range(2, 9))
def test_lagrange_equals_chebyshev_sum_form(n):
    # l_i(x) = 1/n + (2/n) sum_{k=1}^{n-1} T_k(s_i) T_k(x)  (discrete orthogonality)
    s = cheb.nodes(n)
    x = np.random.default_rng(10 + n).uniform(-1.2, 1.2, 50)
    ref = np.full((50, n), 1.0 / n)
    for k in range(1, n):
        e = np.zeros(k + 1)
        e[k] = 1.0
        ref += (2.0 / n) * np.outer(npcheb.chebval(x, e), npcheb.chebval(s, e))
    assert np.allclose(cheb.lagrange_1d(n, x), ref, atol=1e-12)


@pytest.mark.parametrize("n", range(2, 9))
def test_exact_for_polynomials_below_degree_n(n):
    rng = np.random.default_rng(20 + n)
    c = rng.standard_normal(n)              # degree n-1
    s = cheb.nodes(n)
    x = rng.uniform(-1, 1, 100)
    interp = cheb.lagrange_1d(n, x) @ nppoly.polyval(s, c)
    assert np.allclose(interp, nppoly.polyval(x, c), atol=1e-11)


def test_degree_n_is_not_reproduced():
    # a degree-n monomial is not in the span: the interpolant must differ
    n = 4
    s = cheb.nodes(n)
    x = np.linspace(-1, 1, 11)
    interp = cheb.lagrange_1d(n, x) @ s ** n
    assert np.max(np.abs(interp - x ** n)) > 1e-3


@pytest.mark.parametrize("n", [2, 3, 4, 5, 7])
def test_3d_basis_delta_and_exactness(n):
    g = cheb.grid_nodes(n)
    assert g.shape == (n ** 3, 3)
    # node i = i1 + n i2 + n^2 i3 with x fastest
    s = cheb.nodes(n)
    assert np.allclose(g[1, 0], s[1]) and np.allclose(g[n, 1], s[1])
    assert np.allclose(cheb.lagrange_3d(n, g), np.eye(n ** 3), atol=1e-12)
    rng = np.random.default_rng(30 + n)
    c = rng.standard_normal((n, n, n))        # degree < n in every coordinate
    f = lambda p: nppoly.polyval3d(p[:, 0], p[:, 1], p[:, 2], c)
    x = rng.uniform(-1, 1, (64, 3))
    assert np.allclose(cheb.lagrange_3d(n, x) @ f(g), f(x), atol=1e-10)


@pytest.mark.parametrize("n", [3, 4, 6])
@pytest.mark.parametrize("octant", range(8))
def test_m2m_translation_consistency(n, octant):
    """P2M at the parent equals M2M applied to P2M at the child, exactly: the
    parent basis restricted to the child is a polynomial of degree < n."""
    rng = np.random.default_rng(octant + 40 * n)
    # child cell in parent frame: centre (2 bit - 1)/2, half-width 1/2
    shift = np.array([(octant >> d) & 1 for d in range(3)]) - 0.5
    pts = shift + rng.uniform(-0.5, 0.5, (25, 3))
    sig = rng.standard_normal(25)
    m_parent = cheb.lagrange_3d(n, pts).T @ sig
    m_child = cheb.lagrange_3d(n, (pts - shift) / 0.5).T @ sig
    assert np.allclose(cheb.m2m_matrix(n, octant) @ m_child, m_parent, atol=1e-11)
    # L2L is the transpose: L2P in the child of L2L(F) = L2P in the parent of F
    F = rng.standard_normal(n ** 3)
    l2p_parent = cheb.lagrange_3d(n, pts) @ F
    l2p_child = cheb.lagrange_3d(n, (pts - shift) / 0.5) @ (cheb.m2m_matrix(n, octant).T @ F)
    assert np.allclose(l2p_child, l2p_parent, atol=1e-11)


# Equally spaced nodes (Section 2.2: (k-1)/(p-1), k = 1..p, on the cell's
# [-1, 1] frame): the same Lagrange construction on another node set.
@pytest.mark.parametrize("n", range(2, 9))
def test_uniform_nodes_delta_unity_and_exactness(n):
    s = cheb.nodes(n, "uniform")
    assert np.allclose(s, np.linspace(-1.0, 1.0, n), atol=1e-15)
    assert np.allclose(cheb.lagrange_1d(n, s, "uniform"), np.eye(n), atol=1e-12)
    rng = np.random.default_rng(60 + n)
    x = rng.uniform(-1, 1, 200)
    assert np.allclose(cheb.lagrange_1d(n, x, "uniform").sum(axis=1), 1.0, atol=1e-11)
    c = rng.standard_normal(n)              # degree n-1 is reproduced exactly
    interp = cheb.lagrange_1d(n, x, "uniform") @ nppoly.polyval(s, c)
    assert np.allclose(interp, nppoly.polyval(x, c), atol=1e-10)
    # and degree n is not
    assert np.max(np.abs(cheb.lagrange_1d(n, x, "uniform") @ s ** n - x ** n)) > 1e-4


@pytest.mark.parametrize("n", [3, 4, 6])
@pytest.mark.parametrize("octant", [0, 5, 7])
def test_uniform_nodes_translation_consistency(n, octant):
    """M2M / L2L identities hold for the uniform basis too (exactness below
    degree n does not depend on the nodes)."""
    rng = np.random.default_rng(octant + 70 * n)
    shift = np.array([(octant >> d) & 1 for d in range(3)]) - 0.5
    pts = shift + rng.uniform(-0.5, 0.5, (25, 3))
    sig = rng.standard_normal(25)
    m_parent = cheb.lagrange_3d(n, pts, "uniform").T @ sig
    m_child = cheb.lagrange_3d(n, (pts - shift) / 0.5, "uniform").T @ sig
    T = cheb.m2m_matrix(n, octant, "uniform")
    assert np.allclose(T @ m_child, m_parent, atol=1e-10)
    F = rng.standard_normal(n ** 3)
    l2p_parent = cheb.lagrange_3d(n, pts, "uniform") @ F
    l2p_child = cheb.lagrange_3d(n, (pts - shift) / 0.5, "uniform") @ (T.T @ F)
    assert np.allclose(l2p_child, l2p_parent, atol=1e-10)
