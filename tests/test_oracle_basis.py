"""Pins of the oracle's reference elements and quadrature rules against closed forms."""
import math

import numpy as np
import pytest

from oracle.basis import (gauss_legendre, gauss_lobatto, stroud_triangle, Lagrange1D,
                          RefQuad, RefTri, RefSeg, multi_indices)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_gauss_legendre_exact(n):
    x, w = gauss_legendre(n)
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs((w * x ** k).sum() - exact) < 1e-14


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_gauss_lobatto_exact_and_endpoints(n):
    x, w = gauss_lobatto(n)
    assert x[0] == -1.0 and x[-1] == 1.0
    for k in range(2 * n - 2):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs((w * x ** k).sum() - exact) < 1e-14
    # degree 2n-2 is NOT integrated exactly (guards against a Gauss rule in disguise)
    k = 2 * n - 2
    assert abs((w * x ** k).sum() - 2.0 / (k + 1)) > 1e-6


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_stroud_exact_to_degree_2n_minus_1(n):
    pts, w = stroud_triangle(n)
    for a in range(2 * n):
        for b in range(2 * n - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            got = (w * pts[:, 0] ** a * pts[:, 1] ** b).sum()
            assert abs(got - exact) < 1e-14, (a, b)
    assert len(w) == n * n and (w > 0).all()
    assert (pts[:, 0] >= 0).all() and (pts[:, 1] >= 0).all() and (pts.sum(1) <= 1).all()


def test_lagrange_nodal_and_derivative():
    x, _ = gauss_lobatto(4)
    L = Lagrange1D(x)
    assert np.allclose(L(x), np.eye(4), atol=1e-14)
    # d/dx of the interpolant of x^3 is 3x^2
    t = np.linspace(-1, 1, 7)
    assert np.allclose(L(t, 1) @ x ** 3, 3 * t ** 2, atol=1e-13)
    assert np.allclose(L(t, 2) @ x ** 3, 6 * t, atol=1e-12)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_reference_bases_partition_of_unity(p):
    for ref in (RefQuad(p, "gauss"), RefQuad(p, "lobatto"), RefTri(p), RefSeg(p, "gauss")):
        pts = ref.vol_pts
        phi = ref.deriv(pts, (0,) * ref.dim)
        assert np.allclose(phi.sum(1), 1.0, atol=1e-13)
        assert np.allclose(ref.deriv(ref.nodes, (0,) * ref.dim), np.eye(ref.n_loc), atol=1e-12)
        for m in multi_indices(ref.dim, p):
            assert np.allclose(ref.deriv(pts, m).sum(1), 0.0, atol=1e-11)


def test_multi_index_order():
    assert multi_indices(2, 3) == [(1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (3, 0), (2, 1), (1, 2), (0, 3)]
    assert multi_indices(1, 3) == [(1,), (2,), (3,)]
