"""Pins of the oracle's 1D node sets and Lagrange basis (Sec. 3.1: DGSEM on
Legendre-Gauss or Legendre-Gauss-Lobatto points with nodal Lagrange polynomials)."""
import math

import numpy as np
import pytest

from oracle import oracle as O


@pytest.mark.parametrize("N", range(1, 13))
def test_gauss_against_numpy_and_sum(N):
    x, w = O.nodes(N, O.GAUSS)
    xr, wr = np.polynomial.legendre.leggauss(N + 1)
    assert np.max(np.abs(x - xr)) < 2e-15
    assert np.max(np.abs(w - wr)) < 2e-14
    assert abs(w.sum() - 2.0) < 1e-14
    assert np.all(np.diff(x) > 0)


def test_closed_forms():
    x, w = O.nodes(1, O.GAUSS)
    assert np.allclose(x, [-1 / math.sqrt(3), 1 / math.sqrt(3)], atol=4e-16, rtol=0)
    assert np.allclose(w, [1, 1], atol=1e-15, rtol=0)
    x, w = O.nodes(2, O.GAUSS)
    assert np.allclose(x, [-math.sqrt(0.6), 0, math.sqrt(0.6)], atol=4e-16, rtol=0)
    assert np.allclose(w, [5 / 9, 8 / 9, 5 / 9], atol=1e-15, rtol=0)
    x, w = O.nodes(2, O.LGL)
    assert np.allclose(x, [-1, 0, 1], atol=4e-16, rtol=0)
    assert np.allclose(w, [1 / 3, 4 / 3, 1 / 3], atol=1e-15, rtol=0)
    x, w = O.nodes(3, O.LGL)
    assert np.allclose(x, [-1, -1 / math.sqrt(5), 1 / math.sqrt(5), 1], atol=4e-16, rtol=0)
    assert np.allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], atol=1e-15, rtol=0)


@pytest.mark.parametrize("node_set,exact_deg", [(O.GAUSS, lambda N: 2 * N + 1),
                                                 (O.LGL, lambda N: 2 * N - 1)])
@pytest.mark.parametrize("N", range(1, 12))
def test_monomial_exactness(node_set, exact_deg, N):
    x, w = O.nodes(N, node_set)
    deg = exact_deg(N)
    for d in range(deg + 1):
        exact = 0.0 if d % 2 else 2.0 / (d + 1)
        assert abs(np.sum(w * x ** d) - exact) < 1e-13
    # one degree higher (even) is not integrated exactly: catches an off-by-one node count
    d = deg + 1
    assert abs(np.sum(w * x ** d) - 2.0 / (d + 1)) > 1e-11


def test_lgl_interior_are_roots_of_derivative():
    for N in range(2, 12):
        x, _ = O.nodes(N, O.LGL)
        dP = np.polynomial.legendre.Legendre.basis(N).deriv()
        assert np.max(np.abs(dP(x[1:-1]))) < 1e-11
        assert x[0] == -1.0 and x[-1] == 1.0


@pytest.mark.parametrize("node_set", [O.GAUSS, O.LGL])
def test_lagrange_cardinal_and_partition_of_unity(node_set):
    rng = np.random.default_rng(0)
    for N in (1, 3, 5, 9):
        x, _ = O.nodes(N, node_set)
        for j in range(N + 1):
            for i in range(N + 1):
                assert O.lagrange(N, x, j, x[i]) == (1.0 if i == j else 0.0)
        for xi in rng.uniform(-1.3, 1.3, 5):
            vals = [O.lagrange(N, x, j, xi) for j in range(N + 1)]
            assert abs(sum(vals) - 1.0) < 1e-12
            # reproduces x^N
            assert abs(sum(v * x[j] ** N for j, v in enumerate(vals)) - xi ** N) < 1e-11
