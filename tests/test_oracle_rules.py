"""Pins for the oracle's 1D rules: closed forms and exactness properties."""
import numpy as np
import pytest
from scipy.special import eval_legendre

from oracle import gauss_legendre, gll_nodes, lagrange
from tests.oracle_helpers import lagrange_polys


GOLDEN = {  # closed forms of the GLL nodes on [-1, 1] (textbook Lobatto rules)
    1: [-1.0, 1.0],
    2: [-1.0, 0.0, 1.0],
    3: [-1.0, -1 / np.sqrt(5), 1 / np.sqrt(5), 1.0],
    4: [-1.0, -np.sqrt(3 / 7), 0.0, np.sqrt(3 / 7), 1.0],
}


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_gll_closed_forms(k):
    assert np.allclose(gll_nodes(k), (np.array(GOLDEN[k]) + 1) / 2, atol=1e-15)


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6, 7, 8])
def test_gll_lobatto_exactness(k):
    # Lobatto weights 2/(k(k+1) P_k(x_i)^2) with the true nodes integrate
    # degree <= 2k-1 exactly; any wrong node breaks it.
    x = 2 * gll_nodes(k) - 1
    w = 2.0 / (k * (k + 1) * eval_legendre(k, x) ** 2)
    for m in range(2 * k):
        exact = (1 - (-1) ** (m + 1)) / (m + 1)
        assert abs(np.dot(w, x ** m) - exact) < 1e-13
    assert np.all(np.diff(x) > 0)


@pytest.mark.parametrize("nq", [1, 2, 3, 4, 5, 6, 9])
def test_gauss_exactness(nq):
    x, w = gauss_legendre(nq)
    assert abs(w.sum() - 1) < 1e-15
    for m in range(2 * nq):
        assert abs(np.dot(w, x ** m) - 1 / (m + 1)) < 1e-14
    # and not exact one degree higher (the error is visible above rounding)
    if nq <= 6:
        assert abs(np.dot(w, x ** (2 * nq)) - 1 / (2 * nq + 1)) > 1e-12


def test_gauss_closed_forms():
    x, w = gauss_legendre(3)
    assert np.allclose(x, [(1 - np.sqrt(0.6)) / 2, 0.5, (1 + np.sqrt(0.6)) / 2], atol=1e-15)
    assert np.allclose(w, [5 / 18, 8 / 18, 5 / 18], atol=1e-15)


@pytest.mark.parametrize("k,nq", [(1, 2), (2, 3), (3, 5), (4, 6), (7, 9)])
def test_lagrange_tables(k, nq):
    nodes = gll_nodes(k)
    pts, _ = gauss_legendre(nq)
    L, dL = lagrange(nodes, pts)
    Ln, _ = lagrange(nodes, nodes)
    assert np.allclose(Ln, np.eye(k + 1), atol=1e-13)
    assert np.allclose(L.sum(1), 1, atol=1e-13)
    assert np.allclose(dL.sum(1), 0, atol=1e-11)
    polys = lagrange_polys(nodes)
    for a in range(k + 1):
        assert np.allclose(L[:, a], polys[a](pts), atol=1e-11)
        assert np.allclose(dL[:, a], polys[a].deriv()(pts), atol=1e-9)
