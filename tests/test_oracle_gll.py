"""Pins of the oracle's GLL grid and differentiation matrix (Sec. 2.2)."""
import os

import numpy as np
import pytest

from oracle import gll

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "gll_n11_fig1.txt")


def _golden_nodes():
    vals = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                vals.append(float(line))
    return np.array(vals)


def test_nodes_match_printed_figure():
    # Fig. 1 draws the 11-point GLL grid to two decimals.
    printed = _golden_nodes()
    x = gll.gll_nodes(11)
    assert len(printed) == 11
    assert np.max(np.abs(x - printed)) <= 0.005 + 1e-12


@pytest.mark.parametrize("n", [2, 3, 5, 9, 11, 13, 17, 21])
def test_closed_forms(n):
    x = gll.gll_nodes(n)
    w = gll.gll_weights(x)
    N = n - 1
    assert x[0] == -1.0 and x[-1] == 1.0
    assert np.all(np.diff(x) > 0)
    np.testing.assert_allclose(x, -x[::-1], atol=1e-15)
    np.testing.assert_allclose(w[0], 2.0 / (N * (N + 1)), rtol=1e-14)
    np.testing.assert_allclose(w.sum(), 2.0, rtol=1e-14)
    D = gll.diff_matrix(x)
    if n > 2:
        np.testing.assert_allclose(D[0, 0], -N * (N + 1) / 4.0, rtol=1e-12)
        np.testing.assert_allclose(D[-1, -1], N * (N + 1) / 4.0, rtol=1e-12)
    assert np.max(np.abs(D @ np.ones(n))) < 1e-12 * n * n


@pytest.mark.parametrize("n", [3, 6, 11, 17])
def test_exactness_on_polynomials(n):
    x = gll.gll_nodes(n)
    w = gll.gll_weights(x)
    D = gll.diff_matrix(x)
    scale = np.max(np.abs(D))
    for m in range(n):  # degree <= n - 1 is differentiated exactly
        d = D @ x ** m
        exact = m * x ** (m - 1) if m > 0 else np.zeros(n)
        assert np.max(np.abs(d - exact)) < 1e-13 * scale * max(m, 1)
    for m in range(2 * n - 2):  # GLL quadrature is exact to degree 2n - 3
        exact = 0.0 if m % 2 else 2.0 / (m + 1)
        assert abs(w @ x ** m - exact) < 1e-14 * 10


def test_interior_nodes_are_legendre_derivative_roots():
    # Independent route: numpy's companion-matrix roots of P'_{n-1}.
    from numpy.polynomial import legendre as leg
    for n in (5, 11, 17):
        c = np.zeros(n); c[-1] = 1
        roots = np.sort(np.real(leg.legroots(leg.legder(c))))
        np.testing.assert_allclose(gll.gll_nodes(n)[1:-1], roots, atol=1e-13)


def test_second_derivative_exact():
    n = 9
    x = gll.gll_nodes(n)
    D = gll.diff_matrix(x)
    D2 = D @ D
    for m in range(n):
        exact = m * (m - 1) * x ** (m - 2) if m > 1 else np.zeros(n)
        assert np.max(np.abs(D2 @ x ** m - exact)) < 1e-11
    assert np.max(np.abs(D2 @ np.ones(n))) < 1e-11
