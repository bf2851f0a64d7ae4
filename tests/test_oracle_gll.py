"""Pins for oracle.gll: closed forms, tables and exactness properties."""
import os

import numpy as np
import pytest

from oracle.gll import (gll_nodes_weights, deriv_matrix, lagrange_basis,
                        lagrange_eq2, listing_matrices)

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_closed_forms_small_orders():
    xi, w = gll_nodes_weights(2)
    np.testing.assert_allclose(xi, [-1, 0, 1], atol=1e-15)
    np.testing.assert_allclose(w, [1 / 3, 4 / 3, 1 / 3], rtol=1e-15)
    xi, w = gll_nodes_weights(3)
    s = 1 / np.sqrt(5)
    np.testing.assert_allclose(xi, [-1, -s, s, 1], rtol=1e-15)
    np.testing.assert_allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], rtol=1e-14)
    xi, w = gll_nodes_weights(4)
    s = np.sqrt(3 / 7)
    np.testing.assert_allclose(xi, [-1, -s, 0, s, 1], rtol=1e-15, atol=1e-16)
    np.testing.assert_allclose(w, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], rtol=1e-14)


def test_table_n7():
    tab = np.loadtxt(os.path.join(GOLD, "gll_n7.txt"))
    xi, w = gll_nodes_weights(7)
    np.testing.assert_allclose(xi[4:], tab[::-1, 0], atol=1e-15)
    np.testing.assert_allclose(xi[:4], -tab[:, 0], atol=1e-15)
    np.testing.assert_allclose(w[:4], tab[:, 1], atol=1e-15)


@pytest.mark.parametrize("N", range(1, 14))
def test_quadrature_degree(N):
    xi, w = gll_nodes_weights(N)
    assert abs(w.sum() - 2.0) < 1e-14
    for m in range(0, 2 * N):             # exact up to degree 2N - 1
        exact = 2.0 / (m + 1) if m % 2 == 0 else 0.0
        assert abs(w @ xi ** m - exact) < 1e-13, (N, m)
    m = 2 * N                               # and not beyond
    assert abs(w @ xi ** m - 2.0 / (m + 1)) > 1e-10


@pytest.mark.parametrize("N", range(1, 14))
def test_derivative_matrix(N):
    xi, _ = gll_nodes_weights(N)
    D = deriv_matrix(xi)
    for m in range(0, N + 1):               # exact on degree <= N
        d = D @ xi ** m
        ref = m * xi ** (m - 1) if m > 0 else 0 * xi
        assert np.max(np.abs(d - ref)) < 5e-13 * max(1, N ** 2), (N, m)
    assert abs(D[0, 0] + N * (N + 1) / 4) < 1e-12
    assert abs(D[N, N] - N * (N + 1) / 4) < 1e-12
    assert np.all(np.abs(np.diag(D)[1:N]) < 1e-12)
    # one degree higher is not differentiated exactly (N >= 1)
    m = N + 1
    assert np.max(np.abs(D @ xi ** m - m * xi ** (m - 1))) > 1e-8


@pytest.mark.parametrize("N", [2, 4, 7, 11])
def test_eq2_basis(N):
    xi, _ = gll_nodes_weights(N)
    x = np.linspace(-0.987, 0.993, 37)
    np.testing.assert_allclose(lagrange_eq2(N, xi, x), lagrange_basis(xi, x), atol=1e-12)
    np.testing.assert_allclose(lagrange_basis(xi, xi), np.eye(N + 1), atol=1e-14)
    # D is the derivative of the basis: central difference of l_l at node i
    D = deriv_matrix(xi)
    h = 1e-6
    xin = np.clip(xi, -1 + h, 1 - h)
    fd = (lagrange_basis(xi, xin + h) - lagrange_basis(xi, xin - h)) / (2 * h)
    np.testing.assert_allclose(fd[1:-1], D[1:-1], atol=1e-6 * N ** 2)


def test_listing_layout():
    dx, dy, dz, dxt, dyt, dzt = listing_matrices(6)
    xi, _ = gll_nodes_weights(5)
    D = deriv_matrix(xi)
    u = np.sin(xi)                           # Listing 2: r-derivative at i is sum_l dx[l, i] u_l
    np.testing.assert_allclose(np.einsum("li,l->i", dx, u), D @ u, atol=1e-15)
    np.testing.assert_allclose(dxt, dx.T)
