"""Pins for oracle.assemble: textbook stencils and Kronecker closed forms."""
import numpy as np
import pytest

import synth
from oracle.gll import gll_nodes_weights, deriv_matrix
from oracle.mesh import global_ids, n_unique
from oracle.geometry import box_geometry
from oracle.assemble import (assembled_matrix, element_diagonal,
                             element_diagonal_dense)
from oracle.solve import BoxProblem


def _dense_AG(n, lx, a=0.0, h1=None):
    G, _, _ = box_geometry(n, lx, a)
    Dh = deriv_matrix(gll_nodes_weights(lx - 1)[0])
    return assembled_matrix(Dh, h1, G, global_ids(n, lx), n_unique(n, lx)).toarray()


@pytest.mark.parametrize("n", [3, 4])
def test_lx2_is_seven_point_laplacian(n):
    """Trilinear elements with trapezoidal (lx = 2 GLL) quadrature on a uniform
    periodic grid give h times the 7-point graph Laplacian."""
    A = _dense_AG(n, 2)
    h = 1.0 / n
    L = np.zeros((n ** 3, n ** 3))
    for kk in range(n):
        for jj in range(n):
            for ii in range(n):
                g = (kk * n + jj) * n + ii
                L[g, g] = 6
                for d in (-1, 1):
                    L[g, (kk * n + jj) * n + (ii + d) % n] -= 1
                    L[g, (kk * n + (jj + d) % n) * n + ii] -= 1
                    L[g, (((kk + d) % n) * n + jj) * n + ii] -= 1
    np.testing.assert_allclose(A, h * L, atol=1e-15)
    ev = np.sort(np.linalg.eigvalsh(A))
    m = np.arange(n)
    lam1 = 2 - 2 * np.cos(2 * np.pi * m / n)
    ref = np.sort((lam1[:, None, None] + lam1[None, :, None] + lam1[None, None, :]).ravel()) * h
    np.testing.assert_allclose(ev, ref, atol=1e-13)


def test_kronecker_form_uniform_box():
    n, lx = 3, 4
    A = _dense_AG(n, lx)
    xi, w = gll_nodes_weights(lx - 1)
    Dh = deriv_matrix(xi)
    N, M = lx - 1, n * (lx - 1)
    K1 = np.zeros((M, M)); M1 = np.zeros((M, M))
    Kh = Dh.T @ np.diag(w) @ Dh
    for e in range(n):
        q = (e * N + np.arange(lx)) % M
        K1[np.ix_(q, q)] += Kh
        M1[np.ix_(q, q)] += np.diag(w)
    h = 1.0 / n
    ref = 0.5 * h * (np.kron(M1, np.kron(M1, K1)) + np.kron(M1, np.kron(K1, M1))
                     + np.kron(K1, np.kron(M1, M1)))
    np.testing.assert_allclose(A, ref, atol=1e-14 * np.abs(ref).max())


def test_assembled_periodic_properties():
    n, lx = 2, 4
    nu = n_unique(n, lx)
    ids = global_ids(n, lx)
    h1 = synth.unique_uniform(nu, 0.5, 2.0, 1)[ids]
    A = _dense_AG(n, lx, 0.1, h1)
    np.testing.assert_allclose(A, A.T, atol=1e-14 * np.abs(A).max())
    assert np.max(np.abs(A @ np.ones(nu))) < 1e-13 * np.abs(A).max()
    ev = np.linalg.eigvalsh(A)
    assert abs(ev[0]) < 1e-12 * ev[-1]
    assert ev[1] > 1e-6 * ev[-1]                    # exactly one zero eigenvalue


@pytest.mark.parametrize("lx", [2, 3, 5, 8])
def test_diagonal_formula(lx):
    G, h1 = synth.random_spd_factors(2, lx, 4)
    Dh = deriv_matrix(gll_nodes_weights(lx - 1)[0])
    d1 = element_diagonal(Dh, h1, G)
    d2 = element_diagonal_dense(Dh, h1, G)
    assert np.max(np.abs(d1 - d2)) < 1e-13 * np.max(np.abs(d2))


def test_matrix_free_equals_assembled():
    n, lx = 2, 5
    nu = n_unique(n, lx)
    P = BoxProblem(n, lx, 0.1, synth.unique_uniform(nu, 0.5, 2.0, 1))
    A = assembled_matrix(P.Dh, P.h1, P.G, P.ids, nu)
    x = synth.unique_normal(nu, 0)
    np.testing.assert_allclose(P.apply(x), A @ x, atol=1e-13 * np.abs(A @ x).max())
    np.testing.assert_allclose(P.diagonal(), A.diagonal(), rtol=1e-13)
