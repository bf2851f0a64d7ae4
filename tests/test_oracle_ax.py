"""Pins for oracle.ax: three independent forms, invariants, exact energies."""
import itertools

import numpy as np
import pytest

import synth
from oracle.gll import gll_nodes_weights, deriv_matrix, listing_matrices
from oracle.ax import ax_loops, ax_einsum, ax_dense, element_matrix
from oracle.geometry import geometric_factors


def _inputs(nel, lx, seed):
    G, h1 = synth.random_spd_factors(nel, lx, seed)
    u = synth.local_normal(nel, lx, seed + 100)
    return u, G, h1


@pytest.mark.parametrize("lx", [2, 3, 4, 6])
def test_three_forms_agree(lx):
    u, G, h1 = _inputs(3, lx, 7)
    M = listing_matrices(lx)
    xi, _ = gll_nodes_weights(lx - 1)
    Dh = deriv_matrix(xi)
    w1 = ax_loops(u, *M, h1, *G)
    w2 = ax_einsum(u, *M, h1, *G)
    w3 = ax_dense(u, Dh, h1, G)
    s = np.max(np.abs(w3))
    assert np.max(np.abs(w1 - w3)) / s < 1e-14
    assert np.max(np.abs(w2 - w3)) / s < 1e-14


def test_swapped_matrices_detected():
    """Dhat is not symmetric, so exchanging dx and dxt changes the result."""
    lx = 5
    u, G, h1 = _inputs(2, lx, 3)
    dx, dy, dz, dxt, dyt, dzt = listing_matrices(lx)
    good = ax_einsum(u, dx, dy, dz, dxt, dyt, dzt, h1, *G)
    bad = ax_einsum(u, dxt, dyt, dzt, dx, dy, dz, h1, *G)
    assert np.max(np.abs(good - bad)) / np.max(np.abs(good)) > 1e-2


@pytest.mark.parametrize("lx", [3, 5, 8])
def test_symmetry_nullspace_positivity(lx):
    u, G, h1 = _inputs(4, lx, 11)
    v = synth.local_normal(4, lx, 12)
    M = listing_matrices(lx)
    Au = ax_einsum(u, *M, h1, *G)
    Av = ax_einsum(v, *M, h1, *G)
    for e in range(4):
        a, b = np.sum(v[e] * Au[e]), np.sum(u[e] * Av[e])
        assert abs(a - b) <= 1e-12 * (abs(a) + 1)
        assert np.sum(u[e] * Au[e]) >= 0
    A1 = ax_einsum(np.ones_like(u), *M, h1, *G)
    assert np.max(np.abs(A1)) < 1e-12 * np.max(np.abs(Au))
    Dh = deriv_matrix(gll_nodes_weights(lx - 1)[0])
    Ae = element_matrix(Dh, h1[0], tuple(g[0] for g in G))
    ev = np.linalg.eigvalsh(0.5 * (Ae + Ae.T))
    assert abs(ev[0]) < 1e-12 * ev[-1] and ev[1] > 1e-8 * ev[-1]   # one-dimensional kernel


def _poly(N, seed):
    """Random polynomial of total degree <= N in (x, y, z), with its gradient."""
    r = np.random.default_rng(seed)
    terms = [(a, b, c) for a, b, c in itertools.product(range(N + 1), repeat=3) if a + b + c <= N]
    coef = r.standard_normal(len(terms))

    def f(x, y, z):
        return sum(cf * x ** a * y ** b * z ** c for cf, (a, b, c) in zip(coef, terms))

    def grad(x, y, z):
        gx = sum(cf * a * x ** max(a - 1, 0) * y ** b * z ** c for cf, (a, b, c) in zip(coef, terms))
        gy = sum(cf * b * x ** a * y ** max(b - 1, 0) * z ** c for cf, (a, b, c) in zip(coef, terms))
        gz = sum(cf * c * x ** a * y ** b * z ** max(c - 1, 0) for cf, (a, b, c) in zip(coef, terms))
        return gx, gy, gz
    return f, grad


@pytest.mark.parametrize("lx", [3, 5, 8])
def test_energy_exact_on_affine_elements(lx):
    """sum_e u_e^T A_e u_e = int |grad u|^2 for u of total degree <= N on
    sheared affine elements (Eq. 1 with v = u), the integral taken by an
    independent Gauss-Legendre rule in reference coordinates."""
    N = lx - 1
    f, grad = _poly(N, lx)
    r = np.random.default_rng(5)
    xi, _ = gll_nodes_weights(N)
    R = np.stack(np.meshgrid(xi, xi, xi, indexing="ij")[::-1], -1)
    gq, gw = np.polynomial.legendre.leggauss(N + 2)
    Rq = np.stack(np.meshgrid(gq, gq, gq, indexing="ij")[::-1], -1)
    Wq = gw[:, None, None] * gw[None, :, None] * gw[None, None, :]
    energy_ax, energy_exact = 0.0, 0.0
    M = listing_matrices(lx)
    for _ in range(3):
        A = 0.4 * (np.eye(3) + 0.25 * r.standard_normal((3, 3)))
        c = 0.3 * r.standard_normal(3)
        X = R @ A.T + c
        x, y, z = (X[None, ..., d] for d in range(3))
        G, _, _ = geometric_factors(x, y, z, lx)
        u = f(x, y, z)
        w = ax_einsum(u, *M, None, *G)
        energy_ax += np.sum(u * w)
        Xq = Rq @ A.T + c
        gx, gy, gz = grad(Xq[..., 0], Xq[..., 1], Xq[..., 2])
        energy_exact += abs(np.linalg.det(A)) * np.sum(Wq * (gx ** 2 + gy ** 2 + gz ** 2))
    assert abs(energy_ax - energy_exact) <= 1e-12 * abs(energy_exact)


def test_energy_not_exact_beyond_total_degree():
    """Tensor degree N (total degree 3N) exceeds the GLL rule's exactness: the
    identity must fail, showing the previous test has teeth."""
    lx = 5
    xi, _ = gll_nodes_weights(lx - 1)
    R = np.stack(np.meshgrid(xi, xi, xi, indexing="ij")[::-1], -1)
    x, y, z = (R[None, ..., d] for d in range(3))
    G, _, _ = geometric_factors(x, y, z, lx)
    u = (x ** 4) * (y ** 4) * (z ** 4)
    w = ax_einsum(u, *listing_matrices(lx), None, *G)
    gq, gw = np.polynomial.legendre.leggauss(8)
    Wq = gw[:, None, None] * gw[None, :, None] * gw[None, None, :]
    Q = np.stack(np.meshgrid(gq, gq, gq, indexing="ij")[::-1], -1)
    X, Y, Z = Q[..., 0], Q[..., 1], Q[..., 2]
    exact = np.sum(Wq * 16 * ((X ** 3 * Y ** 4 * Z ** 4) ** 2 + (X ** 4 * Y ** 3 * Z ** 4) ** 2
                              + (X ** 4 * Y ** 4 * Z ** 3) ** 2))
    assert abs(np.sum(u * w) - exact) > 1e-3 * exact
