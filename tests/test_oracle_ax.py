"""Pins for oracle.ax: three independent forms, invariants, exact energies."""
import itertools

import numpy as np
import pytest

import synth
from oracle.gll import gll_nodes_weights, deriv_matrix, listing_matrices
from oracle.ax import ax_quadrature, ax_einsum, ax_dense, element_matrix
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
    w1 = ax_quadrature(u, Dh, h1, *G)
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


def _affine_elements(lx, r):
    xi, _ = gll_nodes_weights(lx - 1)
    R = np.stack(np.meshgrid(xi, xi, xi, indexing="ij")[::-1], -1)
    for _ in range(3):
        A = 0.4 * (np.eye(3) + 0.25 * r.standard_normal((3, 3)))
        c = 0.3 * r.standard_normal(3)
        yield A, c, R @ A.T + c


@pytest.mark.parametrize("lx", [3, 5, 8])
def test_helmholtz_exact_on_affine_elements(lx):
    """u^T (A + h2 B) u = int |grad u|^2 + h2 int u^2 for u of total degree
    <= N - 1 on sheared affine elements (the GLL rule integrates u^2 exactly up
    to degree 2N - 1 per coordinate), by an independent Gauss-Legendre rule."""
    from oracle.ax import ax_helmholtz
    N, h2 = lx - 1, 0.7
    f, grad = _poly(N - 1, 10 + lx)
    r = np.random.default_rng(6)
    gq, gw = np.polynomial.legendre.leggauss(N + 2)
    Rq = np.stack(np.meshgrid(gq, gq, gq, indexing="ij")[::-1], -1)
    Wq = gw[:, None, None] * gw[None, :, None] * gw[None, None, :]
    got, exact = 0.0, 0.0
    for A, c, X in _affine_elements(lx, r):
        x, y, z = (X[None, ..., d] for d in range(3))
        G, Bm, _ = geometric_factors(x, y, z, lx)
        u = f(x, y, z)
        got += np.sum(u * ax_helmholtz(u, *listing_matrices(lx), None, *G, h2 * Bm))
        Xq = Rq @ A.T + c
        gx, gy, gz = grad(Xq[..., 0], Xq[..., 1], Xq[..., 2])
        uq = f(Xq[..., 0], Xq[..., 1], Xq[..., 2])
        exact += abs(np.linalg.det(A)) * np.sum(Wq * (gx ** 2 + gy ** 2 + gz ** 2 + h2 * uq ** 2))
    assert abs(got - exact) <= 1e-12 * abs(exact)


def test_helmholtz_mass_not_exact_beyond_degree():
    """With the stiffness switched off (G = 0), u = x^N makes u^2 of degree 2N,
    past the GLL rule: the mass identity must fail, so the test above has teeth."""
    from oracle.ax import ax_helmholtz
    lx = 5
    N = lx - 1
    xi, _ = gll_nodes_weights(N)
    R = np.stack(np.meshgrid(xi, xi, xi, indexing="ij")[::-1], -1)
    x, y, z = (R[None, ..., d] for d in range(3))
    G, Bm, _ = geometric_factors(x, y, z, lx)
    u = x ** N
    w = ax_helmholtz(u, *listing_matrices(lx), None, *[0 * g for g in G], Bm)
    exact = 8.0 / (2 * N + 1)          # int over [-1, 1]^3 of x^(2N)
    assert abs(np.sum(u * w) - exact) > 1e-3 * exact


def test_helmholtz_assembled_is_positive_definite():
    """A alone is singular on the periodic box (constants); A + h2 B is not."""
    from oracle.ax import ax_helmholtz
    from oracle.solve import BoxProblem
    from oracle.gs import gather, scatter
    P = BoxProblem(2, 3, 0.1)
    cols = []
    for j in range(P.nu):
        e = np.zeros(P.nu)
        e[j] = 1.0
        w = ax_helmholtz(scatter(e, P.ids), P.dx, P.dx, P.dx, P.dxt, P.dxt, P.dxt, None, *P.G, 0.5 * P.B)
        cols.append(gather(w, P.ids, P.nu))
    M = np.array(cols).T
    assert np.linalg.norm(M - M.T) <= 1e-13 * np.linalg.norm(M)
    ev = np.linalg.eigvalsh(0.5 * (M + M.T))
    assert ev[0] > 1e-6 * ev[-1]
    A = np.array([gather(ax_helmholtz(scatter(np.eye(P.nu)[j], P.ids), P.dx, P.dx, P.dx, P.dxt, P.dxt,
                                      P.dxt, None, *P.G, 0 * P.B), P.ids, P.nu) for j in range(P.nu)]).T
    assert abs(np.linalg.eigvalsh(0.5 * (A + A.T))[0]) < 1e-10 * ev[-1]
