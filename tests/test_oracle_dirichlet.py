"""Pins for the oracle's Dirichlet box (homogeneous Dirichlet conditions on the
whole boundary of a non-periodic box): the masked numbering against node
coordinates, masked assembly against deleting rows and columns of the
unmasked (Neumann) matrix, the lowest eigenvalue of the unit cube, and the
spectral convergence of a manufactured solution."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle.assemble import assembled_matrix
from oracle.gs import gather, scatter, gs, multiplicity
from oracle.mesh import (global_ids_dirichlet, n_unique_dirichlet, reference_coords)
from oracle.solve import BoxProblem, pcg, fcg1, iterative_refinement


def _points(n, lx):
    """From the undeformed coordinates alone (independent of the id formulas):
    a mask of the nodes on the cube's boundary, and a numbering of the
    distinct points (two local nodes share a number exactly when they sit at
    the same point), with the number of points."""
    X, Y, Z = reference_coords(n, lx)
    on = lambda c: np.isclose(c, 0.0, atol=1e-12) | np.isclose(c, 1.0, atol=1e-12)  # noqa: E731
    boundary = on(X) | on(Y) | on(Z)
    pts = np.round(np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1), 12)
    _, point = np.unique(pts, axis=0, return_inverse=True)
    point = point.reshape(X.shape)
    return boundary, point, int(point.max()) + 1


@pytest.mark.parametrize("n,lx", [(1, 2), (1, 3), (2, 2), (2, 3), (3, 4), (2, 8)])
def test_dirichlet_ids_follow_coordinates(n, lx):
    ids = global_ids_dirichlet(n, lx)
    nu = n_unique_dirichlet(n, lx)
    boundary, point, npts = _points(n, lx)
    M = n * (lx - 1)
    assert npts == (M + 1) ** 3
    np.testing.assert_array_equal(ids < 0, boundary)
    assert nu == max(M - 1, 0) ** 3
    free = ~boundary
    # every interior point gets one id, and two local nodes share an id
    # exactly when they sit at the same point
    assert len(np.unique(ids[free])) == nu
    if nu:
        assert ids[free].min() == 0 and ids[free].max() == nu - 1
    pairs = np.unique(np.stack([point[free], ids[free]], 1), axis=0)
    assert len(pairs) == nu


def test_masked_gs_and_multiplicity():
    n, lx = 3, 4
    ids = global_ids_dirichlet(n, lx)
    nu = n_unique_dirichlet(n, lx)
    m = multiplicity(ids, nu)
    g1 = gs(np.ones(ids.shape), ids, nu)
    np.testing.assert_array_equal(g1[ids >= 0], m[ids >= 0])
    np.testing.assert_array_equal(g1[ids < 0], 0.0)
    np.testing.assert_array_equal(m[ids < 0], 1.0)
    assert np.sum(1.0 / m[ids >= 0]) == pytest.approx(nu, rel=1e-13)
    uG = synth.unique_normal(nu, 0)
    uL = scatter(uG, ids)
    assert np.all(uL[ids < 0] == 0.0)
    np.testing.assert_allclose(gather(uL / m, ids, nu), uG, rtol=1e-14)


@pytest.mark.parametrize("n,lx,a", [(2, 3, 0.1), (2, 4, 0.05)])
def test_masked_assembly_is_principal_submatrix(n, lx, a):
    """Masking the boundary equals deleting its rows and columns from the
    assembled matrix of the unmasked (natural boundary) box."""
    P = BoxProblem(n, lx, a, dirichlet=True)
    _, full, npts = _points(n, lx)                    # non-periodic point ids
    A_full = assembled_matrix(P.Dh, None, P.G, full, npts).toarray()
    A = assembled_matrix(P.Dh, None, P.G, P.ids, P.nu).toarray()
    free = P.ids >= 0
    order = np.zeros(P.nu, dtype=np.int64)
    order[P.ids[free]] = full[free]                   # interior id -> lattice id
    np.testing.assert_allclose(A, A_full[np.ix_(order, order)], rtol=1e-13, atol=1e-13 * np.abs(A).max())
    # the natural-boundary matrix is singular (constants); the masked one is
    # symmetric positive definite
    assert np.abs(A_full @ np.ones(npts)).max() < 1e-12 * np.abs(A_full).max()
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev[0] > 1e-6 * ev[-1]
    # the matrix-free apply is the same operator
    x = synth.unique_normal(P.nu, 3)
    np.testing.assert_allclose(P.apply(x), A @ x, rtol=1e-12, atol=1e-12 * np.abs(A @ x).max())


def test_lowest_eigenvalue_of_the_unit_cube():
    """-lap v = lambda v on the unit cube with v = 0 on the boundary has lowest
    eigenvalue 3 pi^2 (v = sin(pi x) sin(pi y) sin(pi z)); the discrete pencil
    (A, B) with the diagonal GLL mass B reaches it to spectral accuracy."""
    lam = []
    for lx in (4, 8):
        P = BoxProblem(2, lx, 0.0, dirichlet=True)
        A = assembled_matrix(P.Dh, None, P.G, P.ids, P.nu).toarray()
        Bd = gather(P.B, P.ids, P.nu)
        lam.append(sla.eigh(0.5 * (A + A.T), np.diag(Bd), eigvals_only=True, subset_by_index=[0, 0])[0])
    ref = 3 * np.pi ** 2
    assert abs(lam[1] - ref) < 1e-7 * ref
    assert abs(lam[1] - ref) < 1e-3 * abs(lam[0] - ref)


def test_manufactured_solution_spectral_convergence():
    """u = sin(pi x) sin(pi y) sin(pi z) solves -lap u = 3 pi^2 u with u = 0 on
    the unit cube's boundary; no projection: the Dirichlet operator is
    non-singular.  The discrete error falls spectrally in lx."""
    errs = []
    for lx in (4, 6, 8):
        P = BoxProblem(2, lx, 0.0, dirichlet=True)
        x, y, z = P.coords
        u = np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)
        b = gather(P.B * 3 * np.pi ** 2 * u, P.ids, P.nu)
        sol, it, hist = pcg(P.apply, b, 1.0 / P.diagonal(), tol=1e-13, project=False)
        ex = np.zeros(P.nu)
        ex[P.ids[P.ids >= 0]] = u[P.ids >= 0]
        errs.append(np.max(np.abs(sol - ex)))
    assert errs[0] > 30 * errs[1] and errs[1] > 30 * errs[2]
    assert errs[2] < 1e-6


def test_dirichlet_solvers_agree_with_dense_solve():
    n, lx = 2, 4
    P = BoxProblem(n, lx, 0.1, synth.unique_uniform((n * (lx - 1) - 1) ** 3, 0.5, 2.0, 1), dirichlet=True)
    k, amp, ph = synth.fourier_modes(2, count=8, kmax=2)
    b = P.fourier_rhs(k, amp, ph)
    assert abs(b.sum()) > 1e-6 * np.abs(b).sum()      # no projection on this machine
    A = assembled_matrix(P.Dh, P.h1, P.G, P.ids, P.nu).toarray()
    xref = np.linalg.solve(A, b)
    Minv = 1.0 / P.diagonal()
    x, it, hist = pcg(P.apply, b, Minv, tol=1e-12, project=False)
    assert np.max(np.abs(x - xref)) < 1e-9 * np.max(np.abs(xref))
    x2, _, _ = fcg1(P.apply, b, lambda r: Minv * r, tol=1e-12, project=False)
    assert np.max(np.abs(x2 - xref)) < 1e-9 * np.max(np.abs(xref))

    def inner(rhat):
        d, _, _ = pcg(lambda v: P.apply(v.astype(np.float32).astype(np.float64)), rhat, Minv,
                      tol=1e-5, maxit=500, project=False)
        return d
    x3, outer, relres = iterative_refinement(P.apply, b, inner, tol=1e-10, project=False)
    assert relres[-1] <= 1e-10
    assert np.max(np.abs(x3 - xref)) < 1e-8 * np.max(np.abs(xref))
