"""Pins of the plain-C statement (oracle/sem_ref.c) against the numpy oracle,
whose own pins are closed forms, invariants and brute force.  A mistake in
the C statement (a transposed derivative weight, a dropped cross term, a
wrong index in the gather) fails one of these."""
import numpy as np
import pytest

import synth
from oracle import cref
from oracle.gll import gll_nodes_weights, deriv_matrix, listing_matrices
from oracle.ax import ax_einsum
from oracle.assemble import element_diagonal
from oracle.mesh import box_coords
from oracle.geometry import geometric_factors
from oracle.solve import BoxProblem, pcg
from oracle.gs import gather


def _Dh(lx):
    xi, w = gll_nodes_weights(lx - 1)
    return xi, w, deriv_matrix(xi)


@pytest.mark.parametrize("lx", [2, 5, 8, 12])
def test_c_operator_matches_einsum(lx):
    G, h1 = synth.random_spd_factors(5, lx, 21)
    u = synth.local_normal(5, lx, 22)
    M = listing_matrices(lx)
    _, _, Dh = _Dh(lx)
    ref = ax_einsum(u, *M, h1, *G)
    got = cref.ax(u, Dh, h1, G)
    assert np.max(np.abs(got - ref)) < 1e-14 * np.max(np.abs(ref))
    got1 = cref.ax(u, Dh, None, G)
    ref1 = ax_einsum(u, *M, None, *G)
    assert np.max(np.abs(got1 - ref1)) < 1e-14 * np.max(np.abs(ref1))


def test_c_operator_detects_transposed_derivative():
    lx = 5
    G, h1 = synth.random_spd_factors(2, lx, 23)
    u = synth.local_normal(2, lx, 24)
    _, _, Dh = _Dh(lx)
    ref = ax_einsum(u, *listing_matrices(lx), h1, *G)
    bad = cref.ax(u, np.ascontiguousarray(Dh.T), h1, G)
    assert np.max(np.abs(bad - ref)) > 1e-2 * np.max(np.abs(ref))


@pytest.mark.parametrize("lx", [3, 8])
def test_c_diagonal_matches_oracle(lx):
    G, h1 = synth.random_spd_factors(3, lx, 25)
    _, _, Dh = _Dh(lx)
    np.testing.assert_allclose(cref.diag(Dh, h1, G), element_diagonal(Dh, h1, G), rtol=1e-13)


def test_c_coords_and_geometry_match_oracle():
    n, lx, a = 3, 6, 0.12
    xi, w, Dh = _Dh(lx)
    xyz = cref.box_coords(n, lx, a, xi)
    ref = box_coords(n, lx, a)
    for got, want in zip(xyz, ref):
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)
    G, B, dmin = cref.geometry(*xyz, lx, Dh, w)
    Gr, Br, dJ = geometric_factors(*ref, lx)
    for g, gr in zip(G, Gr):
        assert np.max(np.abs(g - gr)) <= 1e-13 * np.max(np.abs(Gr[0]))
    np.testing.assert_allclose(B, Br, rtol=1e-13)
    assert dmin == pytest.approx(dJ.min(), rel=1e-13)


def test_c_fourier_and_gather_match_oracle():
    n, lx, a = 2, 5, 0.1
    P = BoxProblem(n, lx, a)
    k, am, ph = synth.fourier_modes(3)
    b = cref.gather(P.B * cref.fourier(*P.coords, k, am, ph), P.ids, P.nu)
    np.testing.assert_allclose(b - b.mean(), P.fourier_rhs(k, am, ph), rtol=0,
                               atol=1e-13 * np.max(np.abs(b)))
    v = synth.local_normal(n ** 3, lx, 4)
    np.testing.assert_allclose(cref.gather(v, P.ids, P.nu), gather(v, P.ids, P.nu), rtol=1e-14)


@pytest.mark.parametrize("dirichlet", [False, True])
def test_c_pcg_matches_oracle_pcg(dirichlet):
    """Same iterates as the numpy PCG: iteration counts within 1, solutions
    to the solve's accuracy, true residual at the tolerance."""
    n, lx, a = 3, 4, 0.1
    h1u = synth.unique_uniform(10 ** 6, 0.5, 2.0, 1)
    P = BoxProblem(n, lx, a, dirichlet=dirichlet)
    h1 = h1u[:P.nu]
    P = BoxProblem(n, lx, a, h1_unique=h1, dirichlet=dirichlet)
    k, am, ph = synth.fourier_modes(2)
    b = P.fourier_rhs(k, am, ph)
    xr, itr, _ = pcg(P.apply, b, 1.0 / P.diagonal(), tol=1e-11, project=P.project)
    x, it, rel = cref.pcg(b, P.ids, P.nu, P.Dh, P.h1, P.G, tol=1e-11, project=P.project)
    assert abs(it - itr) <= 1
    assert rel <= 1.5e-11
    np.testing.assert_allclose(x, xr, rtol=0, atol=1e-8 * np.max(np.abs(xr)))
    y = cref.apply_assembled(x, P.ids, P.nu, P.Dh, P.h1, P.G)
    np.testing.assert_allclose(y, P.apply(x), rtol=0, atol=1e-13 * np.max(np.abs(y)))


def test_c_pcg_solves_tiny_box_exactly():
    """Against the pseudo-inverse of the dense assembled matrix (the singular
    periodic operator: mean-free solution)."""
    from oracle.assemble import assembled_matrix
    n, lx, a = 2, 3, 0.08
    P = BoxProblem(n, lx, a)
    A = assembled_matrix(P.Dh, None, P.G, P.ids, P.nu).toarray()
    b = synth.unique_normal(P.nu, 9)
    b -= b.mean()
    x, it, rel = cref.pcg(b, P.ids, P.nu, P.Dh, None, P.G, tol=1e-13)
    xs = np.linalg.pinv(A) @ b
    np.testing.assert_allclose(x, xs, rtol=0, atol=1e-10 * np.max(np.abs(xs)))
    assert abs(x.sum()) <= 1e-12 * np.abs(x).sum()


@pytest.mark.parametrize("dirichlet,h2", [(False, None), (True, None), (False, 7.0), (True, 7.0)])
def test_bigbox_equals_oracle_box(dirichlet, h2):
    n, lx, a = 3, 4, 0.1
    P = BoxProblem(n, lx, a, dirichlet=dirichlet, h2=h2)
    h1u = synth.unique_uniform(P.nu, 0.5, 2.0, 1)
    P = BoxProblem(n, lx, a, h1_unique=h1u, dirichlet=dirichlet, h2=h2)
    Bb = cref.BigBox(n, lx, a, h1_unique=h1u, dirichlet=dirichlet, h2=h2)
    assert Bb.nu == P.nu and Bb.project == P.project
    k, am, ph = synth.fourier_modes(2)
    bref = P.fourier_rhs(k, am, ph)
    np.testing.assert_allclose(Bb.fourier_rhs(k, am, ph), bref, rtol=0, atol=1e-13 * np.max(np.abs(bref)))
    x = synth.unique_normal(P.nu, 3)
    y = P.apply(x)
    np.testing.assert_allclose(Bb.apply(x), y, rtol=0, atol=1e-13 * np.max(np.abs(y)))
    xs, its, _ = pcg(P.apply, bref, 1.0 / P.diagonal(), tol=1e-11, project=P.project)
    xc, itc, rel = Bb.pcg(bref, tol=1e-11)
    assert abs(itc - its) <= 1 and rel <= 1.5e-11
    np.testing.assert_allclose(xc, xs, rtol=0, atol=1e-8 * np.max(np.abs(xs)))
