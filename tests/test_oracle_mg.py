"""Pins for oracle.mg: transfers against closed forms, the Chebyshev steps
against the closed-form polynomial, the two-level V-cycle against dense
algebra, and the preconditioner's mesh independence."""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as C

import synth
from oracle import mg
from oracle.solve import BoxProblem, fcg1, pcg


def test_level_shapes():
    assert mg.level_shapes(32, 8) == [(32, 8, "p"), (32, 4, "p"), (32, 2, "h"), (16, 2, "h"), (8, 2, "h"),
                                      (4, 2, "h"), (2, 2, None)]
    assert mg.level_shapes(32, 8, n_coarse=8) == [(32, 8, "p"), (32, 4, "p"), (32, 2, "h"), (16, 2, "h"),
                                                  (8, 2, None)]
    assert mg.level_shapes(3, 10) == [(3, 10, "p"), (3, 5, "p"), (3, 2, None)]
    assert mg.level_shapes(6, 2) == [(6, 2, "h"), (3, 2, None)]


def test_p_transfer_reproduces_coarse_polynomials():
    """On the undeformed Dirichlet box u = x(1-x) y(1-y) z(1-z) is, element by
    element, a polynomial of degree 2 per direction: the lx = 4 level holds it
    exactly and P returns its values at the lx = 8 nodes."""
    n = 2
    fine, coarse = BoxProblem(n, 8, 0.0, dirichlet=True), BoxProblem(n, 4, 0.0, dirichlet=True)
    P = mg.prolongation(fine, coarse, "p")

    def nodal(B):
        x, y, z = B.coords
        u = (x * (1 - x) * y * (1 - y) * z * (1 - z))
        out = np.zeros(B.nu)
        out[B.ids[B.ids >= 0]] = u[B.ids >= 0]
        return out
    np.testing.assert_allclose(P @ nodal(coarse), nodal(fine), rtol=0, atol=1e-15)


def test_h_transfer_is_trilinear_interpolation():
    """Undeformed periodic lx = 2 boxes 4^3 -> 2^3: a fine lattice node with
    coordinates (I, J, K) gets the mean of the coarse values at
    (floor(I/2) or ceil(I/2), ...) -- the coarse value at even coordinates,
    the mean of 2, 4 or 8 neighbours at edge, face and cell midpoints."""
    fine, coarse = BoxProblem(4, 2, 0.0), BoxProblem(2, 2, 0.0)
    P = mg.prolongation(fine, coarse, "h")
    uc = synth.unique_normal(coarse.nu, 3)
    got = P @ uc
    Mf, Mc = 4, 2
    want = np.empty(fine.nu)
    for g in range(fine.nu):
        I, J, K = g % Mf, (g // Mf) % Mf, g // (Mf * Mf)
        acc, cnt = 0.0, 0
        for a in {I // 2, (I + 1) // 2}:
            for b in {J // 2, (J + 1) // 2}:
                for c in {K // 2, (K + 1) // 2}:
                    acc += uc[(c % Mc) * Mc * Mc + (b % Mc) * Mc + (a % Mc)]
                    cnt += 1
        want[g] = acc / cnt
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("kind,shapes", [("p", ((2, 6), (2, 3))), ("h", ((4, 2), (2, 2)))])
def test_transfer_keeps_constants(kind, shapes):
    (nf, lf), (nc, lc) = shapes
    P = mg.prolongation(BoxProblem(nf, lf, 0.12), BoxProblem(nc, lc, 0.12), kind)
    np.testing.assert_allclose(P @ np.ones(P.shape[1]), 1.0, rtol=0, atol=1e-14)


def _pencil(A, dinv):
    """V, lam with D^-1/2 A D^-1/2 = V diag(lam) V^T"""
    Dm = np.sqrt(dinv)
    lam, V = np.linalg.eigh((Dm[:, None] * A) * Dm[None, :])
    return Dm, lam, V


def _cheb_error_matrix(A, dinv, k, lo, hi):
    """Error propagator of k Chebyshev steps: p(D^-1 A), p(l) = T_k((theta - l) /
    delta) / T_k(theta / delta)."""
    Dm, lam, V = _pencil(A, dinv)
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    Tk = np.zeros(k + 1)
    Tk[k] = 1.0
    p = C.chebval((theta - lam) / delta, Tk) / C.chebval(theta / delta, Tk)
    # D^-1 A = D^-1/2 M D^1/2 with M = D^-1/2 A D^-1/2
    return Dm[:, None] * ((V * p) @ V.T) * (1.0 / Dm)[None, :]


@pytest.mark.parametrize("k", [1, 2, 4])
def test_chebyshev_equals_closed_form_polynomial(k):
    B = BoxProblem(2, 3, 0.1, dirichlet=True)
    from oracle.assemble import assembled_matrix
    A = assembled_matrix(B.Dh, None, B.G, B.ids, B.nu).toarray()
    dinv = 1.0 / np.diag(A)
    lmax = _pencil(A, dinv)[1][-1]
    lo, hi = 0.3 * lmax, 1.1 * lmax
    xs = synth.unique_normal(B.nu, 4)
    b = A @ xs
    x0 = synth.unique_normal(B.nu, 5)
    xk = mg.chebyshev(lambda v: A @ v, dinv, b, x0, k, lo, hi)
    E = _cheb_error_matrix(A, dinv, k, lo, hi)
    np.testing.assert_allclose(xs - xk, E @ (xs - x0), rtol=0, atol=1e-12 * np.abs(xs).max())
    # from zero the first step is D^-1 b / theta
    x1 = mg.chebyshev(lambda v: A @ v, dinv, b, None, 1, lo, hi)
    np.testing.assert_allclose(x1, dinv * b / (0.5 * (lo + hi)), rtol=1e-14)


@pytest.mark.parametrize("h2", [None, 5.0])
def test_two_level_vcycle_matches_dense_algebra(h2):
    """Dirichlet box, levels lx = 4 -> 2: I - V A = S (I - P A_c^-1 P^T A) S
    with S the Chebyshev error propagator, and V symmetric positive definite."""
    H = mg.Hierarchy(2, 4, 0.1, dirichlet=True, h2=h2, degree=3)
    assert len(H.shapes) == 2
    A = H.A[0].toarray()
    V = H.matrix()
    S = _cheb_error_matrix(A, H.dinv[0], H.degree, H.lo * H.lmax[0], H.hi * H.lmax[0])
    P = H.P[0].toarray()
    Ac = H.A[1].toarray()
    E = S @ (np.eye(len(A)) - P @ np.linalg.solve(Ac, P.T @ A)) @ S
    np.testing.assert_allclose(np.eye(len(A)) - V @ A, E, rtol=0, atol=1e-10)
    np.testing.assert_allclose(V, V.T, rtol=0, atol=1e-12 * np.abs(V).max())
    assert np.linalg.eigvalsh(0.5 * (V + V.T))[0] > 0


def test_coarse_solve_is_pseudo_inverse_on_mean_free_vectors():
    H = mg.Hierarchy(2, 2, 0.1)                 # a single (periodic, singular) level
    A = H.A[0].toarray()
    b = synth.unique_normal(len(A), 6)
    b -= b.mean()
    np.testing.assert_allclose(H.vcycle(b), np.linalg.pinv(A) @ b, rtol=0, atol=1e-10)


@pytest.mark.parametrize("dirichlet", [False, True])
def test_vcycle_preconditioner_is_mesh_independent(dirichlet):
    """Flexible CG with the V-cycle needs about as many iterations on 8^3 as on
    4^3 elements (lx = 4), and far fewer than Jacobi-PCG."""
    its = []
    for n in (4, 8):
        H = mg.Hierarchy(n, 4, 0.1, dirichlet=dirichlet)
        B = H.boxes[0]
        k, a, ph = synth.fourier_modes(2, kmax=2)
        b = B.fourier_rhs(k, a, ph)
        x, it, _ = fcg1(B.apply, b, H.vcycle, tol=1e-10, project=B.project)
        assert np.linalg.norm(b - B.apply(x)) <= 1.2e-10 * np.linalg.norm(b)
        _, itj, _ = pcg(B.apply, b, 1.0 / B.diagonal(), tol=1e-10, project=B.project)
        assert it < 0.5 * itj
        its.append(it)
    assert its[1] <= 1.5 * its[0], its


def test_folding_coarse_levels_take_a_halved_amplitude():
    """At amplitude 0.15 the lx = 2 box of 4^3 elements folds (its vertex
    Jacobians go negative), the lx = 4 one does not: the hierarchy keeps 0.15
    on the levels that stay unfolded and halves it on the one that folds,
    exactly as often as needed (the amplitude taken has det J > 0, twice it
    does not); the V-cycle stays an SPD preconditioner that beats Jacobi."""
    from oracle.mesh import box_coords
    from oracle.geometry import geometric_factors
    H = mg.Hierarchy(4, 4, 0.15, dirichlet=True)
    assert [s[:2] for s in H.shapes] == [(4, 4), (4, 2), (2, 2)]
    assert H.amps[0] == 0.15 and H.amps[2] == 0.15
    a1 = H.amps[1]
    assert 0 < a1 < 0.15 and 0.15 / a1 == 2 ** round(np.log2(0.15 / a1))
    assert np.min(geometric_factors(*box_coords(4, 2, a1), 2)[2]) > 0
    assert np.min(geometric_factors(*box_coords(4, 2, 2 * a1), 2)[2]) <= 0
    V = H.matrix()
    assert np.allclose(V, V.T, rtol=0, atol=1e-12 * np.abs(V).max())
    assert np.linalg.eigvalsh(0.5 * (V + V.T))[0] > 0
    B = H.boxes[0]
    k, a, ph = synth.fourier_modes(2, kmax=2)
    b = B.fourier_rhs(k, a, ph)
    x, it, _ = fcg1(B.apply, b, H.vcycle, tol=1e-10, project=B.project)
    assert np.linalg.norm(b - B.apply(x)) <= 1.2e-10 * np.linalg.norm(b)
    _, itj, _ = pcg(B.apply, b, 1.0 / B.diagonal(), tol=1e-10, project=B.project)
    assert it < 0.5 * itj


@pytest.mark.parametrize("dirichlet,h2", [(True, None), (False, None), (False, 5.0)])
def test_galerkin_coarse_correction_is_an_a_orthogonal_projection(dirichlet, h2):
    """With Galerkin levels the two-grid coarse correction T = I - P A_c^-1 P^T A
    of every level pair is idempotent and A-self-adjoint (A T = T^T A); the
    re-discretised levels of the same box do not have this property.  On the
    periodic Poisson box the singular levels keep the constants in their null
    space.  The box folds at amplitude 0.15 (4^3 elements, lx = 4 -> 2 -> 2)."""
    kw = dict(dirichlet=dirichlet, h2=h2)
    Hg = mg.Hierarchy(4, 4, 0.15, galerkin=True, **kw)
    Hr = mg.Hierarchy(4, 4, 0.15, **kw)
    assert [s[:2] for s in Hg.shapes] == [(4, 4), (4, 2), (2, 2)]
    assert Hg.galerkin == [False, True, True] and Hg.amps[1:] == [0.0, 0.0]

    def defect(H, q):
        A = H.A[q].toarray()
        P = H.P[q].toarray()
        Ac = H.A[q + 1].toarray()
        if H.boxes[q + 1].project:       # singular: solve on the complement of the constants
            Ac = Ac + np.ones_like(Ac)
        T = np.eye(len(A)) - P @ np.linalg.solve(Ac, P.T @ A)
        scale = np.abs(T).max()
        return np.abs(T @ T - T).max() / scale, np.abs(A @ T - T.T @ A).max() / (np.abs(A).max() * scale)

    for q in range(2):
        idem, sym = defect(Hg, q)
        assert idem <= 1e-10 and sym <= 1e-10, (q, idem, sym)
    assert max(defect(Hr, 0)) > 1e-3        # re-discretised: not a projection
    if not dirichlet and h2 is None:
        for q in (1, 2):
            one = np.ones(Hg.boxes[q].nu)
            assert np.abs(Hg.A[q] @ one).max() <= 1e-12 * abs(Hg.A[q]).max()


def test_galerkin_levels_beat_rediscretised_ones_on_a_folding_box():
    """On an 8^3 lx = 4 Dirichlet box at amplitude 0.15 (its lx = 2 levels
    fold), flexible CG with the Galerkin V-cycle converges in fewer iterations
    than with the re-discretised one; both reach relres 1e-10 and the Galerkin
    V-cycle is symmetric positive definite on a smaller box."""
    its = {}
    for g in (False, True):
        H = mg.Hierarchy(8, 4, 0.15, dirichlet=True, galerkin=g)
        B = H.boxes[0]
        k, a, ph = synth.fourier_modes(2, kmax=2)
        b = B.fourier_rhs(k, a, ph)
        x, its[g], _ = fcg1(B.apply, b, H.vcycle, tol=1e-10, project=B.project)
        assert np.linalg.norm(b - B.apply(x)) <= 1.2e-10 * np.linalg.norm(b)
    assert its[True] < its[False], its
    V = mg.Hierarchy(2, 4, 0.15, dirichlet=True, galerkin=True).matrix()
    assert np.allclose(V, V.T, rtol=0, atol=1e-12 * np.abs(V).max())
    assert np.linalg.eigvalsh(0.5 * (V + V.T))[0] > 0
