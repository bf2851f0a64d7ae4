"""Pins for oracle.solve: pseudo-inverse solutions, FCG = PCG for a fixed
preconditioner, spectral convergence of a manufactured solution."""
import numpy as np
import pytest

import synth
from oracle.assemble import assembled_matrix
from oracle.gs import scatter
from oracle.solve import BoxProblem, pcg, fcg1, iterative_refinement


def test_pcg_matches_pseudoinverse():
    n, lx = 2, 4
    P = BoxProblem(n, lx, 0.1, synth.unique_uniform((n * (lx - 1)) ** 3, 0.5, 2.0, 1))
    k, amp, ph = synth.fourier_modes(2, count=8, kmax=2)
    b = P.fourier_rhs(k, amp, ph)
    assert abs(b.sum()) < 1e-13 * np.abs(b).sum()
    A = assembled_matrix(P.Dh, P.h1, P.G, P.ids, P.nu).toarray()
    xref = np.linalg.pinv(A, rcond=1e-12) @ b
    x, it, hist = pcg(P.apply, b, 1.0 / P.diagonal(), tol=1e-12)
    assert hist[-1] <= 1e-12
    assert np.max(np.abs(x - xref)) < 1e-9 * np.max(np.abs(xref))


def test_fcg_reproduces_pcg_with_fixed_preconditioner():
    P = BoxProblem(3, 4, 0.1)
    k, amp, ph = synth.fourier_modes(5)
    b = P.fourier_rhs(k, amp, ph)
    Minv = 1.0 / P.diagonal()
    x1, it1, h1 = pcg(P.apply, b, Minv, tol=1e-10)
    x2, it2, h2 = fcg1(P.apply, b, lambda r: Minv * r, tol=1e-10)
    assert abs(it1 - it2) <= 1
    n = min(len(h1), len(h2), 30)
    np.testing.assert_allclose(h1[:n], h2[:n], rtol=1e-6)
    assert np.max(np.abs(x1 - x2)) < 1e-8 * np.max(np.abs(x1))


def test_manufactured_solution_spectral_convergence():
    """u = sin(2 pi x) sin(2 pi y) sin(2 pi z) solves -lap u = 12 pi^2 u on the
    periodic unit box; the discrete error must fall spectrally in lx."""
    errs = []
    for lx in (4, 6, 8):
        P = BoxProblem(2, lx, 0.0)
        x, y, z = P.coords
        u = np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y) * np.sin(2 * np.pi * z)
        f = 12 * np.pi ** 2 * u
        from oracle.gs import gather
        b = gather(P.B * f, P.ids, P.nu)
        b -= b.mean()
        sol, it, hist = pcg(P.apply, b, 1.0 / P.diagonal(), tol=1e-13)
        ex = np.zeros(P.nu); ex[P.ids.ravel()] = u.ravel()
        errs.append(np.max(np.abs(sol - (ex - ex.mean()))))
    # each step of 2 in lx gains more than two orders of magnitude
    assert errs[0] > 100 * errs[1] and errs[1] > 100 * errs[2]
    assert errs[2] < 1e-6


def test_refinement_with_float32_inner_reaches_float64_tolerance():
    P = BoxProblem(3, 4, 0.1)
    k, amp, ph = synth.fourier_modes(6)
    b = P.fourier_rhs(k, amp, ph)
    Minv = 1.0 / P.diagonal()

    def apply32(v):
        return P.apply(v.astype(np.float32).astype(np.float64)).astype(np.float32).astype(np.float64)

    def inner(rhat):
        d, _, _ = pcg(apply32, rhat, Minv, tol=1e-5, maxit=500)
        return d

    x, outer, relres = iterative_refinement(P.apply, b, inner, tol=1e-10)
    assert relres[-1] <= 1e-10 and outer >= 2
    xref, _, _ = pcg(P.apply, b, Minv, tol=1e-13)
    assert np.max(np.abs(x - xref)) < 1e-7 * np.max(np.abs(xref))


@pytest.mark.parametrize("dirichlet,h2", [(False, None), (True, None), (False, 7.0)])
def test_operator_at_nodes_matches_whole_mesh(dirichlet, h2):
    """The node-by-node operator used by the full-size GPU solve test equals the
    oracle's assembled operator at every node (periodic and Dirichlet box,
    Poisson and Helmholtz)."""
    from tests.helpers import operator_at_nodes
    from oracle.mesh import global_ids, global_ids_dirichlet
    n, lx, amp = (3, 4, 0.12) if dirichlet else (2, 4, 0.12)
    P = BoxProblem(n, lx, amp, dirichlet=dirichlet, h2=h2)
    xG = synth.unique_normal(P.nu, 3)
    ids = global_ids_dirichlet(n, lx) if dirichlet else global_ids(n, lx)
    got = operator_at_nodes(n, lx, amp, ids, xG, np.arange(P.nu), h2=h2)
    ref = P.apply(xG)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_helmholtz_manufactured_solution():
    """(-lap + h2) u = f on the periodic unit box with u = sin(2 pi x)
    sin(2 pi y) sin(2 pi z), f = (12 pi^2 + h2) u: the Helmholtz operator is
    non-singular, so nothing is projected, and the discrete error falls
    spectrally in lx."""
    from oracle.gs import gather
    h2 = 50.0
    errs = []
    for lx in (4, 6, 8):
        P = BoxProblem(2, lx, 0.0, h2=h2)
        assert not P.project
        x, y, z = P.coords
        u = np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y) * np.sin(2 * np.pi * z)
        b = gather(P.B * (12 * np.pi ** 2 + h2) * u, P.ids, P.nu)
        sol, it, hist = pcg(P.apply, b, 1.0 / P.diagonal(), tol=1e-13, project=False)
        ex = np.zeros(P.nu)
        ex[P.ids.ravel()] = u.ravel()
        errs.append(np.max(np.abs(sol - ex)))
    assert errs[0] > 100 * errs[1] and errs[1] > 100 * errs[2]
    assert errs[2] < 1e-6


@pytest.mark.parametrize("dirichlet", [False, True])
def test_helmholtz_operator_bounds(dirichlet):
    """A + h2 B with the diagonal mass: the matrix-free apply equals the
    assembled stiffness plus the assembled (diagonal) mass, and since A is
    positive semi-definite every eigenvalue is at least h2 min_G (Q^T B)_G."""
    from oracle.gs import gather
    h2 = 3.0
    n, lx = (3, 4) if dirichlet else (2, 4)
    P = BoxProblem(n, lx, 0.1, dirichlet=dirichlet, h2=h2)
    A = assembled_matrix(P.Dh, None, P.G, P.ids, P.nu).toarray()
    m = gather(P.B, P.ids, P.nu)
    H = A + np.diag(h2 * m)
    x = synth.unique_normal(P.nu, 4)
    np.testing.assert_allclose(P.apply(x), H @ x, rtol=1e-12, atol=1e-12 * np.abs(H @ x).max())
    np.testing.assert_allclose(P.diagonal(), np.diag(H), rtol=1e-12)
    ev = np.linalg.eigvalsh(0.5 * (H + H.T))
    assert ev[0] >= h2 * m.min() * (1 - 1e-10)
    b = P.fourier_rhs(*synth.fourier_modes(2, count=8, kmax=2))
    xs, _, _ = pcg(P.apply, b, 1.0 / P.diagonal(), tol=1e-12, project=False)
    np.testing.assert_allclose(xs, np.linalg.solve(H, b), rtol=0, atol=1e-9 * np.abs(xs).max())
