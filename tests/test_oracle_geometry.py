"""Pins for oracle.geometry and oracle.mesh."""
import numpy as np
import pytest

from oracle.gll import gll_nodes_weights
from oracle.mesh import reference_coords, deform, global_ids, n_unique
from oracle.geometry import geometric_factors, box_geometry


@pytest.mark.parametrize("n,lx", [(2, 3), (3, 5), (2, 8)])
def test_axis_aligned_cube(n, lx):
    G, B, detJ = box_geometry(n, lx, 0.0)
    _, w = gll_nodes_weights(lx - 1)
    h = 1.0 / n
    wq = w[:, None, None] * w[None, :, None] * w[None, None, :]
    for g in G[:3]:
        np.testing.assert_allclose(g, np.broadcast_to(0.5 * h * wq, g.shape), rtol=1e-13)
    for g in G[3:]:
        assert np.max(np.abs(g)) < 1e-14
    np.testing.assert_allclose(detJ, h ** 3 / 8, rtol=1e-13)
    assert abs(B.sum() - 1.0) < 1e-13


def test_general_affine_element():
    """x = A r + c with a full (sheared) matrix A: constant Jacobian, so
    G = w_i w_j w_k |det A| A^-1 A^-T exactly."""
    lx = 5
    r = np.random.default_rng(0)
    A = np.eye(3) + 0.3 * r.standard_normal((3, 3))
    c = r.standard_normal(3)
    xi, w = gll_nodes_weights(lx - 1)
    R = np.stack(np.meshgrid(xi, xi, xi, indexing="ij")[::-1], -1)  # [k][j][i] -> (r, s, t)
    X = R @ A.T + c
    x, y, z = (X[None, ..., d] for d in range(3))
    G, B, detJ = geometric_factors(x, y, z, lx)
    Ai = np.linalg.inv(A)
    M = abs(np.linalg.det(A)) * Ai @ Ai.T
    wq = w[:, None, None] * w[None, :, None] * w[None, None, :]
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    for g, (a, b) in zip(G, pairs):
        np.testing.assert_allclose(g[0], M[a, b] * wq, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(detJ, np.linalg.det(A), rtol=1e-12)


def test_isoparametric_jacobian_converges_to_analytic():
    """On the sine-deformed box the GLL-interpolated Jacobian converges
    spectrally to the analytic one: check det J at lx = 12."""
    n, lx, a = 2, 12, 0.1
    X, Y, Z = reference_coords(n, lx)
    _, _, detJ = geometric_factors(*deform(X, Y, Z, a), lx)
    tp = 2 * np.pi
    J = np.empty(X.shape + (3, 3))
    J[..., 0, 0] = 1; J[..., 0, 1] = a * tp * np.cos(tp * Y) * np.sin(tp * Z)
    J[..., 0, 2] = a * tp * np.sin(tp * Y) * np.cos(tp * Z)
    J[..., 1, 1] = 1; J[..., 1, 2] = a * tp * np.cos(tp * Z) * np.sin(tp * X)
    J[..., 1, 0] = a * tp * np.sin(tp * Z) * np.cos(tp * X)
    J[..., 2, 2] = 1; J[..., 2, 0] = a * tp * np.cos(tp * X) * np.sin(tp * Y)
    J[..., 2, 1] = a * tp * np.sin(tp * X) * np.cos(tp * Y)
    ref = np.linalg.det(J) * (0.5 / n) ** 3
    assert np.max(np.abs(detJ - ref)) / np.max(np.abs(ref)) < 1e-6


@pytest.mark.parametrize("a", [0.0, 0.1, 0.15])
def test_deformed_volume(a):
    G, B, detJ = box_geometry(3, 8, a)
    assert abs(B.sum() - 1.0) < 1e-12
    assert detJ.min() > 0


def test_folding_amplitude():
    """The map folds where 1 - (2 pi a)^2 ... reaches zero: det J stays positive
    at a = 0.15 and turns negative at a = 0.2 (the analytic threshold is
    a = 1 / (2 pi))."""
    _, _, d15 = box_geometry(4, 8, 0.15)
    _, _, d20 = box_geometry(4, 8, 0.20)
    assert d15.min() > 0 > d20.min()


def test_global_ids_periodic():
    n, lx = 3, 4
    ids = global_ids(n, lx)
    assert ids.min() == 0 and ids.max() == n_unique(n, lx) - 1
    assert len(np.unique(ids)) == n_unique(n, lx)
    # physical coincidence: copies of an id sit at the same point modulo 1
    X, Y, Z = reference_coords(n, lx)
    P = np.stack([X, Y, Z], -1).reshape(-1, 3) % 1.0
    P = np.where(np.abs(P - 1.0) < 1e-12, 0.0, P)
    flat = ids.ravel()
    order = np.argsort(flat, kind="stable")
    first = {}
    for L in order:
        g = flat[L]
        if g in first:
            assert np.allclose(P[L], P[first[g]], atol=1e-12)
        else:
            first[g] = L
