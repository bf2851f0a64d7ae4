"""Pins for oracle.mlp: finite differences, Adam closed form, invariances."""
import numpy as np
import pytest

import synth
from oracle import mlp
from oracle.solve import BoxProblem
from oracle.gs import scatter


def _small_net(seed, sizes=(10, 7, 6, 5)):
    return synth.mlp_init(seed, sizes)


@pytest.mark.parametrize("metric,linear", [(False, False), (True, False), (False, True)])
def test_backprop_matches_finite_differences(metric, linear):
    r = np.random.default_rng(0)
    params = _small_net(1)
    params = [p + 0.05 * r.standard_normal(p.shape) for p in params]   # non-zero biases too
    X = r.standard_normal((9, 10))
    T = r.standard_normal((9, 5))
    K = None
    if metric:
        L = r.standard_normal((5, 5))
        K = L @ L.T + 0.1 * np.eye(5)
    lval, grads = mlp.backward(params, X, T, K, linear)
    assert lval == pytest.approx(mlp.loss(params, X, T, K, linear), rel=1e-13)
    h = 1e-6
    for pi, p in enumerate(params):
        fd = np.zeros_like(p)
        for idx in np.ndindex(p.shape):
            pp = [q.copy() for q in params]
            pp[pi][idx] += h
            lp = mlp.loss(pp, X, T, K, linear)
            pp[pi][idx] -= 2 * h
            lm = mlp.loss(pp, X, T, K, linear)
            fd[idx] = (lp - lm) / (2 * h)
        assert np.max(np.abs(fd - grads[pi])) <= 1e-6 * max(1.0, np.max(np.abs(fd))), pi


def test_reference_metric():
    """Stiffness part: exact energy of a degree-N polynomial on the reference
    cube [-1, 1]^3 (geometric factors w w w, kappa = mean(w w w)); with the
    mass term the metric is positive definite."""
    lx = 5
    from oracle.gll import gll_nodes_weights
    xi, w = gll_nodes_weights(lx - 1)
    K0 = mlp.reference_metric(lx, mu=0.0)
    K1 = mlp.reference_metric(lx, mu=1.0)
    np.testing.assert_allclose(K1, K1.T, atol=1e-13)
    ev = np.linalg.eigvalsh(K1)
    assert ev[0] > 1e-3
    assert abs(np.linalg.eigvalsh(K0)[0]) < 1e-10        # constants: zero stiffness
    Z, Y, Xc = np.meshgrid(xi, xi, xi, indexing="ij")
    u = (Xc ** 2 * Y + 0.5 * Z ** 3 - Xc * Y * Z).ravel()   # total degree 3 <= N = 4
    kappa = np.mean(w[:, None, None] * w[None, :, None] * w[None, None, :])
    gq, gw = np.polynomial.legendre.leggauss(6)
    Qz, Qy, Qx = np.meshgrid(gq, gq, gq, indexing="ij")
    Wq = gw[:, None, None] * gw[None, :, None] * gw[None, None, :]
    grad2 = (2 * Qx * Qy - Qy * Qz) ** 2 + (Qx ** 2 - Qx * Qz) ** 2 + (1.5 * Qz ** 2 - Qx * Qy) ** 2
    assert u @ K0 @ u == pytest.approx(np.sum(Wq * grad2) / kappa, rel=1e-12)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are exactly g and
    g^2, so every step moves by -lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    p = [np.zeros(3)]
    m, v = [np.zeros(3)], [np.zeros(3)]
    for t in range(1, 6):
        p, m, v = mlp.adam_step(p, [g], m, v, t, lr=1e-2)
    np.testing.assert_allclose(p[0], -5 * 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_features_scale_invariance():
    """Scaling the residual leaves the inputs unchanged; scaling the geometry
    scales kappa and leaves the geometric features unchanged."""
    G, h1 = synth.random_spd_factors(3, 4, 2)
    r = synth.local_normal(3, 4, 3)
    X, s, k = mlp.features(r, G, h1)
    X2, s2, k2 = mlp.features(7.0 * r, tuple(3.0 * g for g in G), h1)
    np.testing.assert_allclose(X, X2, rtol=1e-13)
    np.testing.assert_allclose(s2, 7 * s, rtol=1e-13)
    np.testing.assert_allclose(k2, 3 * k, rtol=1e-13)
    assert X.shape == (3, 518 - 512 + 64)
    np.testing.assert_allclose(np.sum(X[:, :64] ** 2, axis=1), 1.0, rtol=1e-12)


def test_apply_is_continuous():
    P = BoxProblem(2, 4, 0.1)
    sizes = (64 + 6, 16, 16, 64)
    params = synth.mlp_init(4, sizes)
    rG = synth.unique_normal(P.nu, 5)
    r = scatter(rG, P.ids)
    z = mlp.apply(params, r, P.G, None, P.ids, P.nu)
    # every copy of a node carries the same value
    zg = np.zeros(P.nu)
    zg[P.ids.ravel()] = z.ravel()
    np.testing.assert_allclose(z, zg[P.ids], rtol=1e-14)


def test_linear_form_is_linear():
    params = _small_net(3)
    r = np.random.default_rng(1)
    x1, x2 = r.standard_normal((4, 10)), r.standard_normal((4, 10))
    f = lambda x: mlp.forward(params, x, linear=True)[2]  # noqa: E731
    np.testing.assert_allclose(f(2.0 * x1 - 3.0 * x2), 2.0 * f(x1) - 3.0 * f(x2), atol=1e-12)


def _identity_params(nloc, ngeo=6):
    W1 = np.zeros((nloc, nloc + ngeo))
    W1[:, :nloc] = np.eye(nloc)
    W1[:, nloc:] = 1.0      # geometric inputs do not enter the linear form
    return [W1, np.ones(nloc), np.eye(nloc), np.ones(nloc), np.eye(nloc), np.ones(nloc)]


@pytest.mark.parametrize("amp", [0.0, 0.15])
def test_linear_apply_identity_block_is_partition_of_unity(amp):
    """An identity folded matrix gives z_u = r_u * mean_{e containing u} 1/kappa_e
    (sum over copies of S^2 = 1): r / kappa on the undeformed box."""
    lx = 4
    P = BoxProblem(2, lx, amp)
    rG = synth.unique_normal(P.nu, 11)
    z = mlp.apply_linear(_identity_params(lx ** 3), scatter(rG, P.ids), P.G, None, P.ids, P.nu)
    _, _, kappa = mlp.features(scatter(rG, P.ids), P.G)
    inv_k = np.zeros(P.nu)
    cnt = np.zeros(P.nu)
    for e in range(P.ids.shape[0]):
        np.add.at(inv_k, P.ids[e].ravel(), 1.0 / kappa[e])
        np.add.at(cnt, P.ids[e].ravel(), 1.0)
    expect = rG * inv_k / cnt
    np.testing.assert_allclose(z, expect[P.ids], rtol=1e-13, atol=0)
    if amp == 0.0:
        assert np.ptp(kappa) <= 1e-14 * kappa[0]
        np.testing.assert_allclose(z, scatter(rG / kappa[0], P.ids), rtol=1e-13)


def _dense_precond(params, P):
    cols = []
    for j in range(P.nu):
        ej = np.zeros(P.nu)
        ej[j] = 1.0
        z = mlp.apply_linear(params, scatter(ej, P.ids), P.G, None, P.ids, P.nu)
        zu = np.zeros(P.nu)
        zu[P.ids.ravel()] = z.ravel()
        cols.append(zu)
    return np.array(cols).T


def test_linear_apply_symmetric_and_positive_definite():
    """The linear apply is an exactly symmetric operator for any weights, and
    positive definite when the folded matrix is (W = C^T C)."""
    lx = 3
    nloc = lx ** 3
    P = BoxProblem(2, lx, 0.1)
    r = np.random.default_rng(3)
    params = [r.standard_normal(p.shape) for p in synth.mlp_init(5, (nloc + 6, 9, 9, nloc))]
    M = _dense_precond(params, P)
    assert np.linalg.norm(M - M.T) <= 1e-13 * np.linalg.norm(M)
    W = mlp.folded_matrix(params, nloc)
    assert np.linalg.norm(W - W.T) >= 0.1 * np.linalg.norm(W)     # the weights are not symmetric
    C = r.standard_normal((nloc, nloc))
    W1 = np.concatenate([C, r.standard_normal((nloc, 6))], axis=1)
    spd = [W1, np.zeros(nloc), np.eye(nloc), np.zeros(nloc), C.T.copy(), np.zeros(nloc)]
    ev = np.linalg.eigvalsh(_dense_precond(spd, P))
    assert ev[0] > 1e-8 * ev[-1]


def test_linear_apply_at_nodes_matches_whole_mesh():
    """The node-by-node evaluation used by the full-size GPU test equals the
    oracle's whole-mesh linear apply (plus the Jacobi term) at every node."""
    from tests.helpers import linear_apply_at_nodes
    from oracle.assemble import element_diagonal
    n, lx, amp = 2, 4, 0.12
    P = BoxProblem(n, lx, amp)
    r = np.random.default_rng(9)
    params = [r.standard_normal(p.shape) for p in synth.mlp_init(5, (lx ** 3 + 6, 20, 20, lx ** 3))]
    rG = synth.unique_normal(P.nu, 10)
    z = mlp.apply_linear(params, scatter(rG, P.ids), P.G, None, P.ids, P.nu)
    zu = np.zeros(P.nu)
    zu[P.ids.ravel()] = z.ravel()
    zu += rG / P.diagonal()
    got = linear_apply_at_nodes(params, n, lx, amp, P.ids, rG, np.arange(P.nu), jacobi=True)
    np.testing.assert_allclose(got, zu, rtol=1e-12, atol=1e-12 * np.abs(zu).max())
