"""Pins for oracle.mlp: finite differences, Adam closed form, invariances."""
import numpy as np
import pytest

import synth
from oracle import mlp
from oracle.solve import BoxProblem
from oracle.gs import scatter


def _small_net(seed, sizes=(10, 7, 6, 5)):
    return synth.mlp_init(seed, sizes)


def test_backprop_matches_finite_differences():
    r = np.random.default_rng(0)
    params = _small_net(1)
    params = [p + 0.05 * r.standard_normal(p.shape) for p in params]   # non-zero biases too
    X = r.standard_normal((9, 10))
    T = r.standard_normal((9, 5))
    _, grads = mlp.backward(params, X, T)
    h = 1e-6
    for pi, p in enumerate(params):
        fd = np.zeros_like(p)
        for idx in np.ndindex(p.shape):
            pp = [q.copy() for q in params]
            pp[pi][idx] += h
            lp = mlp.loss(pp, X, T)
            pp[pi][idx] -= 2 * h
            lm = mlp.loss(pp, X, T)
            fd[idx] = (lp - lm) / (2 * h)
        assert np.max(np.abs(fd - grads[pi])) <= 1e-6 * max(1.0, np.max(np.abs(fd))), pi


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
