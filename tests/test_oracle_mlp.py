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


# ----------------------------------------------------------------------------
# Closed-form pins of features, targets and the nonlinear apply.  On an
# axis-aligned rectangular element [0, a] x [0, b] x [0, c] the Jacobian is
# diag(a, b, c) / 2, so g11 = w_i w_j w_k bc / (2a), g22 = w w w ac / (2b),
# g33 = w w w ab / (2c) and the off-diagonal factors vanish; the mean of
# w_i w_j w_k over the lx^3 nodes is (sum w)^3 / lx^3 = 8 / lx^3.  Hence
#   kappa = (8 / lx^3) (bc/a + ac/b + ab/c) / 6,
#   geometric features = (bc/a, ac/b, ab/c, 0, 0, 0) * (8 / lx^3) / kappa.
# On the uniform periodic box with side h = 1/n: kappa = 4 h / lx^3 and the
# features are (1, 1, 1, 0, 0, 0).

def _rect_element(lx, a, b, c):
    from oracle.gll import gll_nodes_weights
    xi, _ = gll_nodes_weights(lx - 1)
    Z, Y, X = np.meshgrid(c * (1 + xi) / 2, b * (1 + xi) / 2, a * (1 + xi) / 2, indexing="ij")
    return X[None], Y[None], Z[None]


@pytest.mark.parametrize("lx,dims", [(4, (1.0, 1.0, 1.0)), (5, (0.3, 0.7, 1.9)), (8, (2.0, 0.5, 0.25))])
def test_features_closed_form_on_rectangular_element(lx, dims):
    """kappa (with its 1/3) and the order g11, g22, g33, g12, g13, g23 of the
    geometric features against the rectangle's closed form.  A kappa without
    the 1/3, a permuted feature order or a dropped weight fails."""
    from oracle.geometry import geometric_factors
    a, b, c = dims
    G, _, _ = geometric_factors(*_rect_element(lx, a, b, c), lx)
    r = synth.local_normal(1, lx, 4)
    X, s, kappa = mlp.features(r, G)
    diag = np.array([b * c / a, a * c / b, a * b / c])
    kappa_cf = (8.0 / lx ** 3) * diag.sum() / 6.0
    assert kappa[0] == pytest.approx(kappa_cf, rel=1e-13)
    geo_cf = np.concatenate([diag * (8.0 / lx ** 3) / 2.0 / kappa_cf, np.zeros(3)])
    np.testing.assert_allclose(X[0, lx ** 3:], geo_cf, rtol=1e-13, atol=1e-14)
    assert s[0] == pytest.approx(np.sqrt(np.sum(r ** 2)), rel=1e-14)
    np.testing.assert_allclose(X[0, :lx ** 3], r.ravel() / np.sqrt(np.sum(r ** 2)), rtol=1e-13)


def test_features_sheared_element_off_diagonal_order():
    """An affine element x = A xi (xi in [-1, 1]^3): g_ab = w w w |det A|
    (A^-1 A^-T)_ab, so the off-diagonal features come in the order (r,s),
    (r,t), (s,t).  A is chosen with three distinct off-diagonal entries."""
    from oracle.geometry import geometric_factors
    from oracle.gll import gll_nodes_weights
    lx = 4
    A = np.array([[1.0, 0.2, -0.1], [0.05, 0.8, 0.3], [0.0, -0.15, 1.2]])
    xi, _ = gll_nodes_weights(lx - 1)
    T, S, R = np.meshgrid(xi, xi, xi, indexing="ij")
    P = np.einsum("ca,a...->c...", A, np.stack([R, S, T]))
    G, _, _ = geometric_factors(P[0][None], P[1][None], P[2][None], lx)
    _, _, kappa = mlp.features(synth.local_normal(1, lx, 1), G)
    Ai = np.linalg.inv(A)
    M = Ai @ Ai.T * abs(np.linalg.det(A)) * (8.0 / lx ** 3)
    assert kappa[0] == pytest.approx(np.trace(M) / 3.0, rel=1e-12)
    X, _, _ = mlp.features(synth.local_normal(1, lx, 1), G)
    want = np.array([M[0, 0], M[1, 1], M[2, 2], M[0, 1], M[0, 2], M[1, 2]]) / kappa[0]
    np.testing.assert_allclose(X[0, lx ** 3:], want, rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("n,lx", [(2, 4), (3, 3)])
def test_features_uniform_box_closed_form(n, lx):
    P = BoxProblem(n, lx, 0.0)
    r = synth.local_normal(n ** 3, lx, 2)
    X, _, kappa = mlp.features(r, P.G)
    np.testing.assert_allclose(kappa, 4.0 / n / lx ** 3, rtol=1e-13)
    np.testing.assert_allclose(X[:, lx ** 3:], np.tile([1, 1, 1, 0, 0, 0], (n ** 3, 1)),
                               rtol=1e-13, atol=1e-14)


def test_targets_closed_form():
    """t_e = err_e kappa_e / s_e with the closed-form kappa of the uniform box
    (4 h / lx^3) and s_e the 2-norm of the element's residual."""
    n, lx = 2, 4
    P = BoxProblem(n, lx, 0.0)
    r = synth.local_normal(n ** 3, lx, 5)
    err = synth.local_normal(n ** 3, lx, 6)
    _, s, kappa = mlp.features(r, P.G)
    T = mlp.targets(err, s, kappa)
    norms = np.sqrt(np.sum(r.reshape(n ** 3, -1) ** 2, axis=1))
    np.testing.assert_allclose(T, err.reshape(n ** 3, -1) * (4.0 / n / lx ** 3) / norms[:, None],
                               rtol=1e-13)


def _constant_output_params(lx, out):
    """Network with zero weights and last-layer bias `out`: NN(x) = out."""
    p = synth.mlp_init(3, (lx ** 3 + 6, 16, 16, lx ** 3))
    return [np.zeros_like(p[0]), np.zeros_like(p[1]), np.zeros_like(p[2]),
            np.zeros_like(p[3]), np.zeros_like(p[4]), np.asarray(out, dtype=np.float64)]


@pytest.mark.parametrize("n,lx,c", [(2, 4, 1.0), (3, 3, -2.5)])
def test_nonlinear_apply_constant_residual_closed_form(n, lx, c):
    """NN = 1 at every output and r = c on the uniform box: every element has
    s = |c| sqrt(lx^3) and kappa = 4 h / lx^3, so z_e = s / kappa and the
    partition-of-unity average returns z = |c| sqrt(lx^3) lx^3 n / 4 at every
    node.  A dropped mult^-1 multiplies shared nodes by their multiplicity; a
    dropped s or 1/kappa changes the constant."""
    P = BoxProblem(n, lx, 0.0)
    r = np.full((n ** 3, lx, lx, lx), c)
    z = mlp.apply(_constant_output_params(lx, np.ones(lx ** 3)), r, P.G, None, P.ids, P.nu)
    np.testing.assert_allclose(z, abs(c) * np.sqrt(lx ** 3) * lx ** 3 * n / 4.0, rtol=1e-12)


def test_nonlinear_apply_averages_element_outputs():
    """NN = v (a fixed output vector) on a deformed box: every local node of a
    global node u receives (1 / mult_u) sum over the copies (e, p) of u of
    (s_e / kappa_e) v_p, computed here copy by copy."""
    n, lx = 2, 3
    P = BoxProblem(n, lx, 0.1)
    v = np.linspace(0.5, 1.5, lx ** 3)
    rG = synth.unique_normal(P.nu, 8)
    r = scatter(rG, P.ids)
    z = mlp.apply(_constant_output_params(lx, v), r, P.G, None, P.ids, P.nu)
    E = n ** 3
    acc = np.zeros(P.nu)
    cnt = np.zeros(P.nu)
    for e in range(E):
        s_e = np.sqrt(np.sum(r[e] ** 2))
        g = [gg[e] for gg in P.G]
        kap = np.mean(g[0] + g[1] + g[2]) / 3.0
        for p, gid in enumerate(P.ids[e].ravel()):
            acc[gid] += s_e / kap * v[p]
            cnt[gid] += 1
    np.testing.assert_allclose(z, (acc / cnt)[P.ids], rtol=1e-12)


# ----------------------------------------------------------------------------
# bfloat16-storage emulation (forward_bf16, backward_bf16, apply_bf16,
# apply_block_bf16).  Exactness pin: with operands drawn from a few dyadic
# values and banded weights (at most two nonzeros per row and per column),
# every intermediate has few significant bits, so rounding to bfloat16 or
# float32 changes nothing and the emulation must equal the exact functions.

def _banded(rows, cols, r, scale=0.125):
    W = np.zeros((rows, cols))
    for i in range(rows):
        for j in (i % cols, (i + 1) % cols):
            W[i, j] = scale * r.choice([-1.0, 1.0])
    return W


def _dyadic_net(r, sizes=(10, 7, 6, 4)):
    p = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        p.append(_banded(b, a, r))
        p.append(r.choice([-0.125, 0.0, 0.125, 0.25], size=b))
    return p


@pytest.mark.parametrize("linear", [False, True])
@pytest.mark.parametrize("metric", [False, True])
def test_bf16_forms_exact_on_bf16_numbers(linear, metric):
    r = np.random.default_rng(5)
    params = _dyadic_net(r)
    B = 4          # the loss scales 2 / (B * 4) and 2 / B are powers of two
    X = r.choice([-0.75, -0.5, -0.25, 0.25, 0.5, 0.75], size=(B, 10))
    y3 = mlp.forward(params, X, linear)[2]
    np.testing.assert_array_equal(mlp.forward_bf16(params, X, linear)[2], y3)
    T = y3 - r.choice([-0.125, -0.0625, 0.0625, 0.125], size=y3.shape)
    K = None
    if metric:
        K = _banded(4, 4, r)
        K = 0.5 * (K + K.T)
    l_ref, g_ref = mlp.backward(params, X, T, K, linear)
    l_q, g_q = mlp.backward_bf16(params, X, T, K, linear)
    assert l_q == pytest.approx(l_ref, rel=1e-14)
    for a, b in zip(g_q, g_ref):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-15)


@pytest.mark.parametrize("linear", [False, True])
def test_bf16_forms_within_rounding_of_exact_forms(linear):
    """On random He-initialised data the emulation differs from the exact
    network by bfloat16 rounding: more than zero, a few 2^-8 at most."""
    params = _small_net(3, (40, 32, 32, 24))
    params = [p + (0.05 * np.random.default_rng(7).standard_normal(p.shape) if p.ndim == 1 else 0)
              for p in params]
    r = np.random.default_rng(8)
    X = to_bf16_(r.standard_normal((16, 40)))
    T = r.standard_normal((16, 24))
    y = mlp.forward(params, X, linear)[2]
    yq = mlp.forward_bf16(params, X, linear)[2]
    d = np.linalg.norm(yq - y) / np.linalg.norm(y)
    assert 0 < d < 3 * 2 ** -8
    _, g = mlp.backward(params, X, T, None, linear)
    _, gq = mlp.backward_bf16(params, X, T, None, linear)
    for s in (0, 2, 4):
        d = np.linalg.norm(gq[s] - g[s]) / np.linalg.norm(g[s])
        assert 0 < d < 4 * 2 ** -8, (s, d)


def to_bf16_(a):
    from oracle.quant import to_bf16
    return to_bf16(a)


def test_apply_bf16_within_rounding_of_apply():
    n, lx = 2, 3
    P = BoxProblem(n, lx, 0.1)
    params = synth.mlp_init(4, (lx ** 3 + 6, 16, 16, lx ** 3))
    r = scatter(synth.unique_normal(P.nu, 5), P.ids)
    z = mlp.apply(params, r, P.G, None, P.ids, P.nu)
    zq = mlp.apply_bf16(params, r, P.G, None, P.ids, P.nu)
    d = np.linalg.norm(zq - z) / np.linalg.norm(z)
    assert 0 < d < 3 * 2 ** -8
    zg = np.zeros(P.nu)
    zg[P.ids.ravel()] = zq.ravel()
    np.testing.assert_array_equal(zq, zg[P.ids])          # continuous


@pytest.mark.parametrize("normalise", [False, True])
def test_apply_block_bf16_identity_closed_form(normalise):
    """Identity block (a bfloat16 number) on the uniform box (one kappa): every
    node gets sqrt(mult) q_u / kappa where q = S r.  With r = sqrt(mult) q for
    bfloat16 numbers q the unnormalised path rounds nothing; the normalised
    path rounds q / s_e, within 2^-9 relative."""
    from oracle.gs import multiplicity
    n, lx = 2, 4
    P = BoxProblem(n, lx, 0.0)
    q = to_bf16_(synth.unique_normal(P.nu, 6))
    mult = multiplicity(P.ids, P.nu)
    r = scatter(q, P.ids) * np.sqrt(mult)          # not continuous: only the apply's arithmetic is pinned
    _, _, kappa = mlp.features(r, P.G)
    z = mlp.apply_block_bf16(np.eye(lx ** 3), r, P.G, None, P.ids, P.nu, normalise=normalise)
    want = np.sqrt(mult) * scatter(q, P.ids) / kappa[0]
    if normalise:
        np.testing.assert_allclose(z, want, rtol=2 ** -8, atol=0)
    else:
        np.testing.assert_allclose(z, want, rtol=1e-14, atol=0)
    # and against the exact block apply on a continuous residual
    rc = scatter(synth.unique_normal(P.nu, 7), P.ids)
    W = synth.rng(8).standard_normal((lx ** 3, lx ** 3))
    z0 = mlp.apply_block(W, rc, P.G, None, P.ids, P.nu)
    zq = mlp.apply_block_bf16(W, rc, P.G, None, P.ids, P.nu, normalise=normalise)
    d = np.linalg.norm(zq - z0) / np.linalg.norm(z0)
    assert 0 < d < 3 * 2 ** -8


def test_bf16_forward_rounds_hidden_activations():
    """One path 1 -> 1 -> 1 -> 1 of bfloat16 numbers whose products need 10
    significant bits: (1 + 2^-3)(1 + 2^-6) = 1 + 2^-3 + 2^-6 + 2^-9 rounds to
    1 + 2^-3 + 2^-6 in bfloat16 (8 significant bits); the second layer's
    product (1 + 2^-3 + 2^-6)(1 + 2^-4) is rounded again.  A dropped rounding
    of either hidden layer changes the output."""
    from oracle.quant import to_bf16
    one = np.ones(1)
    X = np.array([[1 + 2 ** -3]])
    params = [np.array([[1 + 2 ** -6]]), 0 * one, np.array([[1 + 2 ** -4]]), 0 * one, np.array([[1.0]]), 0 * one]
    y1 = to_bf16(np.array([(1 + 2 ** -3) * (1 + 2 ** -6)]))
    assert y1[0] == 1 + 2 ** -3 + 2 ** -6
    y2 = to_bf16(y1 * (1 + 2 ** -4))
    assert y2[0] != y1[0] * (1 + 2 ** -4)
    for linear in (False, True):
        assert mlp.forward_bf16(params, X, linear)[2][0, 0] == y2[0]
        assert mlp.forward(params, X, linear)[2][0, 0] != y2[0]


def test_apply_block_bf16_float32_decisions():
    """f32_decisions takes the bfloat16 roundings from float32 values.  Where
    those values are float32 numbers already (a symmetric block of bfloat16
    numbers; a residual of bfloat16 numbers on the nodes of multiplicity 1,
    where S = 1, and 0 elsewhere) it equals the float64-decision form bit for
    bit; on a general residual it stays within bfloat16 rounding of the exact
    block apply.  A dropped S, a missing symmetrisation or a transposed block
    fails one of the two."""
    from oracle.gs import multiplicity
    n, lx = 2, 4
    P = BoxProblem(n, lx, 0.1)
    nloc = lx ** 3
    A = to_bf16_(synth.rng(9).standard_normal((nloc, nloc)))
    Wsym = A + A.T                                  # bfloat16 numbers: halving and rounding are exact
    mult = multiplicity(P.ids, P.nu)
    r = to_bf16_(scatter(synth.unique_normal(P.nu, 10), P.ids)) * (mult == 1)
    z64 = mlp.apply_block_bf16(Wsym, r, P.G, None, P.ids, P.nu, normalise=False)
    z32 = mlp.apply_block_bf16(Wsym, r, P.G, None, P.ids, P.nu, normalise=False, f32_decisions=True)
    np.testing.assert_array_equal(z32, z64)
    W = synth.rng(11).standard_normal((nloc, nloc))
    rc = scatter(synth.unique_normal(P.nu, 12), P.ids)
    z0 = mlp.apply_block(W, rc, P.G, None, P.ids, P.nu)
    zq = mlp.apply_block_bf16(W, rc, P.G, None, P.ids, P.nu, normalise=False, f32_decisions=True)
    d = np.linalg.norm(zq - z0) / np.linalg.norm(z0)
    assert 0 < d < 3 * 2 ** -8
    zt = mlp.apply_block(W.T @ np.diag(np.arange(1.0, nloc + 1)), rc, P.G, None, P.ids, P.nu)
    assert np.linalg.norm(zq - zt) / np.linalg.norm(zt) > 0.1
