"""Per-element learned preconditioner: features, MLP, loss, Adam, apply.

Not in the paper (it stops at the operator); this is the learned component
the library adds around the paper's Poisson solve.  Readings taken:
  * inputs (518 per element): the element's residual r_e / s_e with
    s_e = ||r_e||_2 + eps, then six geometric features mean(h1 g_ab) / kappa_e,
    where kappa_e = mean(h1 (g11 + g22 + g33)) / 3 (the element's stiffness
    scale), in the order g11, g22, g33, g12, g13, g23;
  * target: t_e = e_e kappa_e / s_e (dimensionless), e_e the element's error;
  * network: Linear-ReLU-Linear-ReLU-Linear, 518 -> 256 -> 256 -> 512,
    weights (fan_out, fan_in); or its linear form (identity activations, no
    biases, geometric inputs zeroed), which makes the preconditioner a fixed
    linear map of r -- the element-local linear predictor of the error from
    the residual, whose white-noise optimum is the element block of A^+;
  * loss: mean squared error over all outputs of the batch, or, with a metric
    K, the batch mean of (y - t)^T K (y - t).  The preconditioner is judged
    in the energy norm (the norm CG minimises), so the metric used is
    K = A_ref + mu B_ref: the stiffness of the undeformed reference element
    (geometric factors w_i w_j w_k on the diagonal, scaled so that its kappa
    is 1) plus mu times its mass matrix scaled to unit mean diagonal, which
    pins the element-wise constant the stiffness alone leaves free;
  * optimiser: Adam (Kingma and Ba 2015) with bias correction;
  * apply: z_e = (s_e / kappa_e) t_hat_e, then the partition-of-unity average
    z = Q Q^T (z_local / mult) to make z continuous; the linear form instead
    applies the symmetric part of its folded matrix with square-root
    multiplicity weights on both sides (``apply_linear``), a symmetric
    additive (one-level Schwarz-type) preconditioner.
Pins (tests/test_oracle_mlp.py): backpropagation against central finite
differences (both losses); Adam against its closed form for a constant
gradient; the features' scale invariance; features and kappa against the
closed form of axis-aligned rectangular and sheared affine elements (kappa =
(8 / lx^3)(bc/a + ac/b + ab/c) / 6 for an a x b x c brick, 4 h / lx^3 on the
uniform box, features (1, 1, 1, 0, 0, 0) there); targets against that
closed-form kappa; the nonlinear apply of a constant-output network: a
constant residual c on the uniform box gives |c| sqrt(lx^3) lx^3 n / 4 at
every node, and a general residual gives the copy-by-copy average of
(s_e / kappa_e) NN_p over the element copies of each node;
the reference metric is symmetric positive definite and its stiffness part
gives the exact energy of polynomials of degree <= N on the reference cube;
the linear apply with an identity block returns r / kappa (partition of
unity), is exactly symmetric for any weights, and is positive definite when
the folded matrix's symmetric part is.
"""
import numpy as np

EPS = 1e-30


def features(r_e, G_e, h1_e=None):
    """r_e (E, lx, lx, lx); G_e tuple of six (E, lx, lx, lx); returns
    (X (E, 518), s (E,), kappa (E,))."""
    E = r_e.shape[0]
    r = r_e.reshape(E, -1)
    s = np.sqrt(np.sum(r * r, axis=1)) + EPS
    h = 1.0 if h1_e is None else h1_e.reshape(E, -1)
    Gf = [g.reshape(E, -1) for g in G_e]
    kappa = np.mean(h * (Gf[0] + Gf[1] + Gf[2]), axis=1) / 3.0
    geo = np.stack([np.mean(h * g, axis=1) / kappa for g in Gf], axis=1)
    return np.concatenate([r / s[:, None], geo], axis=1), s, kappa


def targets(err_e, s, kappa):
    E = err_e.shape[0]
    return err_e.reshape(E, -1) * (kappa / s)[:, None]


def forward(params, X, linear=False):
    """Linear=True: identity activations and no biases (y3 = W3 W2 W1 x)."""
    W1, b1, W2, b2, W3, b3 = params
    if linear:
        y1 = X @ W1.T
        y2 = y1 @ W2.T
        return y1, y2, y2 @ W3.T
    a1 = X @ W1.T + b1
    y1 = np.maximum(a1, 0.0)
    a2 = y1 @ W2.T + b2
    y2 = np.maximum(a2, 0.0)
    y3 = y2 @ W3.T + b3
    return y1, y2, y3


def reference_metric(lx=8, mu=1.0):
    """K = A_ref + mu B_ref (see module docstring), (lx^3, lx^3)."""
    from .gll import gll_nodes_weights, deriv_matrix
    from .ax import element_matrix
    xi, w = gll_nodes_weights(lx - 1)
    Dh = deriv_matrix(xi)
    wq = (w[:, None, None] * w[None, :, None] * w[None, None, :])[None]
    zero = np.zeros_like(wq)
    A = element_matrix(Dh, None, (wq, wq, wq, zero[0:1], zero[0:1], zero[0:1]))
    kappa = np.mean(wq)            # mean of (g11 + g22 + g33) / 3
    Bm = np.diag(wq.ravel() / np.mean(wq))
    return A / kappa + mu * Bm


def loss(params, X, T, K=None, linear=False):
    d = forward(params, X, linear)[2] - T
    if K is None:
        return float(np.mean(d ** 2))
    return float(np.mean(np.einsum("bi,ij,bj->b", d, K, d)))


def backward(params, X, T, K=None, linear=False):
    """(loss, grads) of the loss above, grads in params' order (bias gradients
    are zero in the linear form, whose biases are not used)."""
    W1, b1, W2, b2, W3, b3 = params
    y1, y2, y3 = forward(params, X, linear)
    if K is None:
        d3 = 2.0 * (y3 - T) / y3.size
        lval = float(np.mean((y3 - T) ** 2))
    else:
        d = y3 - T
        Kd = d @ K
        d3 = 2.0 * Kd / d.shape[0]
        lval = float(np.mean(np.sum(d * Kd, axis=1)))
    gW3 = d3.T @ y2
    gb3 = d3.sum(axis=0)
    d2 = d3 @ W3 if linear else (d3 @ W3) * (y2 > 0)
    gW2 = d2.T @ y1
    gb2 = d2.sum(axis=0)
    d1 = d2 @ W2 if linear else (d2 @ W2) * (y1 > 0)
    gW1 = d1.T @ X
    gb1 = d1.sum(axis=0)
    if linear:
        gb1, gb2, gb3 = 0 * gb1, 0 * gb2, 0 * gb3
    return lval, [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_step(params, grads, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new (params, m, v)."""
    out_p, out_m, out_v = [], [], []
    for p, g, mi, vi in zip(params, grads, m, v):
        mi = beta1 * mi + (1 - beta1) * g
        vi = beta2 * vi + (1 - beta2) * g * g
        mh = mi / (1 - beta1 ** t)
        vh = vi / (1 - beta2 ** t)
        out_p.append(p - lr * mh / (np.sqrt(vh) + eps))
        out_m.append(mi)
        out_v.append(vi)
    return out_p, out_m, out_v


def apply(params, r_local, G, h1, ids, n_unique, linear=False):
    """Preconditioner on the local layout.  Nonlinear form:
    z = Q Q^T (mult^-1 (s/kappa) NN(features(r))).  Linear form: see
    ``apply_linear``."""
    from .gs import gs, multiplicity
    if linear:
        return apply_linear(params, r_local, G, h1, ids, n_unique)
    X, s, kappa = features(r_local, G, h1)
    t = forward(params, X, linear)[2]
    z = (t * (s / kappa)[:, None]).reshape(r_local.shape)
    mult = multiplicity(ids, n_unique)
    return gs(z / mult, ids, n_unique)


def folded_matrix(params, nloc):
    """The linear form's map of the element residual: (W3 W2 W1)[:, :nloc]."""
    W1, _, W2, _, W3, _ = params
    return W3 @ (W2 @ W1[:, :nloc])


def apply_linear(params, r_local, G, h1, ids, n_unique):
    """Linear form as a symmetric additive preconditioner:
    z = sum_e Q_e S_e W_s S_e Q_e^T r / kappa_e, with W_s the symmetric part
    of the folded matrix and S_e = diag(mult^-1/2) on the element's nodes.
    Since sum over the copies of a node of S^2 = 1, an identity W_s gives
    z = r / kappa on a box of constant kappa; W_s symmetric (positive
    definite) makes the preconditioner symmetric (positive definite), so CG's
    conjugacy holds.  The network is trained on unweighted element pairs
    (r_e, e_e); the white-noise optimum of that regression is the element
    block of A^+, applied here with the square-root weights."""
    return apply_block(folded_matrix(params, r_local[0].size), r_local, G, h1, ids, n_unique)


def apply_block(W, r_local, G, h1, ids, n_unique):
    """The symmetric additive apply of a given element block W (nloc x nloc):
    z = sum_e Q_e S_e W_s S_e Q_e^T r / kappa_e, W_s = (W + W^T) / 2."""
    from .gs import gs, multiplicity
    E = r_local.shape[0]
    nloc = r_local[0].size
    Ws = 0.5 * (W + W.T)
    _, _, kappa = features(r_local, G, h1)
    S = 1.0 / np.sqrt(multiplicity(ids, n_unique).reshape(E, nloc))
    z = ((S * r_local.reshape(E, nloc)) @ Ws.T) * S / kappa[:, None]
    return gs(z.reshape(r_local.shape), ids, n_unique)


# ---------------------------------------------------------------------------
# bfloat16-storage emulation: the same network with its operands rounded as
# the product kernels store them (weights, inputs, hidden activations and the
# back-propagated errors in bfloat16; biases, outputs and gradients in
# float32), every product summed exactly in float64.  The kernels accumulate
# in float32, so they differ from these only by accumulation rounding and by
# the bfloat16 roundings that such rounding can tip (a value within a few
# float32 ulps of a bfloat16 rounding boundary).  Pins: equal to the exact
# functions above when every operand and intermediate is a bfloat16 number;
# within bfloat16 rounding of them otherwise (tests/test_oracle_mlp.py).

def forward_bf16(params, Xq, linear=False):
    """Forward pass of bfloat16 inputs Xq (already rounded) with bfloat16
    weights and bfloat16 hidden activations; returns (y1, y2, y3)."""
    from .quant import to_bf16, to_f32
    W1, b1, W2, b2, W3, b3 = params
    Wq = [to_bf16(W) for W in (W1, W2, W3)]
    if linear:
        y1 = to_bf16(Xq @ Wq[0].T)
        y2 = to_bf16(y1 @ Wq[1].T)
        return y1, y2, to_f32(y2 @ Wq[2].T)
    y1 = to_bf16(np.maximum(Xq @ Wq[0].T + to_f32(b1), 0.0))
    y2 = to_bf16(np.maximum(y1 @ Wq[1].T + to_f32(b2), 0.0))
    return y1, y2, to_f32(y2 @ Wq[2].T + to_f32(b3))


def backward_bf16(params, Xq, T, K=None, linear=False):
    """(loss, grads) with the roundings of the training kernels: the loss
    gradient d3 in float32 and bfloat16 (with the metric, d = y3 - T and K
    rounded to bfloat16 before K d), back-propagated errors rounded to
    bfloat16 after the ReLU mask, weight gradients from bfloat16 factors,
    bias gradients from the float32 errors."""
    from .quant import to_bf16, to_f32
    W1, b1, W2, b2, W3, b3 = params
    Wq = [to_bf16(W) for W in (W1, W2, W3)]
    y1, y2, y3 = forward_bf16(params, Xq, linear)
    B = y3.shape[0]
    if K is None:
        d = to_f32(y3 - T)
        lval = float(np.mean(d * d))
        d3f = to_f32(d * (2.0 / y3.size))
    else:
        d = to_f32(y3 - T)
        Kd = to_f32(to_bf16(d) @ to_bf16(K).T)
        lval = float(np.mean(np.sum(d * Kd, axis=1)))
        d3f = to_f32(Kd * (2.0 / B))
    d3b = to_bf16(d3f)
    gW3 = to_f32(d3b.T @ y2)
    d2f = to_f32(d3b @ Wq[2]) * (1.0 if linear else (y2 > 0))
    d2b = to_bf16(d2f)
    gW2 = to_f32(d2b.T @ y1)
    d1f = to_f32(d2b @ Wq[1]) * (1.0 if linear else (y1 > 0))
    d1b = to_bf16(d1f)
    gW1 = to_f32(d1b.T @ Xq)
    if linear:
        gb = [np.zeros(W1.shape[0]), np.zeros(W2.shape[0]), np.zeros(W3.shape[0])]
    else:
        gb = [d1f.sum(axis=0), d2f.sum(axis=0), d3f.sum(axis=0)]
    return lval, [gW1, gb[0], gW2, gb[1], gW3, gb[2]]


def apply_bf16(params, r_local, G, h1, ids, n_unique):
    """The nonlinear apply with bfloat16 inputs (features rounded float64 ->
    float32 -> bfloat16), the bfloat16 network above and the float32 scale
    s_e / kappa_e (kappa_e held in float32)."""
    from .gs import gs, multiplicity
    from .quant import to_bf16, to_f32
    X, s, kappa = features(r_local, G, h1)
    t = forward_bf16(params, to_bf16(X))[2]
    scale = to_f32(s / to_f32(kappa))
    z = (t * scale[:, None]).reshape(r_local.shape)
    return gs(z / multiplicity(ids, n_unique), ids, n_unique)


def apply_block_bf16(W, r_local, G, h1, ids, n_unique, normalise=True, f32_decisions=False):
    """The symmetric additive apply of a float32 element block W as the
    linear-form kernels evaluate it: W_s = bf16((W + W^T) / 2), the weighted
    element residual S r_e rounded to bfloat16 -- divided by its 2-norm s_e
    first (``normalise``, the local-layout path, output scaled back by s_e)
    or not (the unique-layout path) -- the product summed exactly, the output
    weighted by S / kappa_e and assembled.
    f32_decisions: the two roundings to bfloat16 are taken from the float32
    values the kernels round (both sides decide in the same precision): W_s
    from the float32 sum of the float32 block and its transpose, halved
    (exact), and S r from the float32 product of float32 S and float32 r (a
    product of two float32 numbers is exact in float64, so one rounding to
    float32 reproduces the float32 multiply).  Unnormalised path only."""
    from .gs import gs, multiplicity
    from .quant import to_bf16, to_f32
    E = r_local.shape[0]
    nloc = r_local[0].size
    S = 1.0 / np.sqrt(multiplicity(ids, n_unique).reshape(E, nloc))
    if f32_decisions:
        assert not normalise
        W32 = to_f32(W)
        Wq = to_bf16(0.5 * to_f32(W32 + W32.T))
        v = to_f32(to_f32(S) * to_f32(r_local.reshape(E, nloc)))
    else:
        Wq = to_bf16(0.5 * (W + W.T))
        v = S * r_local.reshape(E, nloc)
    _, _, kappa = features(r_local, G, h1)
    if normalise:
        s = np.sqrt(np.sum(v * v, axis=1)) + EPS
        z = (to_bf16(v / s[:, None]) @ Wq.T) * (s / kappa)[:, None] * S
    else:
        z = (to_bf16(v) @ Wq.T) * S / kappa[:, None]
    return gs(z.reshape(r_local.shape), ids, n_unique)
