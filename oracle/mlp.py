"""Per-element learned preconditioner: features, MLP, loss, Adam, apply.

Not in the paper (it stops at the operator); this is the learned component
the library adds around the paper's Poisson solve.  Readings taken:
  * inputs (518 per element): the element's residual r_e / s_e with
    s_e = ||r_e||_2 + eps, then six geometric features mean(h1 g_ab) / kappa_e,
    where kappa_e = mean(h1 (g11 + g22 + g33)) / 3 (the element's stiffness
    scale), in the order g11, g22, g33, g12, g13, g23;
  * target: t_e = e_e kappa_e / s_e (dimensionless), e_e the element's error;
  * network: Linear-ReLU-Linear-ReLU-Linear, 518 -> 256 -> 256 -> 512,
    weights (fan_out, fan_in);
  * loss: mean squared error over all outputs of the batch;
  * optimiser: Adam (Kingma and Ba 2015) with bias correction;
  * apply: z_e = (s_e / kappa_e) t_hat_e, then the partition-of-unity average
    z = Q Q^T (z_local / mult) to make z continuous.
Pins (tests/test_oracle_mlp.py): backpropagation against central finite
differences; Adam against its closed form for a constant gradient; the
features' scale invariance; apply returns a continuous field.
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


def forward(params, X):
    W1, b1, W2, b2, W3, b3 = params
    a1 = X @ W1.T + b1
    y1 = np.maximum(a1, 0.0)
    a2 = y1 @ W2.T + b2
    y2 = np.maximum(a2, 0.0)
    y3 = y2 @ W3.T + b3
    return y1, y2, y3


def loss(params, X, T):
    return float(np.mean((forward(params, X)[2] - T) ** 2))


def backward(params, X, T):
    """(loss, grads) of the mean squared error, grads in params' order."""
    W1, b1, W2, b2, W3, b3 = params
    y1, y2, y3 = forward(params, X)
    d3 = 2.0 * (y3 - T) / y3.size
    gW3 = d3.T @ y2
    gb3 = d3.sum(axis=0)
    d2 = (d3 @ W3) * (y2 > 0)
    gW2 = d2.T @ y1
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * (y1 > 0)
    gW1 = d1.T @ X
    gb1 = d1.sum(axis=0)
    return float(np.mean((y3 - T) ** 2)), [gW1, gb1, gW2, gb2, gW3, gb3]


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


def apply(params, r_local, G, h1, ids, n_unique):
    """Preconditioner z = Q Q^T (mult^-1 (s/kappa) NN(features(r))) on the
    local layout."""
    from .gs import gs, multiplicity
    X, s, kappa = features(r_local, G, h1)
    t = forward(params, X)[2]
    z = (t * (s / kappa)[:, None]).reshape(r_local.shape)
    mult = multiplicity(ids, n_unique)
    return gs(z / mult, ids, n_unique)
