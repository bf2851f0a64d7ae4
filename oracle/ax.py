"""The element-local Poisson/Helmholtz stiffness operator ("Ax").

Paper Sec. 4.2: per element and node, three derivative passes
    ur_kji = sum_l dx[l, i] u_kjl,  us_kji = sum_l dy[l, j] u_kli,
    ut_kji = sum_l dz[l, k] u_lji,
a pointwise multiply by h1 times the symmetric 3x3 matrix of geometric factors
    [vr, vs, vt] = h1 [[g11, g12, g13], [g12, g22, g23], [g13, g23, g33]] [ur, us, ut],
then three transposed passes
    w_kji = sum_l dxt[l, i] vr_kjl + dyt[l, j] vs_kli + dzt[l, k] vt_lji.
Arrays are [e][k][j][i] with i fastest; the six lx*lx matrices are passed in
the argument layout of the paper's kernel interface (Sec. 4.2; see
oracle.gll.listing_matrices for how they relate to Dhat).

Three independent statements of the same operator:
  ax_quadrature  node by node: gradient along the three grid lines through a
             node, flux h1 G grad, spread back with the transposed weights
             (small cases only; takes Dhat itself, not the argument matrices);
  ax_einsum  the three derivative passes, the multiply and the three
             transposed passes, one einsum per pass (any size that fits memory);
  element_matrix / ax_dense
             A_e = sum_{a,b} D_a^T diag(h1 G_ab) D_b with Kronecker factors
             D_r = I (x) I (x) Dhat, D_s = I (x) Dhat (x) I, D_t = Dhat (x) I (x) I,
             with no sum factorisation at all.
Pins: ax_quadrature = ax_einsum = ax_dense on random inputs; symmetry; A 1 = 0;
u^T A u >= 0; exact energy for polynomials of total degree <= N on affine
elements; lx = 2 reduces to h times the 7-point Laplacian; Kronecker closed
form on uniform boxes; swapping dx and dxt is detected
(tests/test_oracle_ax.py, tests/test_oracle_assemble.py).

ax_helmholtz adds the diagonal mass term of the Helmholtz form (the paper's
kernel is named ax_helm but carries only the h1 stiffness):
w = A_e u + h2b u with h2b = h2 w_i w_j w_k |J| per node.  Pins: on affine
elements u^T w = int |grad u|^2 + h2 int u^2 exactly for total degree <= N - 1,
not beyond; the assembled A + h2 B is positive definite where A is singular.
"""
import numpy as np


def ax_quadrature(u, Dh, h1, g11, g22, g33, g12, g13, g23):
    """w_e = sum_{a,b} D_a^T diag(h1 G_ab) D_b u_e (Sec. 4.2), point by point.

    Pure Python: keep E * lx^4 small.  For every quadrature node m of an
    element the reference gradient grad_b(m) = (D_b u)(m) is the derivative
    matrix Dh (Dh[a, b] = l_b'(xi_a)) applied along the grid line through m
    in direction b; the flux is q_a(m) = h1(m) sum_b G_ab(m) grad_b(m); and
    D_a^T q_a adds Dh[m_a, n_a] q_a(m) to every node n on the line through m
    in direction a.  No temporaries beyond one node's gradient and flux."""
    nel, lx = u.shape[0], u.shape[1]
    w = np.zeros_like(u)
    G = np.empty((3, 3))
    for e in range(nel):
        ue, we = u[e], w[e]
        for m in np.ndindex(lx, lx, lx):          # m = (k, j, i)
            k, j, i = m
            grad = np.zeros(3)
            for n in range(lx):
                grad[0] += Dh[i, n] * ue[k, j, n]   # along r (i)
                grad[1] += Dh[j, n] * ue[k, n, i]   # along s (j)
                grad[2] += Dh[k, n] * ue[n, j, i]   # along t (k)
            G[0, 0], G[1, 1], G[2, 2] = g11[e][m], g22[e][m], g33[e][m]
            G[0, 1] = G[1, 0] = g12[e][m]
            G[0, 2] = G[2, 0] = g13[e][m]
            G[1, 2] = G[2, 1] = g23[e][m]
            flux = (1.0 if h1 is None else h1[e][m]) * (G @ grad)
            for n in range(lx):
                we[k, j, n] += Dh[i, n] * flux[0]
                we[k, n, i] += Dh[j, n] * flux[1]
                we[n, j, i] += Dh[k, n] * flux[2]
    return w


def ax_einsum(u, dx, dy, dz, dxt, dyt, dzt, h1, g11, g22, g33, g12, g13, g23):
    """The operator's sums, one einsum per contraction, with the argument
    matrices dx[l, i] = l_l'(xi_i) and dxt = dx^T (reading R2)."""
    ur = np.einsum("li,ekjl->ekji", dx, u)
    us = np.einsum("lj,ekli->ekji", dy, u)
    ut = np.einsum("lk,elji->ekji", dz, u)
    if h1 is None:
        h1 = 1.0
    vr = h1 * (g11 * ur + g12 * us + g13 * ut)
    vs = h1 * (g12 * ur + g22 * us + g23 * ut)
    vt = h1 * (g13 * ur + g23 * us + g33 * ut)
    return (np.einsum("li,ekjl->ekji", dxt, vr)
            + np.einsum("lj,ekli->ekji", dyt, vs)
            + np.einsum("lk,elji->ekji", dzt, vt))


def kron_derivs(Dh):
    """D_r, D_s, D_t acting on vec(u_e) with i fastest (index (k*lx + j)*lx + i)."""
    lx = Dh.shape[0]
    I = np.eye(lx)
    Dr = np.kron(I, np.kron(I, Dh))
    Ds = np.kron(I, np.kron(Dh, I))
    Dt = np.kron(Dh, np.kron(I, I))
    return Dr, Ds, Dt


def element_matrix(Dh, h1e, ge):
    """Dense A_e = sum_{a,b} D_a^T diag(h1 G_ab) D_b for one element.

    ge = (g11, g22, g33, g12, g13, g23) of that element, each (lx, lx, lx)."""
    Dr, Ds, Dt = kron_derivs(Dh)
    Ds_ = (Dr, Ds, Dt)
    g11, g22, g33, g12, g13, g23 = (np.ravel(g) for g in ge)
    h = np.ravel(h1e) if h1e is not None else np.ones_like(g11)
    Gab = {(0, 0): g11, (1, 1): g22, (2, 2): g33,
           (0, 1): g12, (1, 0): g12, (0, 2): g13, (2, 0): g13,
           (1, 2): g23, (2, 1): g23}
    n = Dr.shape[0]
    A = np.zeros((n, n))
    for a in range(3):
        for b in range(3):
            A += Ds_[a].T @ ((h * Gab[a, b])[:, None] * Ds_[b])
    return A


def ax_dense(u, Dh, h1, G):
    """w_e = A_e u_e with the dense element matrices; G = (g11, ..., g23)."""
    nel, lx = u.shape[0], u.shape[1]
    w = np.empty_like(u)
    for e in range(nel):
        Ae = element_matrix(Dh, None if h1 is None else h1[e], tuple(g[e] for g in G))
        w[e] = (Ae @ u[e].ravel()).reshape(lx, lx, lx)
    return w


def ax_helmholtz(u, dx, dy, dz, dxt, dyt, dzt, h1, g11, g22, g33, g12, g13, g23, h2b):
    """Helmholtz form: the stiffness of ax_einsum plus the diagonal mass term
    h2b * u, with h2b = h2 B per local node (B = w_i w_j w_k |J|)."""
    return ax_einsum(u, dx, dy, dz, dxt, dyt, dzt, h1, g11, g22, g33, g12, g13, g23) + h2b * u
