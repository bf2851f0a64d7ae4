"""The element-local Poisson/Helmholtz stiffness operator ("Ax").

Paper Sec. 4.2, Listing 2: per element and node, three derivative passes
    ur_kji = sum_l dx[l, i] u_kjl,  us_kji = sum_l dy[l, j] u_kli,
    ut_kji = sum_l dz[l, k] u_lji,
a pointwise multiply by h1 times the symmetric 3x3 matrix of geometric factors
    [vr, vs, vt] = h1 [[g11, g12, g13], [g12, g22, g23], [g13, g23, g33]] [ur, us, ut],
then three transposed passes
    w_kji = sum_l dxt[l, i] vr_kjl + dyt[l, j] vs_kli + dzt[l, k] vt_lji.
Arrays are [e][k][j][i] with i fastest; the six lx*lx matrices are passed as
in Listing 1 (see oracle.gll.listing_matrices for how they relate to Dhat).

Three independent statements of the same operator:
  ax_loops   the loop nest in the order Listing 2 prints it (small cases only);
  ax_einsum  the same sums, one einsum per pass (any size that fits memory);
  element_matrix / ax_dense
             A_e = sum_{a,b} D_a^T diag(h1 G_ab) D_b with Kronecker factors
             D_r = I (x) I (x) Dhat, D_s = I (x) Dhat (x) I, D_t = Dhat (x) I (x) I,
             with no sum factorisation at all.
Pins: ax_loops = ax_einsum = ax_dense on random inputs; symmetry; A 1 = 0;
u^T A u >= 0; exact energy for polynomials of total degree <= N on affine
elements; lx = 2 reduces to h times the 7-point Laplacian; Kronecker closed
form on uniform boxes; swapping dx and dxt is detected
(tests/test_oracle_ax.py, tests/test_oracle_assemble.py).

ax_helmholtz adds the diagonal mass term of the Helmholtz form (the routine of
Listing 1 is named ax_helm; Listing 2 carries only the h1 stiffness):
w = A_e u + h2b u with h2b = h2 w_i w_j w_k |J| per node.  Pins: on affine
elements u^T w = int |grad u|^2 + h2 int u^2 exactly for total degree <= N - 1,
not beyond; the assembled A + h2 B is positive definite where A is singular.
"""
import numpy as np


def ax_loops(u, dx, dy, dz, dxt, dyt, dzt, h1, g11, g22, g33, g12, g13, g23):
    """Listing 2, loop for loop.  Pure Python: keep E * lx^4 small."""
    nel, lx = u.shape[0], u.shape[1]
    w = np.zeros_like(u)
    ur = np.zeros_like(u)
    us = np.zeros_like(u)
    ut = np.zeros_like(u)
    vr = np.zeros_like(u)
    vs = np.zeros_like(u)
    vt = np.zeros_like(u)
    for e in range(nel):
        for k in range(lx):
            for j in range(lx):
                for i in range(lx):
                    r = s = t = 0.0
                    for l in range(lx):
                        r += dx[l, i] * u[e, k, j, l]
                        s += dy[l, j] * u[e, k, l, i]
                        t += dz[l, k] * u[e, l, j, i]
                    ur[e, k, j, i], us[e, k, j, i], ut[e, k, j, i] = r, s, t
                    H = h1[e, k, j, i]
                    G00, G01, G02 = g11[e, k, j, i], g12[e, k, j, i], g13[e, k, j, i]
                    G11, G12, G22 = g22[e, k, j, i], g23[e, k, j, i], g33[e, k, j, i]
                    vr[e, k, j, i] = H * (G00 * r + G01 * s + G02 * t)
                    vs[e, k, j, i] = H * (G01 * r + G11 * s + G12 * t)
                    vt[e, k, j, i] = H * (G02 * r + G12 * s + G22 * t)
        for k in range(lx):
            for j in range(lx):
                for i in range(lx):
                    acc = 0.0
                    for l in range(lx):
                        acc += dxt[l, i] * vr[e, k, j, l]
                        acc += dyt[l, j] * vs[e, k, l, i]
                        acc += dzt[l, k] * vt[e, l, j, i]
                    w[e, k, j, i] = acc
    return w


def ax_einsum(u, dx, dy, dz, dxt, dyt, dzt, h1, g11, g22, g33, g12, g13, g23):
    """Listing 2's sums, one einsum per contraction."""
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
