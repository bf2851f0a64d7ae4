"""Assembled operator and its diagonal.

The assembled Poisson matrix is A_G = sum_e Q_e^T A_e Q_e, with A_e the dense
element matrix of oracle.ax.element_matrix and Q_e the element's scatter.  The
paper's solver applies it matrix-free (Ax followed by gather-scatter,
Sec. 2.1 and Sec. 3); here it is built explicitly, as a scipy sparse matrix, so
the matrix-free path can be compared against it.

The Jacobi diagonal diag(A_G) = Q^T diag_e, where per node (i, j, k) of an
element, with V_ab = h1 G_ab,
  diag_e = sum_l Dhat_li^2 V_rr(l,j,k) + sum_l Dhat_lj^2 V_ss(i,l,k)
         + sum_l Dhat_lk^2 V_tt(i,j,l)
         + 2 Dhat_ii Dhat_jj V_rs + 2 Dhat_ii Dhat_kk V_rt + 2 Dhat_jj Dhat_kk V_st
(the diagonal of sum_ab D_a^T diag(V_ab) D_b).
Pins: the formula equals the diagonal of the dense A_e
(tests/test_oracle_assemble.py).
"""
import numpy as np
import scipy.sparse as sp

from .ax import element_matrix


def assembled_matrix(Dh, h1, G, ids, n_unique):
    """Sparse CSR A_G (n_unique x n_unique); rows and columns of Dirichlet
    nodes (negative ids) are left out."""
    nel = ids.shape[0]
    rows, cols, vals = [], [], []
    for e in range(nel):
        Ae = element_matrix(Dh, None if h1 is None else h1[e], tuple(g[e] for g in G))
        q = ids[e].ravel()
        f = np.flatnonzero(q >= 0)
        rows.append(np.repeat(q[f], len(f)))
        cols.append(np.tile(q[f], len(f)))
        vals.append(Ae[np.ix_(f, f)].ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n_unique, n_unique))
    return A.tocsr()


def element_diagonal(Dh, h1, G):
    """diag_e of every element by the closed formula above, (E, lx, lx, lx)."""
    g11, g22, g33, g12, g13, g23 = G
    h = 1.0 if h1 is None else h1
    D2 = Dh * Dh
    dd = np.diag(Dh)
    d = (np.einsum("li,ekjl->ekji", D2, h * g11)
         + np.einsum("lj,ekli->ekji", D2, h * g22)
         + np.einsum("lk,elji->ekji", D2, h * g33))
    d = d + 2.0 * h * (g12 * dd[None, None, :, None] * dd[None, None, None, :]
                       + g13 * dd[None, :, None, None] * dd[None, None, None, :]
                       + g23 * dd[None, :, None, None] * dd[None, None, :, None])
    return d


def element_diagonal_dense(Dh, h1, G):
    """diag_e taken from the dense element matrices (the pin for the formula)."""
    nel, lx = G[0].shape[0], G[0].shape[1]
    out = np.empty((nel, lx, lx, lx))
    for e in range(nel):
        Ae = element_matrix(Dh, None if h1 is None else h1[e], tuple(g[e] for g in G))
        out[e] = np.diag(Ae).reshape(lx, lx, lx)
    return out
