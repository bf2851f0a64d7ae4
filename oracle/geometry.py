"""Isoparametric geometry: Jacobian, geometric factors G_ab and mass weights.

The operator of Listing 2 multiplies the reference-space gradient by six
per-node factors g11..g33 (and h1).  For it to be the weak form of Eq. 1,
    int h1 grad u . grad v dOmega
  = sum_nodes w_i w_j w_k |J| h1 (J^-T grad_r u) . (J^-T grad_r v),
each factor must be
    G_ab = w_i w_j w_k |J| sum_c (dr_a/dx_c)(dr_b/dx_c),
with the GLL weights and the Jacobian determinant folded in (the usual
spectral-element convention; the paper does not spell it out).  The Jacobian
dx_c/dr_a is formed isoparametrically: the derivative matrix applied along
direction a to the node coordinates of x_c.  Mass weights B = w_i w_j w_k |J|.

Pins: axis-aligned cubes give G_rr = G_ss = G_tt = (h/2) w_i w_j w_k and zero
off-diagonal factors; the mass weights of a deformed periodic box sum to its
volume 1 to spectral accuracy (tests/test_oracle_geometry.py); the energy
identity for polynomials on affine elements (tests/test_oracle_ax.py).
"""
import numpy as np

from .gll import gll_nodes_weights, deriv_matrix


def ref_gradient(Dh, f):
    """(df/dr, df/ds, df/dt) at the nodes of each element; f is (E, lx, lx, lx)
    indexed [e][k][j][i]; r runs along i, s along j, t along k."""
    fr = np.einsum("il,ekjl->ekji", Dh, f)
    fs = np.einsum("jl,ekli->ekji", Dh, f)
    ft = np.einsum("kl,elji->ekji", Dh, f)
    return fr, fs, ft


def geometric_factors(x, y, z, lx):
    """Returns (G, B, detJ): G = (g11, g22, g33, g12, g13, g23), each
    (E, lx, lx, lx) float64, with 1 = r, 2 = s, 3 = t; B the mass weights."""
    xi, w = gll_nodes_weights(lx - 1)
    Dh = deriv_matrix(xi)
    E = x.shape[0]
    J = np.empty((E, lx, lx, lx, 3, 3))      # J[..., c, a] = dx_c / dr_a
    for c, f in enumerate((x, y, z)):
        for a, d in enumerate(ref_gradient(Dh, f)):
            J[..., c, a] = d
    detJ = np.linalg.det(J)
    Jinv = np.linalg.inv(J)                  # Jinv[..., a, c] = dr_a / dx_c
    wq = w[:, None, None] * w[None, :, None] * w[None, None, :]   # [k][j][i]
    B = wq[None] * detJ
    Gm = np.einsum("...ac,...bc->...ab", Jinv, Jinv) * B[..., None, None]
    G = (Gm[..., 0, 0], Gm[..., 1, 1], Gm[..., 2, 2],
         Gm[..., 0, 1], Gm[..., 0, 2], Gm[..., 1, 2])
    return tuple(np.ascontiguousarray(g) for g in G), B, detJ


def box_geometry(n, lx, a=0.0):
    """Geometric factors, mass weights and det J of the periodic n^3 box with
    deformation amplitude a (see oracle.mesh)."""
    from .mesh import box_coords
    x, y, z = box_coords(n, lx, a)
    return geometric_factors(x, y, z, lx)
