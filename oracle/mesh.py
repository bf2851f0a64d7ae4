"""Periodic box meshes of lx^3 GLL hexahedra.

The paper measures on cubic meshes of N_E hexahedral elements (Sec. 4.4) and
expands the solution on each element as a tensor product over the GLL points
(Sec. 3, Eq. 3).  Readings taken where the paper is silent:
  * the box is the unit cube, n elements per side, periodic in x, y and z;
  * elements are numbered lexicographically, e = ex + n (ey + n ez), and the
    nodes of one element as [k][j][i] with i fastest (the index order of
    Listing 2);
  * the undeformed position of node (i, j, k) of element (ex, ey, ez) is
    X = (ex + (1 + xi_i) / 2) / n, likewise Y, Z;
  * the deformed position is x = X + a sin(2 pi Y) sin(2 pi Z), with y and z
    following cyclically, which keeps x(X + e_c) = x(X) + e_c, so periodic
    copies of a node still coincide;
  * the global id of a node is its position on the (nN)^3 periodic lattice,
    g = ((ez N + k) mod nN) (nN)^2 + ((ey N + j) mod nN) nN + ((ex N + i) mod nN);
  * the Dirichlet box is the same mesh without the periodic identification and
    with every node on the six faces of the undeformed cube held at zero
    (homogeneous Dirichlet); those nodes get id -1 and are no unknowns, and the
    interior nodes are numbered on the (nN - 1)^3 lattice of interior points,
    g = (K - 1) (nN - 1)^2 + (J - 1) (nN - 1) + (I - 1) with I = ex N + i etc.
Pins: multiplicity counts and unique-node counts (tests/test_oracle_gs.py),
affine volumes and geometric factors (tests/test_oracle_geometry.py).
"""
import numpy as np

from .gll import gll_nodes_weights


def _elements(n, elements):
    return np.arange(n ** 3) if elements is None else np.asarray(elements, dtype=np.int64)


def reference_coords(n, lx, elements=None):
    """Undeformed node positions X, Y, Z, each of shape (E, lx, lx, lx), for
    all n^3 elements or for the listed element numbers."""
    xi, _ = gll_nodes_weights(lx - 1)
    els = _elements(n, elements)
    X = np.empty((len(els), lx, lx, lx))
    Y = np.empty_like(X)
    Z = np.empty_like(X)
    for q, e in enumerate(els):
        ex, ey, ez = e % n, (e // n) % n, e // (n * n)
        px = (ex + 0.5 * (1.0 + xi)) / n
        py = (ey + 0.5 * (1.0 + xi)) / n
        pz = (ez + 0.5 * (1.0 + xi)) / n
        X[q] = px[None, None, :]
        Y[q] = py[None, :, None]
        Z[q] = pz[:, None, None]
    return X, Y, Z


def deform(X, Y, Z, a):
    """The cyclic sine deformation with amplitude a."""
    tp = 2.0 * np.pi
    x = X + a * np.sin(tp * Y) * np.sin(tp * Z)
    y = Y + a * np.sin(tp * Z) * np.sin(tp * X)
    z = Z + a * np.sin(tp * X) * np.sin(tp * Y)
    return x, y, z


def box_coords(n, lx, a=0.0, elements=None):
    return deform(*reference_coords(n, lx, elements), a)


def global_ids(n, lx, elements=None):
    """int64 global ids, shape (E, lx, lx, lx), values in [0, (n N)^3)."""
    N = lx - 1
    M = n * N
    els = _elements(n, elements)
    ids = np.empty((len(els), lx, lx, lx), dtype=np.int64)
    r = np.arange(lx)
    for q, e in enumerate(els):
        ex, ey, ez = e % n, (e // n) % n, e // (n * n)
        gi = (ex * N + r) % M
        gj = (ey * N + r) % M
        gk = (ez * N + r) % M
        ids[q] = gk[:, None, None] * M * M + gj[None, :, None] * M + gi[None, None, :]
    return ids


def n_unique(n, lx):
    return (n * (lx - 1)) ** 3


def global_ids_dirichlet(n, lx, elements=None):
    """int64 ids of the Dirichlet box, shape (E, lx, lx, lx): -1 on the box
    boundary, values in [0, (n N - 1)^3) inside."""
    N = lx - 1
    M = n * N
    els = _elements(n, elements)
    ids = np.empty((len(els), lx, lx, lx), dtype=np.int64)
    r = np.arange(lx)
    for q, e in enumerate(els):
        ex, ey, ez = e % n, (e // n) % n, e // (n * n)
        I, J, K = ex * N + r, ey * N + r, ez * N + r
        inside = ((K > 0) & (K < M))[:, None, None] & ((J > 0) & (J < M))[None, :, None] \
            & ((I > 0) & (I < M))[None, None, :]
        g = (K - 1)[:, None, None] * (M - 1) ** 2 + (J - 1)[None, :, None] * (M - 1) \
            + (I - 1)[None, None, :]
        ids[q] = np.where(inside, g, -1)
    return ids


def n_unique_dirichlet(n, lx):
    return max(n * (lx - 1) - 1, 0) ** 3
