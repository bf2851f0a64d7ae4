"""Shared test helpers: seeded inputs on both sides, error norms."""
import numpy as np


def rel_inf(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    s = np.max(np.abs(ref))
    return float(np.max(np.abs(got - ref)) / (s if s > 0 else 1.0))


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def linear_apply_at_nodes(params, n, lx, amp, ids, r_glob, gids, jacobi=False, bf16=False):
    """The oracle's linear-form apply (oracle.mlp.apply_linear, plus Minv r with
    the Jacobi base) evaluated only at the global ids `gids` of the n^3 box,
    each from the elements that contain it: for large meshes, where the
    whole-mesh oracle is too slow.  ids: the box's global ids (E, lx, lx, lx).
    With bf16, the unique-layout kernels' storage is emulated as in
    oracle.mlp.apply_block_bf16(normalise=False): the symmetric block and
    each element's S r rounded to bfloat16."""
    from oracle.quant import to_bf16
    from oracle import mlp
    from oracle.mesh import box_coords
    from oracle.geometry import geometric_factors
    from oracle.gll import gll_nodes_weights, deriv_matrix
    from oracle.assemble import element_diagonal
    flat = ids.reshape(len(ids), -1)
    counts = np.bincount(flat.ravel())
    W = mlp.folded_matrix(params, lx ** 3)
    Ws = 0.5 * (W + W.T)
    if bf16:
        Ws = to_bf16(Ws)
    xi, _ = gll_nodes_weights(lx - 1)
    Dh = deriv_matrix(xi)
    out = np.empty(len(gids))
    for q, g in enumerate(gids):
        els = np.nonzero((flat == g).any(axis=1))[0]
        x, y, z = box_coords(n, lx, amp, elements=els)
        G, _, _ = geometric_factors(x, y, z, lx)
        _, _, kappa = mlp.features(r_glob[ids[els]], G)
        diag = element_diagonal(Dh, None, G).reshape(len(els), -1)
        acc, dg = 0.0, 0.0
        for a, e in enumerate(els):
            S = 1.0 / np.sqrt(counts[flat[e]])
            xv = S * r_glob[flat[e]]
            yv = Ws @ (to_bf16(xv) if bf16 else xv)
            at = flat[e] == g
            acc += np.sum(S[at] * yv[at]) / kappa[a]
            dg += np.sum(diag[a][at])
        out[q] = acc + (r_glob[g] / dg if jacobi else 0.0)
    return out


def operator_at_nodes(n, lx, amp, ids, x_glob, gids, h1_glob=None, h2=None):
    """(A x)_g of the n^3 box's assembled operator at the global ids `gids`, each
    from the elements that contain it (oracle geometry and einsum operator):
    for large meshes, where the whole-mesh oracle is too slow.  Negative ids
    (Dirichlet nodes) read 0.  With h2, the Helmholtz operator A + h2 B."""
    from oracle.mesh import box_coords
    from oracle.geometry import geometric_factors
    from oracle.gll import listing_matrices
    from oracle.ax import ax_einsum
    from oracle.gs import scatter
    flat = ids.reshape(len(ids), -1)
    M = listing_matrices(lx)
    out = np.empty(len(gids))
    for q, g in enumerate(gids):
        els = np.nonzero((flat == g).any(axis=1))[0]
        G, Bm, _ = geometric_factors(*box_coords(n, lx, amp, els), lx)
        h1 = None if h1_glob is None else scatter(h1_glob, ids[els])
        xe = scatter(x_glob, ids[els])
        w = ax_einsum(xe, *M, h1, *G)
        if h2 is not None:
            w = w + h2 * Bm * xe
        w = w.reshape(len(els), -1)
        out[q] = np.sum(w[flat[els] == g])
    return out
