"""Gather-scatter: assembly of element-local vectors over shared nodes.

Paper Sec. 2.1 names gather-scatter as one of the two main ingredients of the
solver.  With Q the scatter from unique (global) nodes to element-local nodes
(u_L = u_G[id_L]), gather-scatter is u <- Q Q^T u: every local copy of a node
receives the sum of all copies (summation in any order; the assembled value is
unique up to rounding).  A node with a negative id is a Dirichlet node: it is
no unknown, so Q^T skips it and Q gives it the value 0 (the masked
gather-scatter of a homogeneous Dirichlet problem); its multiplicity is taken
as 1.

Pins: gs(1) = multiplicity, exactly; the multiplicity census of a periodic
element ((N-1)^3 ones, 6(N-1)^2 twos, 12(N-1) fours, 8 eights); the weighted
count sum(1/mult) = number of unique nodes; gs(Q u_G) = mult * Q u_G
(tests/test_oracle_gs.py).
"""
import numpy as np


def gather(u_local, ids, n_unique):
    """Q^T u: sum of the local copies per global id (Dirichlet nodes skipped)."""
    free = ids.ravel() >= 0
    return np.bincount(ids.ravel()[free], weights=u_local.ravel()[free], minlength=n_unique)


def scatter(u_unique, ids):
    """Q u: copy each unique value to all its local nodes (0 on Dirichlet nodes)."""
    out = np.zeros(ids.shape, dtype=np.asarray(u_unique).dtype)
    free = ids >= 0
    out[free] = u_unique[ids[free]]
    return out


def gs(u_local, ids, n_unique):
    return scatter(gather(u_local, ids, n_unique), ids)


def multiplicity(ids, n_unique):
    """Number of local copies of each local node's global id."""
    free = ids >= 0
    counts = np.bincount(ids[free], minlength=n_unique)
    mult = np.ones(ids.shape)
    mult[free] = counts[ids[free]]
    return mult


def weighted_dot(u_local, v_local, mult):
    """(u, v) = sum_L u_L v_L / mult_L, which is u_G . v_G for continuous
    u, v (u = Q u_G, v = Q v_G)."""
    return float(np.sum(u_local * v_local / mult))
