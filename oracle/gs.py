"""Gather-scatter: assembly of element-local vectors over shared nodes.

Paper Sec. 2.1 names gather-scatter as one of the two main ingredients of the
solver.  With Q the scatter from unique (global) nodes to element-local nodes
(u_L = u_G[id_L]), gather-scatter is u <- Q Q^T u: every local copy of a node
receives the sum of all copies (summation in any order; the assembled value is
unique up to rounding).  Reading: periodic boxes, so no node is masked.

Pins: gs(1) = multiplicity, exactly; the multiplicity census of a periodic
element ((N-1)^3 ones, 6(N-1)^2 twos, 12(N-1) fours, 8 eights); the weighted
count sum(1/mult) = number of unique nodes; gs(Q u_G) = mult * Q u_G
(tests/test_oracle_gs.py).
"""
import numpy as np


def gather(u_local, ids, n_unique):
    """Q^T u: sum of the local copies per global id."""
    return np.bincount(ids.ravel(), weights=u_local.ravel(), minlength=n_unique)


def scatter(u_unique, ids):
    """Q u: copy each unique value to all its local nodes."""
    return u_unique[ids]


def gs(u_local, ids, n_unique):
    return scatter(gather(u_local, ids, n_unique), ids)


def multiplicity(ids, n_unique):
    """Number of local copies of each local node's global id."""
    counts = np.bincount(ids.ravel(), minlength=n_unique)
    return counts[ids].astype(np.float64)


def weighted_dot(u_local, v_local, mult):
    """(u, v) = sum_L u_L v_L / mult_L, which is u_G . v_G for continuous
    u, v (u = Q u_G, v = Q v_G)."""
    return float(np.sum(u_local * v_local / mult))
