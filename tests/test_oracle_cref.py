"""The plain C loop nest agrees with the numpy oracle forms."""
import numpy as np
import pytest

import synth
from oracle.gll import listing_matrices
from oracle.ax import ax_einsum
from oracle import cref


@pytest.mark.parametrize("lx", [2, 5, 8, 12])
def test_c_loop_nest_matches_einsum(lx):
    G, h1 = synth.random_spd_factors(5, lx, 21)
    u = synth.local_normal(5, lx, 22)
    M = listing_matrices(lx)
    ref = ax_einsum(u, *M, h1, *G)
    got = cref.ax_ref(u, *M, h1, *G)
    assert np.max(np.abs(got - ref)) < 1e-14 * np.max(np.abs(ref))
    got1 = cref.ax_ref(u, *M, None, *G)
    ref1 = ax_einsum(u, *M, None, *G)
    assert np.max(np.abs(got1 - ref1)) < 1e-14 * np.max(np.abs(ref1))
