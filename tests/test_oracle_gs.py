"""Pins for oracle.gs: multiplicities and assembly identities are exact."""
import numpy as np
import pytest

import synth
from oracle.mesh import global_ids, n_unique
from oracle.gs import gs, gather, scatter, multiplicity, weighted_dot


@pytest.mark.parametrize("n,lx", [(2, 3), (3, 5), (4, 8), (2, 2)])
def test_multiplicity(n, lx):
    ids = global_ids(n, lx)
    nu = n_unique(n, lx)
    m = multiplicity(ids, nu)
    np.testing.assert_array_equal(gs(np.ones(ids.shape), ids, nu), m)
    N = lx - 1
    vals, counts = np.unique(m[0], return_counts=True)
    census = dict(zip(vals.astype(int), counts))
    expect = {1: (N - 1) ** 3, 2: 6 * (N - 1) ** 2, 4: 12 * (N - 1), 8: 8}
    expect = {k: v for k, v in expect.items() if v > 0}
    assert census == expect
    assert abs(np.sum(1.0 / m) - nu) < 1e-9 * nu
    assert np.sum(1.0 / m) == pytest.approx(n ** 3 * N ** 3)


def test_gs_of_continuous_field():
    n, lx = 3, 4
    ids = global_ids(n, lx)
    nu = n_unique(n, lx)
    uG = synth.unique_normal(nu, 0)
    uL = scatter(uG, ids)
    m = multiplicity(ids, nu)
    np.testing.assert_allclose(gs(uL, ids, nu), m * uL, rtol=1e-15)
    vG = synth.unique_normal(nu, 1)
    assert weighted_dot(uL, scatter(vG, ids), m) == pytest.approx(uG @ vG, rel=1e-13)
    np.testing.assert_allclose(gather(uL / m, ids, nu), uG, rtol=1e-14)
