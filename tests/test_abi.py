"""The C ABI: every symbol declared in include/sem.h is exported by libsem.so
and bound by the Python layer; host-only entry points work without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sem.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sem_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_2506_20994_amd as P
    lib = ctypes.CDLL(P.lib_path)
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
        assert n in P.EXPORTS, f"{n} not bound in the Python layer"


def test_gll_host_entry_point():
    import paper_2506_20994_amd as P
    from oracle.gll import gll_nodes_weights, listing_matrices
    for lx in range(2, 13):
        xi, w, dx, dxt = P.sem_gll(lx)
        xo, wo = gll_nodes_weights(lx - 1)
        assert np.max(np.abs(xi - xo)) < 1e-15
        assert np.max(np.abs(w - wo)) < 1e-15
        ref = listing_matrices(lx)[0]
        assert np.max(np.abs(dx - ref)) < 1e-14 * np.max(np.abs(ref))
        np.testing.assert_array_equal(dxt, dx.T)
    with pytest.raises(P.SemError) as ei:
        P.sem_gll(13)
    assert ei.value.code == P.SEM_EUNSUPPORTED_LX
    with pytest.raises(P.SemError):
        P.sem_gll(1)
