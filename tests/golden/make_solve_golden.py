"""Write the reference solutions of the 32^3 solves (tests/golden/solve_*.json).

Calls only the oracle (oracle/cref.py, the plain-C statement pinned against
the numpy oracle) and the seeded draws of ``synth``.  For each workload it
solves A x = b by float64 Jacobi-PCG to a relative residual of 1e-13 and
stores, at 1024 unique nodes drawn with a fixed seed, the right-hand side b
and the solution x*, plus the norms of the whole vectors.

Workloads (32^3 box, lx = 8, deformation amplitude 0.1, h1 = 1, the 32
Fourier modes of seed 2, |k|_inf <= 8):
  periodic   Poisson, right-hand side mean removed, x* mean-free;
  dirichlet  Poisson with u = 0 on the boundary (boundary nodes no unknowns);
  helmholtz  A + h2 B with h2 = 1e3 on the periodic box, f = 1 + the Fourier sum.

Usage: python tests/golden/make_solve_golden.py [periodic|dirichlet|helmholtz ...]
(about 5-10 minutes per workload on 8 cores).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import cref  # noqa: E402

N, LX, AMP, SEED_MODES, SEED_NODES, NSAMPLE = 32, 8, 0.1, 2, 61, 1024
WORKLOADS = {
    "periodic": dict(dirichlet=False, h2=None, const=0.0),
    "dirichlet": dict(dirichlet=True, h2=None, const=0.0),
    "helmholtz": dict(dirichlet=False, h2=1e3, const=1.0),
}


def path(name):
    return os.path.join(HERE, f"solve_{name}_n{N}_lx{LX}.json")


def make(name):
    cfg = WORKLOADS[name]
    t0 = time.time()
    box = cref.BigBox(N, LX, AMP, dirichlet=cfg["dirichlet"], h2=cfg["h2"])
    k, am, ph = synth.fourier_modes(SEED_MODES)
    b = box.fourier_rhs(k, am, ph, const=cfg["const"])
    x, its, rel = box.pcg(b, tol=1e-13, maxit=200000)
    gids = synth.choice(SEED_NODES, box.nu, NSAMPLE)
    out = {
        "what": f"float64 Jacobi-PCG reference solution of the {name} 32^3 solve",
        "script": "tests/golden/make_solve_golden.py (calls only oracle/cref.py)",
        "n": N, "lx": LX, "amp": AMP, "h1": 1.0, "h2": cfg["h2"], "dirichlet": cfg["dirichlet"],
        "rhs": {"fourier_modes_seed": SEED_MODES, "count": 32, "kmax": 8, "constant": cfg["const"],
                "mean_removed": box.project},
        "n_unique": int(box.nu), "iterations": int(its), "relres": rel, "tol": 1e-13,
        "b_norm2": float(np.linalg.norm(b)), "x_norm2": float(np.linalg.norm(x)),
        "x_maxabs": float(np.max(np.abs(x))), "x_sum": float(x.sum()),
        "sample_seed": SEED_NODES, "sample_ids": [int(g) for g in gids],
        "b_sample": [float(v) for v in b[gids]], "x_sample": [float(v) for v in x[gids]],
    }
    with open(path(name), "w") as f:
        json.dump(out, f, indent=0)
    print(f"{name}: {its} its, relres {rel:.3e}, {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    for nm in (sys.argv[1:] or list(WORKLOADS)):
        make(nm)
