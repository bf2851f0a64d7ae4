"""Training pipeline of the learned preconditioner: snapshot generation from
float64 Jacobi-PCG solves, minibatch training, held-out evaluation.

Orchestration only: every array is produced by libsem.so kernels (mesh,
geometry, solves, operator, features, MLP, Adam); random draws come from
``synth``.  Recipe:
  * training boxes: n^3 periodic, the network's lx (8 by default),
    deformation amplitude ~ U[0, 0.2],
    draws whose minimum det J falls below 5% of the undeformed value rejected
    (the map folds near 1 / (2 pi));
  * right-hand side: 32 random Fourier modes per box ("fourier"), or white
    noise b_G ~ N(0, 1) per unique node, mean removed ("noise");
  * x* from float64 Jacobi-PCG to 1e-12; snapshots x_k at iterations k spread
    log-uniformly over the solve (k = 0, i.e. r = b and e = x*, included when
    `include_zero`), r_k = b - A x_k, e_k = x* - x_k;
  * per snapshot, `elems_per_snapshot` random elements become training rows.
The preconditioner that beats Jacobi is the linear form trained with the
energy-norm loss (mu = 1) on white-noise pairs at k = 0 (r = b, e = x*): the
regression target is then the element block of the inverse operator.
Smooth (Fourier) right-hand sides or too few rows leave the symmetric part of
the learned block indefinite, and flexible CG falls back to Jacobi.
"""
import time

import numpy as np
import torch

import synth
from . import _binding as B
from .box import BoxOperator


def generate(ctx, lp, n=16, boxes=16, snapshots=16, elems_per_snapshot=64, seed=100,
             amp_range=(0.0, 0.2), min_rel_detj=0.05, rhs="fourier", include_zero=False,
             verbose=False, dirichlet=False):
    """Returns (X bf16 [rows, padded feature width (528 at lx = 8)], T float32
    [rows, lx^3], info) for the network's lx.  With ``dirichlet`` the pairs
    come from boxes with u = 0 on the boundary (no mean projection of the
    right-hand side)."""
    lx = lp.lx
    nel = n ** 3
    rows = boxes * snapshots * elems_per_snapshot
    X = torch.zeros((rows, lp.n_in_pad), dtype=torch.bfloat16, device="cuda")
    T = torch.zeros((rows, lp.n_out), dtype=torch.float32, device="cuda")
    row, box, draw, rejected = 0, 0, 0, 0
    t0 = time.perf_counter()
    amps = []
    while box < boxes:
        a = float(synth.amplitudes(seed + draw, 1, *amp_range)[0])
        draw += 1
        try:
            op = BoxOperator(ctx, n, lx, a, dirichlet=dirichlet)
        except B.SemError:
            rejected += 1
            continue
        if op.min_detj * 8 * n ** 3 <= min_rel_detj:
            rejected += 1
            continue
        amps.append(a)
        if rhs == "noise":
            b = op.scatter(synth.unique_normal(op.n_unique, seed + 10_000 + box))
            if not dirichlet:
                B.sem_remove_mean(op.gs, b)
        else:
            k, am, ph = synth.fourier_modes(seed + 10_000 + box)
            b = op.fourier_rhs(k, am, ph)
        cg = op.solver(B.SEM_SOLVE_F64)
        xs = torch.empty_like(b)
        _, st = B.sem_cg_solve(cg, xs, b, tol=1e-12, maxit=100000)
        kmax = max(1, st["iterations"] - 1)
        its = synth.snapshot_iterations(seed + 20_000 + box, snapshots, kmax)
        if include_zero:
            its = np.concatenate([[0], its])
        its = np.resize(its, snapshots)       # duplicates if the draw collapsed
        op.bind(lp)
        xk = torch.empty_like(b)
        rk = torch.empty_like(b)
        ek = torch.empty_like(b)
        for q, kq in enumerate(its):
            if kq == 0:
                xk.zero_()
            else:
                B.sem_cg_solve(cg, xk, b, tol=1e-12, maxit=int(kq), check_every=int(min(kq, 16)))
            els = torch.from_numpy(synth.choice(seed + 30_000 + box * 1000 + q, nel,
                                                elems_per_snapshot)).cuda()
            B.sem_lp_snapshot(lp, xk, xs, b, rk, ek, els, X, T, row)   # r = b - A x_k, e = x* - x_k
            row += elems_per_snapshot
        cg.close()
        op.gs.close()
        if verbose:
            print(f"[learned] box {box}: amp {a:.3f}, x* in {st['iterations']} its, "
                  f"snapshots {list(its[:4])}...", flush=True)
        box += 1
    torch.cuda.synchronize()
    info = {"rows": rows, "boxes": boxes, "rejected_draws": rejected, "amplitudes": amps,
            "seconds": time.perf_counter() - t0}
    return X, T, info


def train(lp, X, T, epochs=4, batch=1024, lr=1e-3, seed=500, verbose=False):
    """Minibatch Adam over (X, T); returns per-epoch mean losses."""
    rows = X.shape[0]
    nb = rows // batch
    loss = torch.zeros(nb, dtype=torch.float32, device="cuda")
    hist = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.from_numpy(synth.permutation(seed + ep, rows)).cuda()
        for q in range(nb):
            B.sem_lp_train_step(lp, X, T, perm[q * batch:(q + 1) * batch], lr, loss[q:q + 1])
        hist.append(float(loss.mean()))
        if verbose:
            print(f"[learned] epoch {ep}: loss {hist[-1]:.4e} ({time.perf_counter() - t0:.1f} s)",
                  flush=True)
    return hist


def init_network(lp, seed=7, mu=None, jacobi_base=None, out_scale=1.0, linear=None):
    """He-initialised weights (the last layer scaled by out_scale); mu >= 0
    selects the energy-norm loss; jacobi_base selects z = Minv r + network;
    linear selects the linear form (identity activations, no biases).  For the
    linear form, out_scale = 0 starts the folded matrix at zero, so that no
    random (indefinite) component of the initial product survives training."""
    if mu is not None:
        B.sem_lp_set_metric(lp, mu)
    if jacobi_base is not None:
        B.sem_lp_set_jacobi_base(lp, jacobi_base)
    if linear is not None:
        B.sem_lp_set_linear(lp, linear)
    params = synth.mlp_init(seed, (lp.n_in, lp.hidden, lp.hidden, lp.n_out))
    params[4] = params[4] * out_scale
    for s, p in enumerate(params):
        B.sem_lp_set(lp, s, p.astype(np.float32))


def reference_block(ctx, lx=8):
    """The classical counterpart of the learned block: kappa times the inverse
    of the assembled operator restricted to the nodes of one element (the local
    solve of one-level additive Schwarz with minimal overlap) of an undeformed
    periodic box, computed by the library (sem_lp_reference_block).  Returns
    float64 (lx^3, lx^3)."""
    return B.sem_lp_reference_block(ctx, lx)
