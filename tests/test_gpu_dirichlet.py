"""The Dirichlet box on the GPU (homogeneous Dirichlet conditions on the whole
boundary; boundary nodes carry id -1) against the oracle: mesh ids, masked
gather-scatter, multiplicity and owner weights, the solvers in float64 and
with float32 / bfloat16 inner work, and the learned preconditioner's linear
apply and flexible CG on a masked plan."""
import numpy as np
import pytest
import torch

import synth
from oracle import mlp
from oracle.gs import gs as oracle_gs, multiplicity, scatter
from oracle.mesh import box_coords, global_ids_dirichlet, n_unique_dirichlet
from oracle.solve import BoxProblem, pcg

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2506_20994_amd")
from paper_2506_20994_amd.box import BoxOperator  # noqa: E402

GRAD_TOL = 2e-2    # normwise, bf16 operands with float32 accumulation (linear apply)


def _unique(ref, xl):
    """Unique vector from a continuous local one (Dirichlet nodes skipped)."""
    out = np.zeros(ref.nu)
    free = ref.ids >= 0
    out[ref.ids[free]] = xl[free]
    return out


def _plan_order(ids):
    """plan index of every oracle id: the plan numbers the free nodes in order
    of first appearance in the local layout."""
    flat = ids.ravel()
    free = flat[flat >= 0]
    _, first = np.unique(free, return_index=True)
    plan_of = np.empty(len(first), dtype=np.int64)
    plan_of[np.argsort(first)] = np.arange(len(first))
    return plan_of


@pytest.mark.parametrize("n,lx", [(1, 2), (1, 3), (2, 5), (3, 8), (2, 12)])
def test_dirichlet_mesh_and_plan(sem_ctx, n, lx):
    amp = 0.1
    op = BoxOperator(sem_ctx, n, lx, amp, dirichlet=True)
    ids = global_ids_dirichlet(n, lx)
    np.testing.assert_array_equal(op.ids.cpu().numpy(), ids)
    x, y, z = box_coords(n, lx, amp)
    for a, b in ((op.x, x), (op.y, y), (op.z, z)):
        np.testing.assert_allclose(a.cpu().numpy(), b, rtol=0, atol=1e-14)
    nu = n_unique_dirichlet(n, lx)
    assert P.sem_gs_info(op.gs)[0] == nu == op.n_unique
    assert P.sem_gs_dirichlet_count(op.gs) == int((ids < 0).sum())
    np.testing.assert_array_equal(op.mult.cpu().numpy(), multiplicity(ids, nu))
    u = torch.from_numpy(synth.local_normal(n ** 3, lx, 5)).cuda()
    ref = oracle_gs(u.cpu().numpy(), ids, nu)
    P.sem_gs(op.gs, u)
    g = u.cpu().numpy()
    assert np.all(g[ids < 0] == 0.0)
    np.testing.assert_allclose(g, ref, rtol=1e-14, atol=1e-14 * max(np.abs(ref).max(), 1.0))
    owner = torch.empty_like(u)
    P.sem_gs_owner(op.gs, owner)
    w = owner.cpu().numpy()
    assert np.all(w[ids < 0] == 0.0)
    assert w.sum() == nu
    if nu > 0:
        uG = synth.unique_normal(nu, 6)
        sc = op.scatter(uG)
        np.testing.assert_array_equal(sc.cpu().numpy(), scatter(uG, ids))
    with pytest.raises(P.SemError):
        P.sem_remove_mean(op.gs, u)
    if nu == 0:
        with pytest.raises(P.SemError):
            op.solver(P.SEM_SOLVE_F64)
    op.gs.close()


def _setup(ctx, n, lx, amp, with_h1=False, seed_rhs=2):
    nu = n_unique_dirichlet(n, lx)
    h1u = synth.unique_uniform(nu, 0.5, 2.0, 1) if with_h1 else None
    op = BoxOperator(ctx, n, lx, amp, h1_unique=h1u, dirichlet=True)
    k, a, ph = synth.fourier_modes(seed_rhs)
    b = op.fourier_rhs(k, a, ph)
    ref = BoxProblem(n, lx, amp, h1u, dirichlet=True)
    bref = ref.fourier_rhs(k, a, ph)
    return op, b, ref, bref


@pytest.mark.parametrize("n,lx,amp,h1", [(3, 5, 0.1, True), (2, 8, 0.15, False), (1, 3, 0.0, False)])
def test_dirichlet_pcg_f64(sem_ctx, n, lx, amp, h1):
    op, b, ref, bref = _setup(sem_ctx, n, lx, amp, with_h1=h1)
    bl = b.cpu().numpy()
    assert np.all(bl[ref.ids < 0] == 0.0)
    np.testing.assert_allclose(_unique(ref, bl), bref, rtol=0, atol=1e-13 * np.abs(bref).max())
    cg = op.solver(P.SEM_SOLVE_F64)
    x = torch.full_like(b, float("nan"))
    rc, st = P.sem_cg_solve(cg, x, b, tol=1e-10)
    torch.cuda.synchronize()
    assert rc == P.SEM_OK and st["converged"], st
    xl = x.cpu().numpy()
    assert np.all(xl[ref.ids < 0] == 0.0)
    xg = _unique(ref, xl)
    rel = np.linalg.norm(bref - ref.apply(xg)) / np.linalg.norm(bref)
    assert rel <= 1.2e-10 and st["relres"] <= 1e-10
    xo, ito, _ = pcg(ref.apply, bref, 1.0 / ref.diagonal(), tol=1e-10, project=False)
    assert abs(st["iterations"] - ito) <= 2, (st["iterations"], ito)
    xs, _, _ = pcg(ref.apply, bref, 1.0 / ref.diagonal(), tol=1e-13, project=False)
    assert np.max(np.abs(xg - xs)) <= 1e-6 * np.max(np.abs(xs))
    # the solution has a non-zero mean: nothing was projected
    assert abs(xg.sum()) > 1e-3 * np.abs(xg).sum()
    cg.close()
    op.gs.close()


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_dirichlet_refinement(sem_ctx, prec, mode):
    n, lx, amp = 3, 8, 0.1
    op, b, ref, bref = _setup(sem_ctx, n, lx, amp)
    code = P.SEM_SOLVE_F32_IR if prec == "f32" else P.SEM_SOLVE_BF16_IR
    cg = op.solver(code)
    x = torch.empty_like(b)
    rc, st = P.sem_cg_solve(cg, x, b, tol=1e-10, precision=code, ir_mode=mode)
    torch.cuda.synchronize()
    assert rc == P.SEM_OK and st["converged"], st
    xl = x.cpu().numpy()
    assert np.all(xl[ref.ids < 0] == 0.0)
    xg = _unique(ref, xl)
    rel = np.linalg.norm(bref - ref.apply(xg)) / np.linalg.norm(bref)
    assert rel <= 1.2e-10
    xs, _, _ = pcg(ref.apply, bref, 1.0 / ref.diagonal(), tol=1e-13, project=False)
    assert np.max(np.abs(xg - xs)) <= 1e-6 * np.max(np.abs(xs))
    cg.close()
    op.gs.close()


@pytest.mark.parametrize("jb", [False, True])
def test_dirichlet_linear_apply_unique(sem_ctx, jb):
    """The linear form's apply on a masked plan (27 elements, every one
    touching the boundary) against the oracle's symmetric block apply."""
    n, amp = 3, 0.1
    op = BoxOperator(sem_ctx, n, 8, amp, dirichlet=True)
    lp = P.sem_lp_create(sem_ctx, op.nel)
    P.sem_lp_set_linear(lp, 1)
    P.sem_lp_set_jacobi_base(lp, int(jb))
    op.bind(lp)
    W = synth.rng(70).standard_normal((512, 512)) * 0.05
    P.sem_lp_set_block(lp, W)
    ref = BoxProblem(n, 8, amp, dirichlet=True)
    rG = synth.unique_normal(ref.nu, 71)
    zl = mlp.apply_block(W.astype(np.float32).astype(np.float64), scatter(rG, ref.ids), ref.G, None,
                         ref.ids, ref.nu)
    zref = _unique(ref, zl)
    if jb:
        zref += rG / ref.diagonal()
    plan_of = _plan_order(ref.ids)
    rp = np.empty(ref.nu)
    rp[plan_of] = rG
    for dt in (torch.float64, torch.float32):
        r = torch.from_numpy(rp).to(dt).cuda()
        z = torch.full_like(r, float("nan"))
        P.sem_lp_apply_unique(lp, z, r)
        torch.cuda.synchronize()
        zg = z.double().cpu().numpy()[plan_of]
        assert np.all(np.isfinite(zg))
        assert np.linalg.norm(zg - zref) <= GRAD_TOL * np.linalg.norm(zref)
    lp.close()
    op.gs.close()


@pytest.mark.parametrize("prec", [P.SEM_SOLVE_F64, P.SEM_SOLVE_F32_IR])
def test_dirichlet_flexible_cg_with_block(sem_ctx, prec):
    """Flexible CG preconditioned by the classical element block on a masked
    plan: converges to the oracle's solution in fewer iterations than
    Jacobi-PCG."""
    from paper_2506_20994_amd import learned as LR
    n, lx, amp = 4, 8, 0.1
    op, b, ref, bref = _setup(sem_ctx, n, lx, amp)
    lp = P.sem_lp_create(sem_ctx, op.nel)
    op.bind(lp)
    P.sem_lp_set_block(lp, LR.reference_block(sem_ctx))
    x = torch.empty_like(b)
    cgj = op.solver(prec)
    _, stj = P.sem_cg_solve(cgj, x, b, tol=1e-10, precision=prec, ir_mode=1)
    cg = op.solver(prec, learned=lp)
    rc, st = P.sem_cg_solve(cg, x, b, tol=1e-10, precision=prec, ir_mode=1, learned=lp)
    torch.cuda.synchronize()
    assert rc == P.SEM_OK and st["converged"] and st["jacobi_steps"] == 0, st
    xl = x.cpu().numpy()
    assert np.all(xl[ref.ids < 0] == 0.0)
    xg = _unique(ref, xl)
    assert np.linalg.norm(bref - ref.apply(xg)) / np.linalg.norm(bref) <= 1.2e-10
    xs, _, _ = pcg(ref.apply, bref, 1.0 / ref.diagonal(), tol=1e-13, project=False)
    assert np.max(np.abs(xg - xs)) <= 1e-6 * np.max(np.abs(xs))
    print(f"dirichlet {n}^3 lx={lx} prec={prec}: jacobi {stj['iterations']} block {st['iterations']}")
    assert st["iterations"] < 0.6 * stj["iterations"]
    cg.close()
    cgj.close()
    lp.close()
    op.gs.close()
