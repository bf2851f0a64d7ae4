"""The multigrid V-cycle (sem_mg_*) against the oracle (oracle/mg.py): level
shapes, Lanczos estimates of lmax against the oracle's exact eigenvalues, the
V-cycle applied to random vectors element by element (the oracle taking the
GPU's lmax, so both run the same Chebyshev polynomial), flexible-CG solves
with it against the oracle's solution, and the iteration count's independence
of the mesh size."""
import numpy as np
import pytest
import torch

import synth
from oracle import mg as omg
from oracle.solve import BoxProblem, pcg

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2506_20994_amd")
from paper_2506_20994_amd.box import BoxOperator  # noqa: E402

# float32 V-cycle against the float64 oracle, max |z - z_ref| / max |z_ref|:
# every level's vectors and operators are float32 (relative rounding 6e-8 per
# operation, a few hundred operations along any path through the levels) and
# the coarse solve multiplies by an inverse of condition number below 1e3 on
# these boxes; bound 1e-4.
MG_TOL = 1e-4


def _plan_order(ids, nu):
    """plan index of every global id (unique nodes numbered by first appearance)"""
    flat = ids.ravel()
    free = flat >= 0
    _, first = np.unique(flat[free], return_index=True)
    plan_of = np.empty(nu, dtype=np.int64)
    plan_of[np.argsort(first)] = np.arange(nu)
    return plan_of


CASES = [  # n, lx, amp, dirichlet, h2, degree, lo, galerkin
    (4, 8, 0.1, False, None, 2, 0.3, False),
    (4, 4, 0.15, True, None, 2, 0.15, False),   # the lx = 2 level folds at 0.15: halved amplitude
    (4, 6, 0.12, True, None, 3, 0.2, False),
    (2, 5, 0.1, False, 20.0, 3, 0.3, False),
    (4, 3, 0.1, True, 5.0, 1, 0.2, False),
    # Galerkin lx = 2 levels: from a p-level (lx 4, 3, 5 -> 2), then h-levels; the
    # periodic singular coarsest level; Helmholtz; a first level of lx = 2 (its
    # own element matrices feed the h-product)
    (4, 4, 0.15, True, None, 2, 0.15, True),
    (4, 8, 0.1, False, None, 2, 0.3, True),
    (4, 6, 0.12, True, None, 3, 0.2, True),
    (2, 5, 0.1, False, 20.0, 3, 0.3, True),
    (4, 2, 0.1, True, 5.0, 2, 0.2, True),
    # every p-transfer pair the level shapes produce (lx 7 -> 3, 9 -> 4, 10 -> 5, 11 -> 5, 12 -> 6)
    (2, 7, 0.1, True, None, 2, 0.2, False),
    (2, 9, 0.1, False, None, 2, 0.3, True),
    (2, 10, 0.1, False, None, 2, 0.3, True),
    (2, 11, 0.1, True, None, 2, 0.2, True),
    (2, 12, 0.1, False, None, 2, 0.3, True),
]


@pytest.mark.parametrize("n,lx,amp,dirichlet,h2,degree,lo,galerkin", CASES)
def test_vcycle_matches_oracle(sem_ctx, n, lx, amp, dirichlet, h2, degree, lo, galerkin):
    op = BoxOperator(sem_ctx, n, lx, amp, dirichlet=dirichlet, keep_coords=False)
    mg = op.multigrid(h2=h2 or 0.0, degree=degree, lo=lo, galerkin=galerkin)
    H = omg.Hierarchy(n, lx, amp, dirichlet=dirichlet, h2=h2, degree=degree, lo=lo, galerkin=galerkin)
    nl = P.sem_mg_levels(mg)
    assert nl == len(H.shapes)
    lmax = []
    for q, (nq, lq, _) in enumerate(H.shapes):
        gn, glx, gnu, glm, gam = P.sem_mg_level_info(mg, q)
        assert (gn, glx, gnu, gam) == (nq, lq, H.boxes[q].nu, H.amps[q]), q
        if q + 1 < nl:
            # Lanczos Ritz values lie below lmax; 20 steps come within a few per cent
            assert 0.95 * H.lmax[q] <= glm <= (1 + 1e-4) * H.lmax[q], (q, glm, H.lmax[q])
            lmax.append(glm)
    H.set_lmax(lmax)
    B = H.boxes[0]
    plan_of = _plan_order(B.ids, B.nu)
    rG = synth.unique_normal(B.nu, 70)
    zref = H.vcycle(rG)
    rp = np.empty(B.nu)
    rp[plan_of] = rG
    for dt in (torch.float64, torch.float32):
        r = torch.from_numpy(rp).to(dt).cuda()
        z = torch.full_like(r, float("nan"))
        P.sem_mg_apply(mg, z, r)
        torch.cuda.synchronize()
        zg = z.double().cpu().numpy()[plan_of]
        err = np.max(np.abs(zg - zref)) / np.max(np.abs(zref))
        assert err <= MG_TOL, (dt, err)
    mg.close()
    op.gs.close()


def test_vcycle_with_bf16_fine_level_matches_oracle(sem_ctx):
    """fine_bf16: the finest level's smoothing operator with bfloat16 factors,
    against the oracle whose finest operator is assembled from the same
    bfloat16-rounded factors (float64 -> float32 -> bfloat16, reading R16);
    the Jacobi diagonal stays the float64 one on both sides."""
    from oracle.assemble import assembled_matrix
    from oracle.quant import to_bf16
    n, lx, amp = 4, 8, 0.1
    op = BoxOperator(sem_ctx, n, lx, amp, keep_coords=False)
    mg = op.multigrid(degree=2, lo=0.15, fine_bf16=True)
    H = omg.Hierarchy(n, lx, amp, degree=2, lo=0.15)
    B = H.boxes[0]
    H.A[0] = assembled_matrix(B.Dh, None, tuple(to_bf16(g) for g in B.G), B.ids, B.nu).tocsr()
    H.set_lmax([P.sem_mg_level_info(mg, q)[3] for q in range(len(H.shapes) - 1)])
    plan_of = _plan_order(B.ids, B.nu)
    rG = synth.unique_normal(B.nu, 73)
    zref = H.vcycle(rG)
    rp = np.empty(B.nu)
    rp[plan_of] = rG
    r = torch.from_numpy(rp).cuda()
    z = torch.full_like(r, float("nan"))
    P.sem_mg_apply(mg, z, r)
    torch.cuda.synchronize()
    zg = z.cpu().numpy()[plan_of]
    err = np.max(np.abs(zg - zref)) / np.max(np.abs(zref))
    assert err <= MG_TOL, err
    mg.close()
    op.gs.close()


def test_vcycle_is_symmetric(sem_ctx):
    """V is a symmetric map: u^T V(v) = v^T V(u) up to float32 rounding."""
    op = BoxOperator(sem_ctx, 4, 6, 0.1, keep_coords=False)
    mg = op.multigrid()
    nu = op.n_unique
    u = torch.from_numpy(synth.unique_normal(nu, 71)).cuda()
    v = torch.from_numpy(synth.unique_normal(nu, 72)).cuda()
    Vu, Vv = torch.empty_like(u), torch.empty_like(v)
    P.sem_mg_apply(mg, Vu, u)
    P.sem_mg_apply(mg, Vv, v)
    torch.cuda.synchronize()
    a, b = float(u @ Vv), float(v @ Vu)
    assert abs(a - b) <= 1e-5 * (abs(a) + abs(b))
    assert float(u @ Vu) > 0 and float(v @ Vv) > 0
    mg.close()
    op.gs.close()


def test_vcycle_graph_replays_equal_eager_launches(sem_ctx):
    """The V-cycle replayed as a captured graph (the default) equals its
    launches one by one, bit for bit, on every replay, with eager work (new
    right-hand sides written in between) and float64 / float32 vectors."""
    op = BoxOperator(sem_ctx, 4, 8, 0.1, keep_coords=False)
    mg = op.multigrid(n_coarse=2)
    nu = op.n_unique
    for dt in (torch.float64, torch.float32):
        r = torch.empty(nu, dtype=dt, device="cuda")
        z_graph, z_eager = torch.empty_like(r), torch.empty_like(r)
        for rep in range(3):
            r.copy_(torch.from_numpy(synth.unique_normal(nu, 90 + rep)))
            P.sem_mg_set_graphs(mg, 1)
            P.sem_mg_apply(mg, z_graph, r)
            torch.cuda.synchronize()
            P.sem_mg_set_graphs(mg, 0)
            P.sem_mg_apply(mg, z_eager, r)
            torch.cuda.synchronize()
            assert torch.equal(z_graph, z_eager), (dt, rep)
            assert torch.isfinite(z_graph).all()
    mg.close()
    op.gs.close()


@pytest.mark.parametrize("dirichlet,h2", [(False, None), (True, None), (False, 20.0)])
@pytest.mark.parametrize("prec,mode", [("f64", 0), ("f32", 1)])
def test_flexible_cg_with_multigrid(sem_ctx, dirichlet, h2, prec, mode):
    """Flexible CG with the V-cycle on a 4^3 lx = 8 box: converges to relres
    1e-10 (recomputed by the oracle), to the oracle's solution, in far fewer
    iterations than Jacobi-PCG."""
    n, lx, amp = 4, 8, 0.1
    op = BoxOperator(sem_ctx, n, lx, amp, dirichlet=dirichlet)
    ref = BoxProblem(n, lx, amp, dirichlet=dirichlet, h2=h2)
    k, a, ph = synth.fourier_modes(3)
    b = op.fourier_rhs(k, a, ph, project=(not dirichlet and h2 is None))
    bref = ref.fourier_rhs(k, a, ph)
    mg = op.multigrid(h2=h2 or 0.0)
    code = P.SEM_SOLVE_F64 if prec == "f64" else P.SEM_SOLVE_F32_IR
    h2b = None if h2 is None else h2 * op.bm
    cg = op.solver(code, h2b=h2b, mg=mg)
    x = torch.empty_like(b)
    rc, st = P.sem_cg_solve(cg, x, b, tol=1e-10, precision=code, ir_mode=mode, mg=mg)
    torch.cuda.synchronize()
    assert rc == P.SEM_OK and st["converged"] and st["jacobi_steps"] == 0 and not st["fell_back"], st
    free = ref.ids >= 0
    xg = np.zeros(ref.nu)
    xg[ref.ids[free]] = x.cpu().numpy()[free]
    assert np.linalg.norm(bref - ref.apply(xg)) / np.linalg.norm(bref) <= 1.2e-10
    xs, itj, _ = pcg(ref.apply, bref, 1.0 / ref.diagonal(), tol=1e-13, project=ref.project)
    assert np.max(np.abs(xg - xs)) <= 1e-6 * np.max(np.abs(xs))
    _, itj, _ = pcg(ref.apply, bref, 1.0 / ref.diagonal(), tol=1e-10, project=ref.project)
    print(f"dirichlet={dirichlet} h2={h2} {prec}: multigrid FCG {st['iterations']} its, Jacobi-PCG {itj}")
    assert st["iterations"] <= 0.25 * itj
    cg.close()
    mg.close()
    op.gs.close()


def test_multigrid_iterations_do_not_grow_with_the_mesh(sem_ctx):
    """The V-cycle keeps the flexible-CG iteration count nearly flat from 8^3
    to 16^3 elements (lx = 8, amplitude 0.1), where Jacobi-PCG's doubles."""
    its = {}
    for n in (8, 16):
        op = BoxOperator(sem_ctx, n, 8, 0.1)
        k, a, ph = synth.fourier_modes(2)
        b = op.fourier_rhs(k, a, ph)
        mg = op.multigrid()
        cg = op.solver(P.SEM_SOLVE_F32_IR, mg=mg)
        x = torch.empty_like(b)
        rc, st = P.sem_cg_solve(cg, x, b, tol=1e-10, precision=P.SEM_SOLVE_F32_IR, ir_mode=1, mg=mg)
        assert rc == P.SEM_OK and st["converged"], st
        its[n] = st["iterations"]
        cg.close()
        mg.close()
        op.gs.close()
    print(f"multigrid FCG iterations: {its}")
    assert its[16] <= 1.5 * its[8], its


def test_galerkin_levels_on_a_folding_box(sem_ctx):
    """8^3 lx = 8 Dirichlet box at amplitude 0.15, where the re-discretised
    lx = 2 levels fold and take a halved amplitude: flexible CG with Galerkin
    lx = 2 levels converges to relres 1e-10 (recomputed by the oracle) in fewer
    iterations than with the re-discretised ones."""
    n, lx, amp = 8, 8, 0.15
    op = BoxOperator(sem_ctx, n, lx, amp, dirichlet=True)
    ref = BoxProblem(n, lx, amp, dirichlet=True)
    k, a, ph = synth.fourier_modes(3)
    b = op.fourier_rhs(k, a, ph, project=False)
    bref = ref.fourier_rhs(k, a, ph)
    free = ref.ids >= 0
    its = {}
    for g in (False, True):
        mg = op.multigrid(galerkin=g, n_coarse=2)
        amps = [P.sem_mg_level_info(mg, q)[4] for q in range(P.sem_mg_levels(mg))]
        cg = op.solver(P.SEM_SOLVE_F32_IR, mg=mg)
        x = torch.empty_like(b)
        rc, st = P.sem_cg_solve(cg, x, b, tol=1e-10, precision=P.SEM_SOLVE_F32_IR, ir_mode=1, mg=mg)
        torch.cuda.synchronize()
        assert rc == P.SEM_OK and st["converged"] and not st["fell_back"], st
        xg = np.zeros(ref.nu)
        xg[ref.ids[free]] = x.cpu().numpy()[free]
        assert np.linalg.norm(bref - ref.apply(xg)) / np.linalg.norm(bref) <= 1.2e-10
        its[g] = st["iterations"]
        print(f"galerkin={g}: {its[g]} its, level amplitudes {amps}")
        if g:
            assert amps[0] == amp and all(v == 0.0 for v, (_, l, _) in zip(amps[1:], omg.level_shapes(n, lx)[1:])
                                          if l == 2)
        cg.close()
        mg.close()
    assert its[True] < its[False], its
    op.gs.close()


def test_multigrid_errors(sem_ctx):
    import ctypes
    from paper_2506_20994_amd import _binding as Bd
    op = BoxOperator(sem_ctx, 2, 4, 0.1, h1_unique=np.ones(216), keep_coords=False)
    A = Bd.SemOperator(*[t.data_ptr() for t in op.D], op.h1.data_ptr(), *[t.data_ptr() for t in op.G],
                       op.nel, op.lx, None)
    o = Bd.SemMgOpts(2, 0.1, 0, 0.0, 0, 0.0, 0.0, 0, 0)
    out = ctypes.c_void_p()
    rc = Bd.lib().sem_mg_create(sem_ctx.bind(), op.gs.handle, ctypes.byref(A), ctypes.byref(o), ctypes.byref(out))
    assert rc == P.SEM_EINVAL and not out.value       # the levels are built with h1 = 1
    op.gs.close()
    op = BoxOperator(sem_ctx, 2, 4, 0.1, keep_coords=False)
    with pytest.raises(P.SemError) as ei:             # n does not match the operator
        P.sem_mg_create(sem_ctx, op.gs, op.D, op.G, op.nel, op.lx, 3, 0.1)
    assert ei.value.code == P.SEM_EINVAL
    with pytest.raises(P.SemError) as ei:             # Dirichlet flag does not match the plan
        P.sem_mg_create(sem_ctx, op.gs, op.D, op.G, op.nel, op.lx, 2, 0.1, dirichlet=True)
    assert ei.value.code == P.SEM_EINVAL
    with pytest.raises(P.SemError) as ei:             # mass term without h2
        P.sem_mg_create(sem_ctx, op.gs, op.D, op.G, op.nel, op.lx, 2, 0.1, h2b=op.bm)
    assert ei.value.code == P.SEM_EINVAL
    mg = op.multigrid()
    lp = P.sem_lp_create(sem_ctx, op.nel)
    with pytest.raises(P.SemError) as ei:             # two preconditioners
        op.solver(P.SEM_SOLVE_F64, mg=mg, learned=lp)
    assert ei.value.code == P.SEM_EINVAL
    with pytest.raises(P.SemError) as ei:
        P.sem_mg_set_lmax(mg, P.sem_mg_levels(mg) - 1, 1.0)     # the coarsest level has none
    assert ei.value.code == P.SEM_EINVAL
    lp.close()
    mg.close()
    op.gs.close()
    op = BoxOperator(sem_ctx, 13, 2, 0.05, keep_coords=False)  # 13^3 coarsest unknowns > 2048
    with pytest.raises(P.SemError) as ei:
        op.multigrid()
    assert ei.value.code == P.SEM_EINVAL
    op.gs.close()
