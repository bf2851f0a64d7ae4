"""GPU solves (float64 Jacobi-PCG and float64 refinement around float32 /
bfloat16 inner solves) against the oracle: right-hand-side parity, residuals
recomputed by the oracle's operator, errors against an oracle solution."""
import numpy as np
import pytest
import torch

import synth
from oracle.solve import BoxProblem, pcg
from oracle.gs import scatter

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2506_20994_amd")
from paper_2506_20994_amd.box import BoxOperator  # noqa: E402


def _setup(ctx, n, lx, amp, seed_rhs=2, with_h1=False):
    nu = (n * (lx - 1)) ** 3
    h1u = synth.unique_uniform(nu, 0.5, 2.0, 1) if with_h1 else None
    op = BoxOperator(ctx, n, lx, amp, h1_unique=h1u)
    k, a, ph = synth.fourier_modes(seed_rhs)
    b = op.fourier_rhs(k, a, ph)
    ref = BoxProblem(n, lx, amp, h1u)
    bref = ref.fourier_rhs(k, a, ph)
    return op, b, ref, bref


def _unique(ref, xl):
    """unique vector from a continuous local one (take the owner copy)"""
    out = np.zeros(ref.nu)
    out[ref.ids.ravel()] = xl.ravel()
    return out


@pytest.mark.parametrize("n,lx,amp,h1", [(3, 5, 0.1, True), (2, 8, 0.15, False), (4, 4, 0.0, False)])
def test_pcg_f64(sem_ctx, n, lx, amp, h1):
    op, b, ref, bref = _setup(sem_ctx, n, lx, amp, with_h1=h1)
    np.testing.assert_allclose(_unique(ref, b.cpu().numpy()), bref, rtol=0,
                               atol=1e-13 * np.abs(bref).max())
    cg = op.solver(P.SEM_SOLVE_F64)
    x = torch.empty_like(b)
    rc, st = P.sem_cg_solve(cg, x, b, tol=1e-10)
    torch.cuda.synchronize()
    assert rc == P.SEM_OK and st["converged"], st
    xg = _unique(ref, x.cpu().numpy())
    # the oracle re-checks the residual with its own operator and right-hand side
    rel = np.linalg.norm(bref - ref.apply(xg)) / np.linalg.norm(bref)
    assert rel <= 1.2e-10 and st["relres"] <= 1e-10
    assert abs(xg.sum()) <= 1e-10 * np.abs(xg).sum()
    xo, ito, _ = pcg(ref.apply, bref, 1.0 / ref.diagonal(), tol=1e-10)
    assert abs(st["iterations"] - ito) <= 2, (st["iterations"], ito)
    xs, _, _ = pcg(ref.apply, bref, 1.0 / ref.diagonal(), tol=1e-13)
    assert np.max(np.abs(xg - xs)) <= 1e-6 * np.max(np.abs(xs))
    cg.close()


@pytest.mark.parametrize("lx,prec,h1", [(7, "f64", True), (9, "f64", False), (11, "f64", True), (12, "f64", False),
                                        (7, "f32", False), (9, "bf16", True), (12, "f32", True), (12, "bf16", False)])
def test_solver_form_at_lx_with_shared_flux_storage(sem_ctx, lx, prec, h1):
    """The solver's operator at lx = 7, 9, 11, 12, where the r-flux of a slice
    overwrites the slice of u in LDS after a workgroup barrier (and lx = 12
    runs under a register floor): float64 Jacobi-PCG and float32 / bfloat16
    residual replacement on a 2^3 box against the oracle's operator and
    solution."""
    op, b, ref, bref = _setup(sem_ctx, 2, lx, 0.1, with_h1=h1)
    code = {"f64": P.SEM_SOLVE_F64, "f32": P.SEM_SOLVE_F32_IR, "bf16": P.SEM_SOLVE_BF16_IR}[prec]
    cg = op.solver(code)
    x = torch.empty_like(b)
    rc, st = P.sem_cg_solve(cg, x, b, tol=1e-10, precision=code, ir_mode=0 if prec == "f64" else 1)
    torch.cuda.synchronize()
    assert rc == P.SEM_OK and st["converged"], st
    xg = _unique(ref, x.cpu().numpy())
    rel = np.linalg.norm(bref - ref.apply(xg)) / np.linalg.norm(bref)
    assert rel <= 1.2e-10, rel
    xs, ito, _ = pcg(ref.apply, bref, 1.0 / ref.diagonal(), tol=1e-13)
    assert np.max(np.abs(xg - xs)) <= 1e-6 * np.max(np.abs(xs))
    if prec == "f64":
        _, ito, _ = pcg(ref.apply, bref, 1.0 / ref.diagonal(), tol=1e-10)
        assert abs(st["iterations"] - ito) <= 2, (st["iterations"], ito)
    cg.close()


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_refinement(sem_ctx, prec, mode):
    """mode 0: restarted refinement; mode 1: residual replacement."""
    n, lx, amp = 3, 8, 0.1
    op, b, ref, bref = _setup(sem_ctx, n, lx, amp)
    code = P.SEM_SOLVE_F32_IR if prec == "f32" else P.SEM_SOLVE_BF16_IR
    cg = op.solver(code)
    x = torch.empty_like(b)
    rc, st = P.sem_cg_solve(cg, x, b, tol=1e-10, precision=code, ir_mode=mode)
    torch.cuda.synchronize()
    assert rc == P.SEM_OK and st["converged"], st
    assert st["outer"] >= 2
    xg = _unique(ref, x.cpu().numpy())
    rel = np.linalg.norm(bref - ref.apply(xg)) / np.linalg.norm(bref)
    assert rel <= 1.2e-10
    xs, _, _ = pcg(ref.apply, bref, 1.0 / ref.diagonal(), tol=1e-13)
    err = np.max(np.abs(xg - xs)) / np.max(np.abs(xs))
    print(f"{prec} IR mode {mode}: outer={st['outer']} iters={st['iterations']} "
          f"relres={st['relres']:.2e} err={err:.2e}")
    assert err <= 1e-6
    cg.close()


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_refinement_with_h1(sem_ctx, prec):
    """A variable h1 (the bfloat16 solver copy folds it into the six factors):
    the refined solution still meets the oracle's residual and solution."""
    op, b, ref, bref = _setup(sem_ctx, 3, 8, 0.1, with_h1=True)
    code = P.SEM_SOLVE_F32_IR if prec == "f32" else P.SEM_SOLVE_BF16_IR
    cg = op.solver(code)
    x = torch.empty_like(b)
    rc, st = P.sem_cg_solve(cg, x, b, tol=1e-10, precision=code, ir_mode=1)
    torch.cuda.synchronize()
    assert rc == P.SEM_OK and st["converged"], st
    xg = _unique(ref, x.cpu().numpy())
    rel = np.linalg.norm(bref - ref.apply(xg)) / np.linalg.norm(bref)
    assert rel <= 1.2e-10
    xs, _, _ = pcg(ref.apply, bref, 1.0 / ref.diagonal(), tol=1e-13)
    assert np.max(np.abs(xg - xs)) <= 1e-6 * np.max(np.abs(xs))
    cg.close()


def test_solve_is_deterministic(sem_ctx):
    op, b, _, _ = _setup(sem_ctx, 2, 6, 0.1)
    cg = op.solver(P.SEM_SOLVE_F64)
    x1, x2 = torch.empty_like(b), torch.empty_like(b)
    P.sem_cg_solve(cg, x1, b, tol=1e-10)
    P.sem_cg_solve(cg, x2, b, tol=1e-10)
    torch.cuda.synchronize()
    assert torch.equal(x1, x2)
    cg.close()


def test_not_converged_and_errors(sem_ctx):
    op, b, _, _ = _setup(sem_ctx, 2, 6, 0.1)
    cg = op.solver(P.SEM_SOLVE_F64)
    x = torch.empty_like(b)
    rc, st = P.sem_cg_solve(cg, x, b, tol=1e-10, maxit=3, check_every=1)
    assert rc == P.SEM_NOT_CONVERGED and st["iterations"] == 3 and not st["converged"]
    with pytest.raises(P.SemError):
        P.sem_cg_solve(cg, x, b, tol=1e-10, precision=P.SEM_SOLVE_F32_IR)   # differs from set-up
    with pytest.raises(P.SemError):
        P.sem_cg_solve(cg, x, b, tol=0.0)
    # zero right-hand side: x = 0 immediately
    z = torch.zeros_like(b)
    rc, st = P.sem_cg_solve(cg, x, z, tol=1e-10)
    assert rc == P.SEM_OK and st["iterations"] == 0 and float(x.abs().max()) == 0.0
    cg.close()


def test_remove_mean_and_owner(sem_ctx):
    n, lx = 2, 5
    op = BoxOperator(sem_ctx, n, lx, 0.0, keep_coords=False)
    nu = (n * (lx - 1)) ** 3
    uu = synth.unique_normal(nu, 3) + 5.0
    u = op.scatter(uu)
    wgt = torch.empty_like(u)
    P.sem_gs_owner(op.gs, wgt)
    assert float(wgt.sum()) == nu
    assert float((wgt * u).sum()) == pytest.approx(uu.sum(), rel=1e-13)
    P.sem_remove_mean(op.gs, u)
    torch.cuda.synchronize()
    np.testing.assert_allclose(u.cpu().numpy(), scatter(uu - uu.mean(), op.ids.cpu().numpy()),
                               atol=1e-13)


_BIG = {}


def _bigbox(dirichlet, h2):
    """The C oracle's 32^3 lx = 8 box (amplitude 0.1) of the benchmark's solves;
    one held at a time (about 1.5 GB of host memory)."""
    from oracle import cref
    key = (dirichlet, h2)
    if key not in _BIG:
        _BIG.clear()
        _BIG[key] = cref.BigBox(32, 8, 0.1, dirichlet=dirichlet, h2=h2)
    return _BIG[key]


# error of a solve to relres 1e-10 against the oracle's solution to 1e-12,
# sqrt(sum (x - x*)^2 / sum x*^2) over 1024 sampled unique nodes
FULL_SIZE_ERR = 1e-6


@pytest.mark.parametrize("prec,mode,dirichlet,h2", [("f64", 0, False, None), ("f32", 1, False, None),
                                                     ("bf16", 1, False, None), ("f64", 0, True, None),
                                                     ("f32", 1, True, None), ("f32", 1, False, 1e3)])
def test_solve_full_size(sem_ctx, prec, mode, dirichlet, h2):
    """The benchmark's solves (32^3 box, lx = 8, amplitude 0.1, 32 Fourier modes,
    relres 1e-10; periodic, with Dirichlet conditions on the boundary, and the
    Helmholtz operator with h2 = 1e3 and source 1 + the Fourier sum) in float64
    PCG and float32 / bfloat16 residual replacement, against the plain-C oracle
    (oracle/sem_ref.c, pinned against the numpy oracle): the right-hand side
    (sem_fourier, sem_gs, projection) at every unique node, the residual 2-norm
    of the GPU's x recomputed by the oracle over all unique nodes, and x against
    the oracle's reference solution (tests/golden, relres 1e-12) at 1024 nodes."""
    import json
    import os
    from oracle.mesh import global_ids, global_ids_dirichlet
    n, lx, amp = 32, 8, 0.1
    op = BoxOperator(sem_ctx, n, lx, amp, dirichlet=dirichlet)
    k, a, ph = synth.fourier_modes(2)
    b = op.fourier_rhs(k, a, ph, project=(not dirichlet and h2 is None))
    if h2 is not None:              # the constant source f = 1: b += Q Q^T B 1
        mass = op.bm.clone()
        P.sem_gs(op.gs, mass)
        b += mass
    code = {"f64": P.SEM_SOLVE_F64, "f32": P.SEM_SOLVE_F32_IR, "bf16": P.SEM_SOLVE_BF16_IR}[prec]
    cg = op.solver(code, h2b=None if h2 is None else h2 * op.bm)
    x = torch.empty_like(b)
    rc, st = P.sem_cg_solve(cg, x, b, tol=1e-10, precision=code, ir_mode=mode)
    torch.cuda.synchronize()
    assert rc == P.SEM_OK and st["converged"] and st["relres"] <= 1e-10, st
    ids = global_ids_dirichlet(n, lx) if dirichlet else global_ids(n, lx)
    nu = op.n_unique
    free = ids >= 0
    bl, xl = b.cpu().numpy(), x.cpu().numpy()
    cg.close()
    op.gs.close()
    del op, b, x
    assert np.all(bl[~free] == 0.0) and np.all(xl[~free] == 0.0)
    bg = np.zeros(nu)
    xg = np.zeros(nu)
    bg[ids[free]] = bl[free]
    xg[ids[free]] = xl[free]
    big = _bigbox(dirichlet, h2)
    assert big.nu == nu
    bref = big.fourier_rhs(k, a, ph, const=0.0 if h2 is None else 1.0)
    assert np.max(np.abs(bg - bref)) <= 1e-12 * np.max(np.abs(bref))
    rel = np.linalg.norm(bref - big.apply(xg)) / np.linalg.norm(bref)
    assert rel <= 1.1e-10, rel
    if not dirichlet and h2 is None:
        assert abs(xg.sum()) <= 1e-10 * np.abs(xg).sum()
    name = "dirichlet" if dirichlet else ("periodic" if h2 is None else "helmholtz")
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", f"solve_{name}_n32_lx8.json")))
    gid = np.array(gold["sample_ids"])
    np.testing.assert_allclose(bref[gid], gold["b_sample"], rtol=0, atol=1e-14 * np.max(np.abs(bref)))
    xs = np.array(gold["x_sample"])
    err = np.linalg.norm(xg[gid] - xs) / np.linalg.norm(xs)
    print(f"{name} {prec} mode {mode}: {st['iterations']} its, relres {rel:.3e}, err vs oracle {err:.3e}")
    assert err <= FULL_SIZE_ERR, err


def test_ax_gs_full_size_against_c_oracle(sem_ctx):
    """gs(Ax(Q u_G)) on the 32^3 box at lx = 8 (amplitude 0.1, h1 ~ U[0.5, 2] per
    unique node, u_G ~ N(0,1)), the sizes of the throughput benchmark, equals
    Q (A_G u_G) of the plain-C oracle at every local node to 1e-12."""
    from oracle import cref
    n, lx, amp = 32, 8, 0.1
    nu = (n * (lx - 1)) ** 3
    h1u = synth.unique_uniform(nu, 0.5, 2.0, 1)
    uu = synth.unique_normal(nu, 0)
    op = BoxOperator(sem_ctx, n, lx, amp, h1_unique=h1u, keep_coords=False)
    u = op.scatter(uu)
    w = torch.empty_like(u)
    op.apply(w, u)
    torch.cuda.synchronize()
    wl = w.cpu().numpy()
    ids = op.ids.cpu().numpy()
    op.gs.close()
    del op, u, w
    _BIG.clear()
    big = cref.BigBox(n, lx, amp, h1_unique=h1u)
    ref = big.apply(uu)[ids]
    del big
    err = np.max(np.abs(wl - ref)) / np.max(np.abs(ref))
    assert err <= 1e-12, err


@pytest.mark.parametrize("dirichlet", [False, True])
@pytest.mark.parametrize("prec,mode", [("f64", 0), ("f32", 0), ("f32", 1), ("bf16", 1)])
def test_helmholtz_solve(sem_ctx, prec, mode, dirichlet):
    """The Helmholtz operator A + h2 B (h2 = 20, velocity-type solve) on the
    periodic and the Dirichlet box, against the oracle's: no projection, the
    residual recomputed by the oracle, the solution error, float64 iteration
    counts within 2 of the oracle's PCG, and on the periodic box the exact
    balance h2 (Q^T B) . x = sum b (the stiffness annihilates constants)."""
    n, lx, amp, h2 = 3, 8, 0.1, 20.0
    op = BoxOperator(sem_ctx, n, lx, amp, dirichlet=dirichlet)
    ref = BoxProblem(n, lx, amp, dirichlet=dirichlet, h2=h2)
    k, a, ph = synth.fourier_modes(3)
    # plus the constant source f = 1, so that the solution has a clear mean
    b = op.fourier_rhs(k, a, ph, project=False)
    mass = op.bm.clone()
    P.sem_gs(op.gs, mass)
    b += mass
    from oracle.gs import gather
    m = gather(ref.B, ref.ids, ref.nu)
    bref = ref.fourier_rhs(k, a, ph) + m
    free = ref.ids >= 0
    bg = np.zeros(ref.nu)
    bg[ref.ids[free]] = b.cpu().numpy()[free]
    np.testing.assert_allclose(bg, bref, rtol=0, atol=1e-13 * np.abs(bref).max())
    code = {"f64": P.SEM_SOLVE_F64, "f32": P.SEM_SOLVE_F32_IR, "bf16": P.SEM_SOLVE_BF16_IR}[prec]
    cg = op.solver(code, h2b=h2 * op.bm)
    x = torch.empty_like(b)
    rc, st = P.sem_cg_solve(cg, x, b, tol=1e-10, precision=code, ir_mode=mode)
    torch.cuda.synchronize()
    assert rc == P.SEM_OK and st["converged"], st
    xl = x.cpu().numpy()
    xg = np.zeros(ref.nu)
    xg[ref.ids[free]] = xl[free]
    assert np.linalg.norm(bref - ref.apply(xg)) / np.linalg.norm(bref) <= 1.2e-10
    xs, ito, _ = pcg(ref.apply, bref, 1.0 / ref.diagonal(), tol=1e-13, project=False)
    assert np.max(np.abs(xg - xs)) <= 1e-6 * np.max(np.abs(xs))
    if prec == "f64":
        _, ito, _ = pcg(ref.apply, bref, 1.0 / ref.diagonal(), tol=1e-10, project=False)
        assert abs(st["iterations"] - ito) <= 2, (st["iterations"], ito)
    if not dirichlet:
        assert h2 * (m @ xg) == pytest.approx(bref.sum(), rel=1e-7)
        assert m @ xg > 0.5 / h2           # the constant source's share: nothing projected
    cg.close()
    op.gs.close()


def test_helmholtz_flexible_cg_with_block(sem_ctx):
    """Flexible CG with the classical element block on the Helmholtz operator
    (float32 residual replacement): converges to the oracle's solution."""
    from paper_2506_20994_amd import learned as LR
    n, lx, amp, h2 = 4, 8, 0.1, 20.0
    op = BoxOperator(sem_ctx, n, lx, amp)
    ref = BoxProblem(n, lx, amp, h2=h2)
    k, a, ph = synth.fourier_modes(3)
    b = op.fourier_rhs(k, a, ph, project=False)
    bref = ref.fourier_rhs(k, a, ph)
    lp = P.sem_lp_create(sem_ctx, op.nel)
    op.bind(lp)
    P.sem_lp_set_block(lp, LR.reference_block(sem_ctx))
    cg = op.solver(P.SEM_SOLVE_F32_IR, h2b=h2 * op.bm, learned=lp)
    x = torch.empty_like(b)
    rc, st = P.sem_cg_solve(cg, x, b, tol=1e-10, precision=P.SEM_SOLVE_F32_IR, ir_mode=1, learned=lp)
    torch.cuda.synchronize()
    assert rc == P.SEM_OK and st["converged"] and st["jacobi_steps"] == 0, st
    xg = np.zeros(ref.nu)
    xg[ref.ids.ravel()] = x.cpu().numpy().ravel()
    assert np.linalg.norm(bref - ref.apply(xg)) / np.linalg.norm(bref) <= 1.2e-10
    xs, _, _ = pcg(ref.apply, bref, 1.0 / ref.diagonal(), tol=1e-13, project=False)
    assert np.max(np.abs(xg - xs)) <= 1e-6 * np.max(np.abs(xs))
    cg.close()
    lp.close()
    op.gs.close()



def test_box_64cubed_against_c_oracle(sem_ctx):
    """The full stack at scale (64^3 box, E = 262144, lx = 8, 134M local nodes,
    amplitude 0.15) against the plain-C oracle:
      * geometry: the GPU's factors against the oracle's own, within 1e-10 of
        their maximum (coordinates of size 1 differentiated over elements of
        size 1/64 lose about three digits, and G ~ J^-1 J^-T det J amplifies
        that by the Jacobian's conditioning where the map is strongly bent);
      * operator: gs(Ax(u)) at every local node against the oracle's
        assembled operator on the same factors, within 1e-13 of the node's
        rounding bound (the operator on |u| with |D| and |G| bounds every
        partial sum either side forms);
      * right-hand side at every unique node (1e-11: it carries the geometry's
        rounding through the mass weights);
      * a solve to relres 1e-10 with float32 residual replacement and the
        multigrid V-cycle, its residual 2-norm recomputed by the oracle (with
        the GPU's factors, the operator that was solved) over all 89.9M unique
        nodes (<= 1.1e-10)."""
    from oracle import cref
    from oracle.mesh import global_ids
    n, lx, amp = 64, 8, 0.15
    nu = (n * (lx - 1)) ** 3
    op = BoxOperator(sem_ctx, n, lx, amp)
    k, a, ph = synth.fourier_modes(2)
    b = op.fourier_rhs(k, a, ph)
    op.x = op.y = op.z = None
    uu = synth.unique_normal(nu, 0)
    u = op.scatter(uu)
    w = torch.empty_like(u)
    op.apply(w, u)
    torch.cuda.synchronize()
    wl = w.cpu().numpy()
    del u, w
    mg = op.multigrid(n_coarse=8)
    cg = op.solver(P.SEM_SOLVE_F32_IR, mg=mg)
    x = torch.empty_like(b)
    rc, st = P.sem_cg_solve(cg, x, b, tol=1e-10, precision=P.SEM_SOLVE_F32_IR, ir_mode=1, mg=mg)
    torch.cuda.synchronize()
    assert rc == P.SEM_OK and st["converged"] and st["relres"] <= 1e-10, st
    ids = global_ids(n, lx)
    bg = np.zeros(nu)
    xg = np.zeros(nu)
    bg[ids] = b.cpu().numpy()
    xg[ids] = x.cpu().numpy()
    Gg = [g.cpu().numpy() for g in op.G]
    for h in (cg, mg):
        h.close()
    op.gs.close()
    del op, b, x
    torch.cuda.empty_cache()
    _BIG.clear()
    big = cref.BigBox(n, lx, amp)
    errG = max(float(np.max(np.abs(g - r)) / np.max(np.abs(r))) for g, r in zip(Gg, big.G))
    big.G = None
    ref = cref.apply_assembled(uu, ids, nu, big.Dh, None, Gg)[ids]
    S = cref.gather(cref.ax(np.abs(uu[ids]), np.abs(big.Dh), None, [np.abs(g) for g in Gg]), ids, nu)[ids]
    d = np.abs(wl - ref)
    print(f"64^3: geometry {errG:.2e}; operator max |dw| / max |w| = {np.max(d) / np.max(np.abs(ref)):.2e}, "
          f"max |dw| / bound = {np.max(d / S):.2e}")
    assert errG <= 1e-10
    assert np.max(d / S) <= 1e-13
    del wl, ref, S, d
    bref = big.fourier_rhs(k, a, ph)
    errb = np.max(np.abs(bg - bref)) / np.max(np.abs(bref))
    rel = np.linalg.norm(bg - cref.apply_assembled(xg, ids, nu, big.Dh, None, Gg)) / np.linalg.norm(bg)
    print(f"64^3 lx=8: right-hand side {errb:.2e}; multigrid float32 residual replacement "
          f"{st['iterations']} its, relres {rel:.3e}")
    assert errb <= 1e-11
    assert rel <= 1.1e-10, rel
