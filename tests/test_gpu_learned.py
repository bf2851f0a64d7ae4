"""GPU kernels of the learned preconditioner against the FP64 oracle
(oracle/mlp.py): forward, gradients, Adam, features, apply; training
determinism and checkpoint/resume; flexible CG with its Jacobi fallbacks."""
import numpy as np
import pytest
import torch

import synth
from oracle import mlp
from oracle.quant import to_bf16
from oracle.mesh import global_ids
from oracle.solve import BoxProblem, pcg
from tests.helpers import to_dev

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2506_20994_amd")
from paper_2506_20994_amd.box import BoxOperator  # noqa: E402

GRAD_TOL = 2e-2    # normwise, against the unquantised oracle: bf16 operands with float32 accumulation
# Element-wise bounds against the oracle's bfloat16-storage emulation
# (oracle/mlp.py *_bf16: the same roundings, products summed exactly), each as
# max |got - ref| / max |ref| over the compared array:
#  * EW_BLOCK: every rounding to bfloat16 is decided from the same float32
#    value on both sides (a given float32 block, S r formed in float32), so only
#    the float32 accumulation order of the 512-term products differs
#    (~sqrt(512) 2^-24 relative to the output: 1e-6); bound 1e-4.
#  * EW_NET: the kernels round float32 sums to bfloat16 (hidden activations,
#    the folded block, back-propagated errors, S r / s_e), the oracle exact
#    sums.  A value within a float32 rounding error (~1e-6) of a bfloat16
#    rounding boundary rounds to the neighbouring bfloat16 number on one side
#    only (a fraction ~5e-4 of the values); each such value moves the outputs it
#    feeds by one bfloat16 ulp times its weight, 2^-8 / sqrt(fan-in) ~ 2e-4 of
#    max |y| for fan-ins of 256 to 518; bound 2e-3.
EW_BLOCK = 1e-4
EW_NET = 2e-3


def _ew(got, ref):
    """max |got - ref| / max |ref|, element by element"""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


def _nrm(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _params(seed, bias_scale=0.1):
    p = synth.mlp_init(seed)
    r = synth.rng(seed + 1)
    return [q if q.ndim == 2 else bias_scale * r.standard_normal(q.shape) for q in p]


def _load(lp, params):
    for s, q in enumerate(params):
        P.sem_lp_set(lp, s, q.astype(np.float32))


def _inputs(B, seed):
    r = synth.rng(seed)
    X = r.standard_normal((B, 518))
    X[:, :512] /= np.linalg.norm(X[:, :512], axis=1, keepdims=True)
    Xq = to_bf16(X)
    Xpad = np.zeros((B, 528), dtype=np.float32)
    Xpad[:, :518] = Xq
    T = r.standard_normal((B, 512)) * 0.1
    return Xq, torch.from_numpy(Xpad).to(torch.bfloat16).cuda(), T


def _qparams(params):
    return [to_bf16(q) if q.ndim == 2 else q.astype(np.float32).astype(np.float64) for q in params]


def _f32(params):
    """the float32 master copy the library holds"""
    return [q.astype(np.float32).astype(np.float64) for q in params]


def test_forward(sem_ctx):
    B = 300
    params = _params(10)
    lp = P.sem_lp_create(sem_ctx, 512)
    _load(lp, params)
    Xq, Xd, _ = _inputs(B, 11)
    Y = torch.empty((B, 512), dtype=torch.float32, device="cuda")
    P.sem_lp_forward(lp, Xd, Y)
    torch.cuda.synchronize()
    ref = mlp.forward(_qparams(params), Xq)[2]
    assert _nrm(Y.cpu().numpy(), ref) <= GRAD_TOL
    refq = mlp.forward_bf16(_f32(params), Xq)[2]
    assert _ew(Y.cpu().numpy(), refq) <= EW_NET, _ew(Y.cpu().numpy(), refq)
    lp.close()


def test_gradients(sem_ctx):
    B = 256
    params = _params(20)
    lp = P.sem_lp_create(sem_ctx, B)
    _load(lp, params)
    Xq, Xd, T = _inputs(B, 21)
    loss = P.sem_lp_gradients(lp, Xd, to_dev(T.astype(np.float32)))
    l_ref, g_ref = mlp.backward(_qparams(params), Xq, T)
    assert abs(loss - l_ref) <= GRAD_TOL * l_ref
    lq, gq = mlp.backward_bf16(_f32(params), Xq, T.astype(np.float32).astype(np.float64))
    assert abs(loss - lq) <= 1e-4 * lq
    for s in range(6):
        g = P.sem_lp_get(lp, 18 + s)
        assert _nrm(g, g_ref[s]) <= GRAD_TOL, (s, _nrm(g, g_ref[s]))
        assert _ew(g, gq[s]) <= EW_NET, (s, _ew(g, gq[s]))
    lp.close()


def test_gradients_energy_metric(sem_ctx):
    B = 128
    params = _params(22)
    lp = P.sem_lp_create(sem_ctx, B)
    _load(lp, params)
    P.sem_lp_set_metric(lp, 1.0)
    Xq, Xd, T = _inputs(B, 23)
    loss = P.sem_lp_gradients(lp, Xd, to_dev(T.astype(np.float32)))
    K = mlp.reference_metric(8, 1.0)
    l_ref, g_ref = mlp.backward(_qparams(params), Xq, T, K)
    assert abs(loss - l_ref) <= GRAD_TOL * l_ref
    lq, gq = mlp.backward_bf16(_f32(params), Xq, T.astype(np.float32).astype(np.float64), K)
    assert abs(loss - lq) <= 1e-3 * lq
    for s in range(6):
        g = P.sem_lp_get(lp, 18 + s)
        assert _nrm(g, g_ref[s]) <= GRAD_TOL, s
        assert _ew(g, gq[s]) <= EW_NET, (s, _ew(g, gq[s]))
    P.sem_lp_set_metric(lp, -1.0)        # back to the mean squared error
    loss2 = P.sem_lp_gradients(lp, Xd, to_dev(T.astype(np.float32)))
    assert abs(loss2 - mlp.loss(_qparams(params), Xq, T)) <= GRAD_TOL * loss2
    lp.close()


def test_gradients_linear_form(sem_ctx):
    B = 128
    params = _params(24)
    lp = P.sem_lp_create(sem_ctx, B)
    _load(lp, params)
    P.sem_lp_set_linear(lp, 1)
    Xq, Xd, T = _inputs(B, 25)
    loss = P.sem_lp_gradients(lp, Xd, to_dev(T.astype(np.float32)))
    l_ref, g_ref = mlp.backward(_qparams(params), Xq, T, linear=True)
    assert abs(loss - l_ref) <= GRAD_TOL * l_ref
    lq, gq = mlp.backward_bf16(_f32(params), Xq, T.astype(np.float32).astype(np.float64), linear=True)
    assert abs(loss - lq) <= 1e-4 * lq
    for s in (0, 2, 4):
        g = P.sem_lp_get(lp, 18 + s)
        assert _nrm(g, g_ref[s]) <= GRAD_TOL, s
        assert _ew(g, gq[s]) <= EW_NET, (s, _ew(g, gq[s]))
    for s in (1, 3, 5):
        assert np.all(P.sem_lp_get(lp, 18 + s) == 0)
    lp.close()


def test_adam_matches_oracle(sem_ctx):
    lp = P.sem_lp_create(sem_ctx, 8)
    params = _params(30)
    _load(lp, params)
    r = synth.rng(31)
    grads = [r.standard_normal(q.shape) for q in params]
    m = [np.zeros(q.shape) for q in params]
    v = [np.zeros(q.shape) for q in params]
    p_ref = [q.astype(np.float32).astype(np.float64) for q in params]
    for t in range(1, 4):
        for s, g in enumerate(grads):
            P.sem_lp_set(lp, 18 + s, (g * t).astype(np.float32))
        P.sem_lp_adam(lp, lr=1e-2)
        p_ref, m, v = mlp.adam_step(p_ref, [g * t for g in grads], m, v, t, lr=1e-2)
    assert P.sem_lp_get_step(lp) == 3
    for s in range(6):
        got = P.sem_lp_get(lp, s)
        assert np.max(np.abs(got - p_ref[s])) <= 1e-5 * max(1.0, np.max(np.abs(p_ref[s]))), s
        assert _nrm(P.sem_lp_get(lp, 6 + s), m[s]) <= 1e-6
        assert _nrm(P.sem_lp_get(lp, 12 + s), v[s]) <= 1e-6
    lp.close()


def _box_with_lp(ctx, n, amp, seed=40, max_rows=None):
    op = BoxOperator(ctx, n, 8, amp)
    lp = P.sem_lp_create(ctx, max_rows or op.nel)
    op.bind(lp)
    return op, lp


def test_features_and_targets(sem_ctx):
    n, amp = 2, 0.1
    op, lp = _box_with_lp(sem_ctx, n, amp)
    ref = BoxProblem(n, 8, amp)
    rG = synth.unique_normal(ref.nu, 41)
    eG = synth.unique_normal(ref.nu, 42)
    r = op.scatter(rG)
    e = op.scatter(eG)
    els = torch.tensor([3, 0, 7, 5], dtype=torch.int64, device="cuda")
    X = torch.zeros((6, 528), dtype=torch.bfloat16, device="cuda")
    T = torch.zeros((6, 512), dtype=torch.float32, device="cuda")
    P.sem_lp_samples(lp, r, e, els, X, T, 2)
    torch.cuda.synchronize()
    ids = ref.ids
    sel = els.cpu().numpy()
    Xr, s, kap = mlp.features(rG[ids][sel], tuple(g[sel] for g in ref.G), None)
    Tr = mlp.targets(eG[ids][sel], s, kap)
    Xg = X.float().cpu().numpy()
    assert np.all(Xg[:2] == 0) and np.all(Xg[2:, 518:] == 0)
    # bf16 of the same float64 quantity: equal up to one bf16 ulp
    assert np.max(np.abs(Xg[2:, :518] - to_bf16(Xr)) / np.maximum(np.abs(to_bf16(Xr)), 1e-30)) <= 2 ** -7
    np.testing.assert_allclose(T[2:].cpu().numpy(), Tr, rtol=1e-5, atol=1e-7 * np.abs(Tr).max())
    lp.close()


def test_apply_matches_oracle(sem_ctx):
    n, amp = 2, 0.1
    op, lp = _box_with_lp(sem_ctx, n, amp)
    params = _params(50)
    _load(lp, params)
    ref = BoxProblem(n, 8, amp)
    rG = synth.unique_normal(ref.nu, 51)
    for dt in (torch.float64, torch.float32):
        r = op.scatter(rG).to(dt)
        z = torch.empty_like(r)
        P.sem_lp_apply(lp, z, r)
        torch.cuda.synchronize()
        zref = mlp.apply(_qparams(params), rG[ref.ids], ref.G, None, ref.ids, ref.nu)
        assert _nrm(z.double().cpu().numpy(), zref) <= GRAD_TOL
        zq = mlp.apply_bf16(_f32(params), rG[ref.ids], ref.G, None, ref.ids, ref.nu)
        assert _ew(z.double().cpu().numpy(), zq) <= EW_NET, (dt, _ew(z.double().cpu().numpy(), zq))
        zu = np.zeros(ref.nu)
        zu[ref.ids.ravel()] = z.double().cpu().numpy().ravel()
        np.testing.assert_array_equal(z.double().cpu().numpy(), zu[ref.ids])   # continuous
    lp.close()


def test_apply_linear_form_matches_oracle(sem_ctx):
    """Linear form: the symmetric part of the folded matrix applied with
    mult^-1/2 weights on both sides, local layout, float64 and float32."""
    n, amp = 2, 0.1
    op, lp = _box_with_lp(sem_ctx, n, amp)
    params = _params(52)
    P.sem_lp_set_linear(lp, 1)
    _load(lp, params)
    ref = BoxProblem(n, 8, amp)
    rG = synth.unique_normal(ref.nu, 53)
    f32 = [q.astype(np.float32).astype(np.float64) for q in params]
    zref = mlp.apply_linear(f32, rG[ref.ids], ref.G, None, ref.ids, ref.nu)
    zq = mlp.apply_block_bf16(mlp.folded_matrix(f32, 512), rG[ref.ids], ref.G, None, ref.ids, ref.nu,
                              normalise=True)
    for dt in (torch.float64, torch.float32):
        r = op.scatter(rG).to(dt)
        z = torch.empty_like(r)
        P.sem_lp_apply(lp, z, r)
        torch.cuda.synchronize()
        assert _nrm(z.double().cpu().numpy(), zref) <= GRAD_TOL
        assert _ew(z.double().cpu().numpy(), zq) <= EW_NET, (dt, _ew(z.double().cpu().numpy(), zq))
    lp.close()


@pytest.mark.parametrize("n,jb", [(3, False), (5, True)])
def test_apply_unique_linear_form_matches_oracle(sem_ctx, n, jb):
    """Fused linear-form apply on unique-node vectors (27 and 125 elements: a
    partial and a ragged 64-element block), float64 and float32, with and
    without the Jacobi base, against the oracle's symmetric apply."""
    amp = 0.1
    op = BoxOperator(sem_ctx, n, 8, amp)
    lp = P.sem_lp_create(sem_ctx, op.nel)
    P.sem_lp_set_linear(lp, 1)
    P.sem_lp_set_jacobi_base(lp, int(jb))
    op.bind(lp)
    params = _params(54)
    _load(lp, params)
    ref = BoxProblem(n, 8, amp)
    rG = synth.unique_normal(ref.nu, 55)
    f32 = [q.astype(np.float32).astype(np.float64) for q in params]
    zl = mlp.apply_linear(f32, rG[ref.ids], ref.G, None, ref.ids, ref.nu)
    zref = np.zeros(ref.nu)
    zref[ref.ids.ravel()] = zl.ravel()
    zlq = mlp.apply_block_bf16(mlp.folded_matrix(f32, 512), rG[ref.ids], ref.G, None, ref.ids, ref.nu,
                               normalise=False, f32_decisions=True)
    zq = np.zeros(ref.nu)
    zq[ref.ids.ravel()] = zlq.ravel()
    if jb:
        zref += rG / ref.diagonal()
        zq += rG / ref.diagonal()
    # the plan numbers unique nodes in order of first appearance in the local layout
    _, first = np.unique(ref.ids.ravel(), return_index=True)
    plan_of = np.empty(ref.nu, dtype=np.int64)
    plan_of[np.argsort(first)] = np.arange(ref.nu)
    rp = np.empty(ref.nu)
    rp[plan_of] = rG
    for dt in (torch.float64, torch.float32):
        r = torch.from_numpy(rp).to(dt).cuda()
        z = torch.full_like(r, float("nan"))
        P.sem_lp_apply_unique(lp, z, r)
        torch.cuda.synchronize()
        zg = z.double().cpu().numpy()[plan_of]
        assert np.all(np.isfinite(zg))
        assert _nrm(zg, zref) <= GRAD_TOL
        assert _ew(zg, zq) <= EW_NET, (dt, _ew(zg, zq))
    lp.close()
    op.gs.close()


def _train(lp, X, T, steps, seed, B=64):
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    out = []
    for k in range(steps):
        rows = torch.from_numpy(synth.choice(seed + k, X.shape[0], B)).cuda()
        P.sem_lp_train_step(lp, X, T, rows, 1e-3, loss)
        out.append(float(loss))
    return out


def test_training_reduces_loss_and_resumes_bitwise(sem_ctx):
    N = 512
    r = synth.rng(60)
    Xf = np.zeros((N, 528), dtype=np.float32)
    Xf[:, :518] = to_bf16(r.standard_normal((N, 518)) * 0.2)
    A = r.standard_normal((518, 512)) * 0.05
    T = (Xf[:, :518] @ A).astype(np.float32)
    X = torch.from_numpy(Xf).to(torch.bfloat16).cuda()
    Td = to_dev(T)
    params = _params(61)
    lp = P.sem_lp_create(sem_ctx, 64)
    _load(lp, params)
    losses = _train(lp, X, Td, 40, 1000)
    assert np.mean(losses[-5:]) < 0.5 * np.mean(losses[:5])
    # resume: 20 steps, save, reload into a new network, 20 more == 40 straight
    lp2 = P.sem_lp_create(sem_ctx, 64)
    _load(lp2, params)
    _train(lp2, X, Td, 20, 1000)
    saved = [P.sem_lp_get(lp2, s) for s in range(18)]
    step = P.sem_lp_get_step(lp2)
    lp3 = P.sem_lp_create(sem_ctx, 64)
    for s in range(18):
        P.sem_lp_set(lp3, s, saved[s])
    P.sem_lp_set_step(lp3, step)
    _train(lp3, X, Td, 20, 1020)
    for s in range(6):
        np.testing.assert_array_equal(P.sem_lp_get(lp3, s), P.sem_lp_get(lp, s))
    for h in (lp, lp2, lp3):
        h.close()


def test_checkpoint_file_round_trip(sem_ctx, tmp_path):
    """sem_lp_save / sem_lp_load: the form, metric, step, parameters and Adam
    moments come back exactly; training continued from the loaded file equals
    training continued in place; a foreign file is rejected and changes
    nothing."""
    N = 512
    r = synth.rng(62)
    Xf = np.zeros((N, 528), dtype=np.float32)
    Xf[:, :518] = to_bf16(r.standard_normal((N, 518)) * 0.2)
    T = to_dev((Xf[:, :518] @ (r.standard_normal((518, 512)) * 0.05)).astype(np.float32))
    X = torch.from_numpy(Xf).to(torch.bfloat16).cuda()
    lp = P.sem_lp_create(sem_ctx, 64)
    P.sem_lp_set_linear(lp, 1)
    P.sem_lp_set_metric(lp, 1.0)
    _load(lp, _params(63))
    _train(lp, X, T, 10, 2000)
    path = str(tmp_path / "net.semlp")
    P.sem_lp_save(lp, path)
    lp2 = P.sem_lp_create(sem_ctx, 64)
    P.sem_lp_load(lp2, path)
    assert P.sem_lp_get_step(lp2) == P.sem_lp_get_step(lp) == 10
    for s in range(18):
        np.testing.assert_array_equal(P.sem_lp_get(lp2, s), P.sem_lp_get(lp, s))
    _train(lp, X, T, 5, 2100)
    _train(lp2, X, T, 5, 2100)          # same linear form and energy metric, or this would differ
    for s in range(6):
        np.testing.assert_array_equal(P.sem_lp_get(lp2, s), P.sem_lp_get(lp, s))
    bad = tmp_path / "bad.semlp"
    bad.write_bytes(b"SEMLP001" + bytes(16))
    before = P.sem_lp_get(lp2, 0)
    with pytest.raises(P.SemError):
        P.sem_lp_load(lp2, str(bad))
    np.testing.assert_array_equal(P.sem_lp_get(lp2, 0), before)
    for h in (lp, lp2):
        h.close()


@pytest.mark.parametrize("kind", ["nan", "zero"])
def test_fcg_falls_back_to_jacobi(sem_ctx, kind):
    """A network that outputs NaN (or zero) is replaced by Jacobi on every
    iteration: FCG then reproduces Jacobi-PCG and still converges."""
    n, amp = 2, 0.1
    op, lp = _box_with_lp(sem_ctx, n, amp)
    params = _params(70)
    if kind == "nan":
        params[5] = params[5] + np.nan
    else:
        params = [0 * q for q in params]
    _load(lp, params)
    k, a, ph = synth.fourier_modes(2)
    b = op.fourier_rhs(k, a, ph)
    x = torch.empty_like(b)
    cg = op.solver(P.SEM_SOLVE_F64, learned=lp)
    rc, st = P.sem_cg_solve(cg, x, b, tol=1e-10, learned=lp)
    assert st["converged"] and st["relres"] <= 1e-10
    assert st["jacobi_steps"] == st["iterations"]
    cg0 = op.solver(P.SEM_SOLVE_F64)
    x0 = torch.empty_like(b)
    _, st0 = P.sem_cg_solve(cg0, x0, b, tol=1e-10)
    assert abs(st["iterations"] - st0["iterations"]) <= 1
    torch.cuda.synchronize()
    assert float((x - x0).abs().max()) <= 1e-8 * float(x0.abs().max())
    for h in (cg, cg0, lp):
        h.close()


@pytest.mark.parametrize("prec,mode", [(0, 0), (1, 1)])
def test_stagnating_network_switches_to_jacobi(sem_ctx, prec, mode):
    """A network that is accepted on every iteration (r.z > 0) but stalls the
    solve -- the linear form with the all-ones block, a positive semidefinite
    preconditioner of rank <= nel -- trips the stagnation guard: the solve
    switches to Jacobi for good (float64 flexible CG, and float32 residual
    replacement) and converges."""
    n, amp = 3, 0.1
    op, lp = _box_with_lp(sem_ctx, n, amp)
    P.sem_lp_set_linear(lp, 1)
    W1 = np.zeros((256, 518)); W1[0, :512] = 1.0
    W2 = np.zeros((256, 256)); W2[0, 0] = 1.0
    W3 = np.zeros((512, 256)); W3[:, 0] = 1.0
    _load(lp, [W1, np.zeros(256), W2, np.zeros(256), W3, np.zeros(512)])
    k, a, ph = synth.fourier_modes(6)
    b = op.fourier_rhs(k, a, ph)
    x = torch.empty_like(b)
    cg = op.solver(prec, learned=lp)
    rc, st = P.sem_cg_solve(cg, x, b, tol=1e-10, precision=prec, ir_mode=mode, learned=lp, maxit=20000)
    assert st["fell_back"] == 1 and rc == P.SEM_FELL_BACK, st
    assert st["converged"] and st["relres"] <= 1e-10
    for h in (cg, lp):
        h.close()


@pytest.mark.parametrize("prec,linear", [(0, False), (1, False), (0, True), (1, True)])
def test_fcg_untrained_network_converges(sem_ctx, prec, linear):
    n, amp = 3, 0.1
    op, lp = _box_with_lp(sem_ctx, n, amp)
    P.sem_lp_set_linear(lp, int(linear))
    _load(lp, _params(80))
    k, a, ph = synth.fourier_modes(3)
    b = op.fourier_rhs(k, a, ph)
    ref = BoxProblem(n, 8, amp)
    bref = ref.fourier_rhs(k, a, ph)
    x = torch.empty_like(b)
    cg = op.solver(prec, learned=lp)
    rc, st = P.sem_cg_solve(cg, x, b, tol=1e-10, precision=prec, learned=lp, maxit=20000)
    torch.cuda.synchronize()
    assert st["converged"], st
    xg = np.zeros(ref.nu)
    xg[ref.ids.ravel()] = x.cpu().numpy().ravel()
    assert np.linalg.norm(bref - ref.apply(xg)) / np.linalg.norm(bref) <= 1.2e-10
    print(f"untrained FCG prec={prec}: {st}")
    for h in (cg, lp):
        h.close()


def test_pipeline_small(sem_ctx):
    """Snapshot generation from float64 Jacobi-PCG on 4^3 boxes, GPU training,
    and a held-out flexible-CG solve with the trained network: the samples
    match the oracle's features of the same snapshot, training lowers the
    loss, and the solve converges (the gain itself is reported, not asserted:
    it is an empirical property of the trained network)."""
    from paper_2506_20994_amd import learned as LR
    lp = P.sem_lp_create(sem_ctx, 6 ** 3)
    LR.init_network(lp, 7, mu=-1.0, jacobi_base=False)
    X, T, info = LR.generate(sem_ctx, lp, n=4, boxes=3, snapshots=4, elems_per_snapshot=16,
                             seed=300, rhs="noise", include_zero=True)
    assert X.shape == (3 * 4 * 16, 528) and info["boxes"] == 3
    Xf = X.float().cpu().numpy()
    assert np.all(np.isfinite(Xf)) and np.all(Xf[:, 518:] == 0)
    np.testing.assert_allclose(np.sum(Xf[:, :512] ** 2, axis=1), 1.0, rtol=2e-2)
    hist = LR.train(lp, X, T, epochs=30, batch=64, lr=1e-3)
    assert hist[-1] < hist[0]
    op = BoxOperator(sem_ctx, 6, 8, 0.1)
    op.bind(lp)
    k, a, ph = synth.fourier_modes(9)
    b = op.fourier_rhs(k, a, ph)
    x = torch.empty_like(b)
    cg = op.solver(0, learned=lp)
    rc, st = P.sem_cg_solve(cg, x, b, tol=1e-10, learned=lp, maxit=20000)
    assert st["converged"] and st["relres"] <= 1e-10
    cg0 = op.solver(0)
    _, st0 = P.sem_cg_solve(cg0, x, b, tol=1e-10)
    print(f"pipeline: trained FCG {st['iterations']} its ({st['jacobi_steps']} Jacobi, "
          f"fell back {st['fell_back']}) vs Jacobi-PCG {st0['iterations']}")
    for h in (cg, cg0, lp):
        h.close()


@pytest.mark.parametrize("dirichlet", [False, True])
def test_trained_linear_network_beats_jacobi(sem_ctx, dirichlet):
    """What the trained network gains: the linear form trained on the GPU with
    the energy-norm loss on float64 Jacobi-PCG pairs (white-noise right-hand
    sides) from 256 8^3 boxes (131k element rows: with a few tens of thousands
    the learned block stays indefinite) cuts the flexible-CG iteration count on a held-out
    12^3 box well below Jacobi-PCG's, with no Jacobi fallback, in float64 and
    inside float32 residual replacement; on periodic boxes, and trained and
    tested on boxes with u = 0 on the boundary."""
    from paper_2506_20994_amd import learned as LR
    n = 12
    lp = P.sem_lp_create(sem_ctx, n ** 3)
    LR.init_network(lp, 7, mu=1.0, jacobi_base=True, out_scale=0.0, linear=True)
    X, T, info = LR.generate(sem_ctx, lp, n=8, boxes=256, snapshots=1, elems_per_snapshot=512,
                             seed=400, rhs="noise", include_zero=True, dirichlet=dirichlet)
    assert torch.isfinite(T).all()
    hist = LR.train(lp, X, T, epochs=60, batch=1024, lr=3e-4)
    assert hist[-1] < hist[0]
    del X, T
    op = BoxOperator(sem_ctx, n, 8, 0.1, dirichlet=dirichlet)
    op.bind(lp)
    k, a, ph = synth.fourier_modes(5)
    b = op.fourier_rhs(k, a, ph)
    x = torch.empty_like(b)
    cg0 = op.solver(P.SEM_SOLVE_F64)
    _, st0 = P.sem_cg_solve(cg0, x, b, tol=1e-10)
    out = {}
    for name, prec, mode in (("f64", P.SEM_SOLVE_F64, 0), ("f32_rr", P.SEM_SOLVE_F32_IR, 1)):
        cg = op.solver(prec, learned=lp)
        _, st = P.sem_cg_solve(cg, x, b, tol=1e-10, precision=prec, ir_mode=mode, learned=lp)
        assert st["converged"] and st["relres"] <= 1e-10
        assert st["jacobi_steps"] == 0 and not st["fell_back"]
        out[name] = st["iterations"]
        cg.close()
    print(f"dirichlet={dirichlet}: Jacobi-PCG {st0['iterations']} its; learned FCG {out}")
    assert out["f64"] <= 0.6 * st0["iterations"]
    assert out["f32_rr"] <= 0.6 * st0["iterations"]
    for h in (cg0, lp):
        h.close()
    op.gs.close()


def test_apply_unique_linear_full_size_sampled(sem_ctx):
    """The linear-form apply at the benchmark size (32^3 box, lx = 8, 16.8M local
    nodes, the launch configuration of the solves), float64 and float32, with
    the Jacobi base: z at 48 sampled unique nodes against the oracle evaluated
    node by node from the (at most 8) elements containing each node
    (tests/helpers.linear_apply_at_nodes, itself checked against the oracle's
    whole-mesh apply on the CPU)."""
    from oracle.mesh import global_ids
    from tests.helpers import linear_apply_at_nodes
    n, lx, amp = 32, 8, 0.1
    op = BoxOperator(sem_ctx, n, lx, amp, keep_coords=False)
    lp = P.sem_lp_create(sem_ctx, op.nel)
    P.sem_lp_set_linear(lp, 1)
    P.sem_lp_set_jacobi_base(lp, 1)
    op.bind(lp)
    params = _params(56)
    _load(lp, params)
    ids = global_ids(n, lx)
    _, first = np.unique(ids.ravel(), return_index=True)
    gid_of_plan = np.argsort(first)             # plan index -> global id
    nu = len(first)
    r_plan = synth.unique_normal(nu, 57)
    r_glob = np.empty(nu)
    r_glob[gid_of_plan] = r_plan
    f32 = [q.astype(np.float32).astype(np.float64) for q in params]
    samples = synth.choice(58, nu, 48)
    zref = linear_apply_at_nodes(f32, n, lx, amp, ids, r_glob, gid_of_plan[samples], jacobi=True)
    zq = linear_apply_at_nodes(f32, n, lx, amp, ids, r_glob, gid_of_plan[samples], jacobi=True, bf16=True)
    for dt in (torch.float64, torch.float32):
        r = torch.from_numpy(r_plan).to(dt).cuda()
        z = torch.empty_like(r)
        P.sem_lp_apply_unique(lp, z, r)
        torch.cuda.synchronize()
        zs = z.double().cpu().numpy()[samples]
        assert np.all(np.isfinite(zs))
        assert _nrm(zs, zref) <= GRAD_TOL, (dt, _nrm(zs, zref))
        assert _ew(zs, zq) <= EW_NET, (dt, _ew(zs, zq))
    lp.close()
    op.gs.close()


def test_set_block_matches_oracle(sem_ctx):
    """sem_lp_set_block: a given 512 x 512 block, applied by the linear form's
    kernels on unique-node vectors, against the oracle's symmetric block apply."""
    n, amp = 3, 0.1
    op = BoxOperator(sem_ctx, n, 8, amp)
    lp = P.sem_lp_create(sem_ctx, op.nel)
    op.bind(lp)
    W = synth.rng(64).standard_normal((512, 512)) * 0.05
    P.sem_lp_set_block(lp, W)
    ref = BoxProblem(n, 8, amp)
    rG = synth.unique_normal(ref.nu, 65)
    zl = mlp.apply_block(W.astype(np.float32).astype(np.float64), rG[ref.ids], ref.G, None, ref.ids, ref.nu)
    zref = np.zeros(ref.nu)
    zref[ref.ids.ravel()] = zl.ravel()
    _, first = np.unique(ref.ids.ravel(), return_index=True)
    plan_of = np.empty(ref.nu, dtype=np.int64)
    plan_of[np.argsort(first)] = np.arange(ref.nu)
    rp = np.empty(ref.nu)
    rp[plan_of] = rG
    r = torch.from_numpy(rp).cuda()
    z = torch.empty_like(r)
    P.sem_lp_apply_unique(lp, z, r)
    torch.cuda.synchronize()
    assert _nrm(z.cpu().numpy()[plan_of], zref) <= GRAD_TOL
    zlq = mlp.apply_block_bf16(W, rG[ref.ids], ref.G, None, ref.ids, ref.nu, normalise=False,
                               f32_decisions=True)
    zq = np.zeros(ref.nu)
    zq[ref.ids.ravel()] = zlq.ravel()
    assert _ew(z.cpu().numpy()[plan_of], zq) <= EW_BLOCK, _ew(z.cpu().numpy()[plan_of], zq)
    # float32 vectors: S r is formed from float32 r on both sides
    r32 = r.float()
    z32 = torch.empty_like(r32)
    P.sem_lp_apply_unique(lp, z32, r32)
    torch.cuda.synchronize()
    rG32 = rG.astype(np.float32).astype(np.float64)
    zlq = mlp.apply_block_bf16(W, rG32[ref.ids], ref.G, None, ref.ids, ref.nu, normalise=False,
                               f32_decisions=True)
    zq[ref.ids.ravel()] = zlq.ravel()
    assert _ew(z32.double().cpu().numpy()[plan_of], zq) <= EW_BLOCK
    lp.close()
    op.gs.close()


def test_reference_block_preconditioner(sem_ctx):
    """The classical comparison: the kappa-normalised inverse of the assembled
    operator on one undeformed element (additive Schwarz, minimal overlap),
    applied by the same kernels, in flexible CG on a held-out 12^3 box."""
    from paper_2506_20994_amd import learned as LR
    W = LR.reference_block(sem_ctx)
    assert np.allclose(W, W.T, rtol=0, atol=1e-10 * np.abs(W).max())
    assert np.linalg.eigvalsh(W)[0] > 0
    n = 12
    op = BoxOperator(sem_ctx, n, 8, 0.1)
    lp = P.sem_lp_create(sem_ctx, op.nel)
    op.bind(lp)
    P.sem_lp_set_block(lp, W)
    k, a, ph = synth.fourier_modes(5)
    b = op.fourier_rhs(k, a, ph)
    x = torch.empty_like(b)
    cg0 = op.solver(P.SEM_SOLVE_F64)
    _, st0 = P.sem_cg_solve(cg0, x, b, tol=1e-10)
    cg = op.solver(P.SEM_SOLVE_F32_IR, learned=lp)
    _, st = P.sem_cg_solve(cg, x, b, tol=1e-10, precision=P.SEM_SOLVE_F32_IR, ir_mode=1, learned=lp)
    print(f"Jacobi-PCG {st0['iterations']} its; reference block {st['iterations']} its")
    assert st["converged"] and st["jacobi_steps"] == 0 and not st["fell_back"]
    assert st["iterations"] <= 0.6 * st0["iterations"]
    for h in (cg0, cg, lp):
        h.close()
    op.gs.close()


def test_reference_block_matches_oracle(sem_ctx):
    """sem_lp_reference_block against the oracle: kappa times the inverse of
    the principal submatrix of the assembled operator of the undeformed
    periodic 3^3 box on the centre element's nodes (lx = 4 and 8)."""
    from oracle.assemble import assembled_matrix
    for lx in (4, 8):
        ref = BoxProblem(3, lx, 0.0)
        A = assembled_matrix(ref.Dh, None, ref.G, ref.ids, ref.nu).toarray()
        g = ref.ids[13].ravel()
        Ae = A[np.ix_(g, g)]
        kappa = np.mean(ref.G[0][13] + ref.G[1][13] + ref.G[2][13]) / 3.0
        Wref = kappa * np.linalg.inv(Ae)
        W = P.sem_lp_reference_block(sem_ctx, lx)
        assert np.max(np.abs(W - Wref)) <= 1e-9 * np.max(np.abs(Wref)), lx
    with pytest.raises(P.SemError):
        P.sem_lp_reference_block(sem_ctx, 13)


def test_snapshot_pairs(sem_ctx):
    """sem_lp_snapshot forms r = b - gs(A x) (against the oracle's assembled
    operator) and err = x* - x (exactly) on the device, and writes the same
    rows as sem_lp_samples on those fields."""
    n, amp = 2, 0.1
    op, lp = _box_with_lp(sem_ctx, n, amp)
    ref = BoxProblem(n, 8, amp)
    xG, sG, bG = (synth.unique_normal(ref.nu, s) for s in (80, 81, 82))
    x, xs, b = op.scatter(xG), op.scatter(sG), op.scatter(bG)
    r, e = torch.empty_like(x), torch.empty_like(x)
    els = torch.tensor([5, 1, 6], dtype=torch.int64, device="cuda")
    X = torch.zeros((3, 528), dtype=torch.bfloat16, device="cuda")
    T = torch.zeros((3, 512), dtype=torch.float32, device="cuda")
    P.sem_lp_snapshot(lp, x, xs, b, r, e, els, X, T, 0)
    torch.cuda.synchronize()
    rref = (bG - ref.apply(xG))[ref.ids]
    assert np.max(np.abs(r.cpu().numpy() - rref)) <= 1e-12 * np.max(np.abs(rref))
    assert torch.equal(e, xs - x)
    X2, T2 = torch.zeros_like(X), torch.zeros_like(T)
    P.sem_lp_samples(lp, r, e, els, X2, T2, 0)
    torch.cuda.synchronize()
    assert torch.equal(X, X2) and torch.equal(T, T2)
    with pytest.raises(P.SemError):
        P.sem_lp_snapshot(lp, x, xs, b, x, e, els, X, T, 0)          # r_out aliases x
    lp.close()
    op.gs.close()
