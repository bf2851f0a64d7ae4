"""GPU parity of sem_ax against the oracle (element by element)."""
import numpy as np
import pytest
import torch

import synth
from oracle.ax import ax_einsum
from oracle.gll import listing_matrices
from oracle.quant import to_bf16, to_f32
from oracle.mesh import box_coords, global_ids
from oracle.geometry import geometric_factors
from tests.helpers import rel_inf, to_dev

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2506_20994_amd")

TOL64 = 1e-12      # relative inf-norm, float64 operator
TOL_LOW = 1e-5     # float32 / bfloat16 storage vs the input-quantised oracle


def _gpu_D(lx, dtype=torch.float64):
    _, _, dx, dxt = P.sem_gll(lx)
    d = to_dev(dx, dtype)
    t = to_dev(dxt, dtype)
    return (d, d.clone(), d.clone(), t, t.clone(), t.clone())


def _run(ctx, u, G, h1, lx, dtype=torch.float64, out=torch.float64):
    nel = u.shape[0]
    du = to_dev(u, dtype)
    dG = [to_dev(g, dtype) for g in G]
    dh = None if h1 is None else to_dev(h1, dtype)
    w = torch.full(u.shape, float("nan"), dtype=out, device="cuda")
    D = _gpu_D(lx, torch.float64 if dtype == torch.float64 else torch.float32)
    P.sem_ax(ctx, w, du, *D, dh, *dG, nel, lx)
    torch.cuda.synchronize()
    return w.double().cpu().numpy()


@pytest.mark.parametrize("lx", list(range(2, 13)))
@pytest.mark.parametrize("nel", [1, 7, 64])
def test_ax_f64_random(sem_ctx, lx, nel):
    G, h1 = synth.random_spd_factors(nel, lx, 1000 + lx)
    u = synth.local_normal(nel, lx, 2000 + lx)
    got = _run(sem_ctx, u, G, h1, lx)
    ref = ax_einsum(u, *listing_matrices(lx), h1, *G)
    assert rel_inf(got, ref) <= TOL64


@pytest.mark.parametrize("lx", [3, 8, 12])
def test_ax_f64_no_h1(sem_ctx, lx):
    G, _ = synth.random_spd_factors(5, lx, 31)
    u = synth.local_normal(5, lx, 32)
    got = _run(sem_ctx, u, G, None, lx)
    ref = ax_einsum(u, *listing_matrices(lx), None, *G)
    assert rel_inf(got, ref) <= TOL64


def test_ax_detects_swapped_matrices(sem_ctx):
    """The GPU honours each of the six matrices: passing dxt where dx belongs
    must change the result (Dhat is not symmetric)."""
    lx, nel = 6, 4
    G, h1 = synth.random_spd_factors(nel, lx, 41)
    u = synth.local_normal(nel, lx, 42)
    dx, dy, dz, dxt, dyt, dzt = _gpu_D(lx)
    ref = ax_einsum(u, *listing_matrices(lx), h1, *G)
    for swap in range(3):
        D = [dx, dy, dz, dxt, dyt, dzt]
        D[swap], D[swap + 3] = D[swap + 3], D[swap]
        w = torch.empty(u.shape, dtype=torch.float64, device="cuda")
        P.sem_ax(sem_ctx, w, to_dev(u), *D, to_dev(h1), *[to_dev(g) for g in G], nel, lx)
        torch.cuda.synchronize()
        assert rel_inf(w.cpu().numpy(), ref) > 1e-3


@pytest.mark.parametrize("lx", [4, 8, 10])
def test_ax_f32(sem_ctx, lx):
    nel = 33
    G, h1 = synth.random_spd_factors(nel, lx, 51)
    u = synth.local_normal(nel, lx, 52)
    got = _run(sem_ctx, u, G, h1, lx, torch.float32, torch.float32)
    M = [to_f32(m) for m in listing_matrices(lx)]
    ref = ax_einsum(to_f32(u), *M, to_f32(h1), *[to_f32(g) for g in G])
    assert rel_inf(got, ref) <= TOL_LOW
    assert rel_inf(got, ax_einsum(u, *listing_matrices(lx), h1, *G)) <= TOL_LOW


@pytest.mark.parametrize("lx", [4, 8, 10])
def test_ax_bf16(sem_ctx, lx):
    nel = 33
    G, h1 = synth.random_spd_factors(nel, lx, 61)
    u = synth.local_normal(nel, lx, 62)
    du = to_dev(to_bf16(u), torch.bfloat16)
    dG = [to_dev(to_bf16(g), torch.bfloat16) for g in G]
    dh = to_dev(to_bf16(h1), torch.bfloat16)
    w = torch.empty(u.shape, dtype=torch.float32, device="cuda")
    P.sem_ax(sem_ctx, w, du, *_gpu_D(lx, torch.float32), dh, *dG, nel, lx)
    torch.cuda.synchronize()
    M = [to_f32(m) for m in listing_matrices(lx)]
    ref = ax_einsum(to_bf16(u), *M, to_bf16(h1), *[to_bf16(g) for g in G])
    assert rel_inf(w.double().cpu().numpy(), ref) <= TOL_LOW


@pytest.mark.parametrize("lx", [6, 8, 10, 12])
def test_ax_full_size_sampled(sem_ctx, lx):
    """32^3 box (E = 32768), amplitude 0.1, h1 ~ U[0.5, 2] per unique node,
    u ~ N(0, 1) per unique node: the benchmark's workload and launch at lx = 8,
    and the lx = 6, 10, 12 points of the throughput sweep (up to 56.6M local
    nodes).  Sampled elements are recomputed by the oracle from its own
    geometry."""
    from paper_2506_20994_amd.box import BoxOperator
    n, amp = 32, 0.1
    nu = (n * (lx - 1)) ** 3
    h1u = synth.unique_uniform(nu, 0.5, 2.0, 1)
    uu = synth.unique_normal(nu, 0)
    op = BoxOperator(sem_ctx, n, lx, amp, h1_unique=h1u, keep_coords=False)
    u = op.scatter(uu)
    w = torch.empty_like(u)
    op.ax(w, u)
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    els = np.unique(np.concatenate([[0, n ** 3 - 1], rng.integers(0, n ** 3, 48)]))
    G, _, _ = geometric_factors(*box_coords(n, lx, amp, els), lx)
    ids = global_ids(n, lx, els)
    ref = ax_einsum(uu[ids], *listing_matrices(lx), h1u[ids], *G)
    got = w[torch.as_tensor(els, device="cuda")].cpu().numpy()
    assert rel_inf(got, ref) <= TOL64


def test_ax_is_deterministic(sem_ctx):
    lx, nel = 8, 300
    G, h1 = synth.random_spd_factors(nel, lx, 71)
    u = synth.local_normal(nel, lx, 72)
    a = _run(sem_ctx, u, G, h1, lx)
    b = _run(sem_ctx, u, G, h1, lx)
    np.testing.assert_array_equal(a, b)


def test_ax_errors(sem_ctx):
    lx, nel = 4, 2
    u = torch.zeros((nel, lx, lx, lx), dtype=torch.float64, device="cuda")
    G = [torch.zeros_like(u) for _ in range(6)]
    D = _gpu_D(lx)
    w = torch.empty_like(u)
    with pytest.raises(P.SemError) as ei:
        P.sem_ax(sem_ctx, w, u, *D, None, *G, nel, 13)
    assert ei.value.code == P.SEM_EUNSUPPORTED_LX
    with pytest.raises(P.SemError) as ei:
        P.sem_ax(sem_ctx, u, u, *D, None, *G, nel, lx)        # w aliases u
    assert ei.value.code == P.SEM_EINVAL
    with pytest.raises(P.SemError) as ei:
        P.sem_ax(sem_ctx, w, u, *D, None, *G, -1, lx)
    assert ei.value.code == P.SEM_EINVAL
    P.sem_ax(sem_ctx, w, u, *D, None, *G, 0, lx)              # empty: no-op
    with pytest.raises(P.SemError):
        P.sem_ax(sem_ctx, w.float(), u, *D, None, *G, nel, lx, out_dtype=P.SEM_BF16)


def _run_helm(ctx, u, G, h1, hb, lx, dtype=torch.float64, out=torch.float64):
    nel = u.shape[0]
    du = to_dev(u, dtype)
    dG = [to_dev(g, dtype) for g in G]
    dh = None if h1 is None else to_dev(h1, dtype)
    dhb = to_dev(hb, dtype)
    w = torch.full(u.shape, float("nan"), dtype=out, device="cuda")
    D = _gpu_D(lx, torch.float64 if dtype == torch.float64 else torch.float32)
    P.sem_ax_helmholtz(ctx, w, du, *D, dh, *dG, dhb, nel, lx)
    torch.cuda.synchronize()
    return w.double().cpu().numpy()


@pytest.mark.parametrize("lx", [2, 3, 5, 8, 10, 12])
def test_ax_helmholtz(sem_ctx, lx):
    """w = A_e u + h2b u (the lx = 3 one-thread-per-node kernel included), in
    float64 against the oracle to 1e-12, in float32 and bfloat16 storage
    against the input-quantised oracle to 1e-5; the Helmholtz term changes the
    result (it is not dropped)."""
    from oracle.ax import ax_helmholtz
    nel = 7
    G, h1 = synth.random_spd_factors(nel, lx, 3000 + lx)
    u = synth.local_normal(nel, lx, 3100 + lx)
    hb = synth.local_normal(nel, lx, 3200 + lx) ** 2 + 0.1
    M = listing_matrices(lx)
    got = _run_helm(sem_ctx, u, G, h1, hb, lx)
    ref = ax_helmholtz(u, *M, h1, *G, hb)
    assert rel_inf(got, ref) <= TOL64
    assert rel_inf(ax_einsum(u, *M, h1, *G), ref) > 1e3 * TOL64    # the term is not dropped
    for dt, q in ((torch.float32, to_f32), (torch.bfloat16, to_bf16)):
        got = _run_helm(sem_ctx, u, G, h1, hb, lx, dt, torch.float32)
        ref = ax_helmholtz(q(u), *[to_f32(m) for m in M], q(h1), *[q(g) for g in G], q(hb))
        assert rel_inf(got, ref) <= TOL_LOW


def test_ax_helmholtz_full_size_sampled(sem_ctx):
    """32^3 box, lx = 8, amplitude 0.1, h1 and h2 ~ U[0.5, 2] per unique node,
    h2b = h2 * bm (the mass from the library's geometry): sampled elements
    against the oracle's own geometry and mass."""
    from oracle.ax import ax_helmholtz
    from paper_2506_20994_amd.box import BoxOperator
    n, lx, amp = 32, 8, 0.1
    nu = (n * (lx - 1)) ** 3
    h1u = synth.unique_uniform(nu, 0.5, 2.0, 1)
    h2u = synth.unique_uniform(nu, 0.5, 2.0, 3)
    uu = synth.unique_normal(nu, 0)
    op = BoxOperator(sem_ctx, n, lx, amp, h1_unique=h1u, keep_coords=False)
    u = op.scatter(uu)
    h2b = op.scatter(h2u) * op.bm
    w = torch.empty_like(u)
    P.sem_ax_helmholtz(sem_ctx, w, u, *op.D, op.h1, *op.G, h2b, op.nel, lx)
    torch.cuda.synchronize()
    els = np.unique(np.concatenate([[0, n ** 3 - 1], np.random.default_rng(8).integers(0, n ** 3, 32)]))
    G, Bm, _ = geometric_factors(*box_coords(n, lx, amp, els), lx)
    ids = global_ids(n, lx, els)
    ref = ax_helmholtz(uu[ids], *listing_matrices(lx), h1u[ids], *G, h2u[ids] * Bm)
    got = w[torch.as_tensor(els, device="cuda")].cpu().numpy()
    assert rel_inf(got, ref) <= TOL64
    with pytest.raises(P.SemError):
        P.sem_ax_helmholtz(sem_ctx, w, u, *op.D, op.h1, *op.G, None, op.nel, lx)
    op.gs.close()


def _variant_exists(lx, v):
    if v == P.SEM_AX_3D:
        return lx <= 10
    if v == P.SEM_AX_WAVE:
        return lx in (3, 5, 6, 7)
    return True


@pytest.mark.parametrize("lx", list(range(2, 13)))
def test_ax_variants_match_oracle(sem_ctx, lx):
    """Every kernel variant of the float64 operator that exists at lx, with and
    without h1, 1 and 13 elements (partial workgroups of every variant), and
    the Helmholtz form, against the oracle."""
    from oracle.ax import ax_helmholtz
    try:
        for nel in (1, 13):
            G, h1 = synth.random_spd_factors(nel, lx, 3000 + lx)
            u = synth.local_normal(nel, lx, 4000 + lx)
            hb = synth.local_normal(nel, lx, 5000 + lx) ** 2
            ref = ax_einsum(u, *listing_matrices(lx), h1, *G)
            ref0 = ax_einsum(u, *listing_matrices(lx), None, *G)
            refh = ax_helmholtz(u, *listing_matrices(lx), h1, *G, hb)
            for v in range(P.SEM_AX_VARIANTS):
                if not _variant_exists(lx, v):
                    with pytest.raises(P.SemError):
                        P.sem_ax_set_variant(sem_ctx, lx, v)
                    continue
                P.sem_ax_set_variant(sem_ctx, lx, v)
                assert P.sem_ax_get_variant(sem_ctx, lx) == v
                assert rel_inf(_run(sem_ctx, u, G, h1, lx), ref) <= TOL64, (v, nel)
                assert rel_inf(_run(sem_ctx, u, G, None, lx), ref0) <= TOL64, (v, nel)
                w = torch.full(u.shape, float("nan"), dtype=torch.float64, device="cuda")
                P.sem_ax_helmholtz(sem_ctx, w, to_dev(u), *_gpu_D(lx), to_dev(h1), *[to_dev(g) for g in G],
                                   to_dev(hb), nel, lx)
                torch.cuda.synchronize()
                assert rel_inf(w.cpu().numpy(), refh) <= TOL64, (v, nel)
    finally:
        P.sem_ax_set_variant(sem_ctx, lx, P.SEM_AX_DEFAULT)


def test_ax_tune_selects_the_fastest_variant(sem_ctx):
    for lx, missing in ((6, []), (8, [P.SEM_AX_WAVE]), (12, [P.SEM_AX_3D, P.SEM_AX_WAVE])):
        try:
            best, us = P.sem_ax_tune(sem_ctx, lx, 256, reps=3)
            assert len(us) == P.SEM_AX_VARIANTS
            for v in range(P.SEM_AX_VARIANTS):
                assert (us[v] == -1.0) == (v in missing), (lx, v, us)
            assert us[best] == min(t for t in us if t > 0)
            assert P.sem_ax_get_variant(sem_ctx, lx) == best
            # the tuned context still computes the operator
            G, h1 = synth.random_spd_factors(3, lx, 77)
            u = synth.local_normal(3, lx, 78)
            assert rel_inf(_run(sem_ctx, u, G, h1, lx), ax_einsum(u, *listing_matrices(lx), h1, *G)) <= TOL64
        finally:
            P.sem_ax_set_variant(sem_ctx, lx, P.SEM_AX_DEFAULT)
    with pytest.raises(P.SemError):
        P.sem_ax_tune(sem_ctx, 13, 8)


@pytest.mark.parametrize("lx,use_h1", [(5, True), (8, True), (8, False)])
def test_ax_tune_on_the_callers_operands(sem_ctx, lx, use_h1):
    """sem_ax_tune_on times the variants on the caller's own fields (w is
    scratch), selects the fastest, and the tuned operator on those fields
    equals the oracle; an output overlapping an input is refused."""
    nel = 200
    G, h1 = synth.random_spd_factors(nel, lx, 91)
    h1 = h1 if use_h1 else None
    u = synth.local_normal(nel, lx, 92)
    du = to_dev(u, torch.float64)
    dG = [to_dev(g, torch.float64) for g in G]
    dh = None if h1 is None else to_dev(h1, torch.float64)
    D = _gpu_D(lx, torch.float64)
    w = torch.empty_like(du)
    try:
        best, us = P.sem_ax_tune_on(sem_ctx, w, du, *D, dh, *dG, nel, lx, reps=3)
        assert us[best] == min(t for t in us if t > 0)
        assert P.sem_ax_get_variant(sem_ctx, lx) == best
        w.fill_(float("nan"))
        P.sem_ax(sem_ctx, w, du, *D, dh, *dG, nel, lx)
        torch.cuda.synchronize()
        ref = ax_einsum(u, *listing_matrices(lx), h1, *G)
        assert rel_inf(w.cpu().numpy(), ref) <= TOL64
        with pytest.raises(P.SemError) as ei:
            P.sem_ax_tune_on(sem_ctx, du, du, *D, dh, *dG, nel, lx, reps=1)
        assert ei.value.code == P.SEM_EINVAL
    finally:
        P.sem_ax_set_variant(sem_ctx, lx, P.SEM_AX_DEFAULT)
