"""GPU parity of the set-up steps and gather-scatter against the oracle."""
import numpy as np
import pytest
import torch

import synth
from oracle.mesh import box_coords, global_ids, n_unique
from oracle.geometry import geometric_factors
from oracle.gs import gs as gs_ref, multiplicity
from oracle.assemble import element_diagonal, assembled_matrix
from oracle.gll import gll_nodes_weights, deriv_matrix
from oracle.quant import to_bf16
from tests.helpers import rel_inf, to_dev

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2506_20994_amd")
from paper_2506_20994_amd.box import BoxOperator  # noqa: E402


@pytest.mark.parametrize("n,lx,amp", [(1, 2, 0.0), (3, 5, 0.1), (2, 8, 0.15), (2, 12, 0.1)])
def test_mesh_and_geometry(sem_ctx, n, lx, amp):
    op = BoxOperator(sem_ctx, n, lx, amp)
    torch.cuda.synchronize()
    xr, yr, zr = box_coords(n, lx, amp)
    for got, ref in zip((op.x, op.y, op.z), (xr, yr, zr)):
        assert np.max(np.abs(got.cpu().numpy() - ref)) <= 1e-15
    np.testing.assert_array_equal(op.ids.cpu().numpy(), global_ids(n, lx))
    G, B, detJ = geometric_factors(xr, yr, zr, lx)
    for got, ref in zip(op.G, G):
        assert np.max(np.abs(got.cpu().numpy() - ref)) <= 1e-12 * np.max(np.abs(G[0]))
    assert rel_inf(op.bm.cpu().numpy(), B) <= 1e-12
    assert op.min_detj == pytest.approx(detJ.min(), rel=1e-12)


def test_folded_mesh_rejected(sem_ctx):
    with pytest.raises(P.SemError) as ei:
        BoxOperator(sem_ctx, 4, 8, 0.2)
    assert ei.value.code == P.SEM_EGEOMETRY


@pytest.mark.parametrize("n,lx", [(1, 3), (2, 2), (3, 4), (4, 8), (3, 11)])
def test_gs_and_multiplicity(sem_ctx, n, lx):
    op = BoxOperator(sem_ctx, n, lx, 0.0, keep_coords=False)
    ids = global_ids(n, lx)
    nu = n_unique(n, lx)
    assert P.sem_gs_info(op.gs)[0] == nu
    np.testing.assert_array_equal(op.mult.cpu().numpy(), multiplicity(ids, nu))
    u = synth.local_normal(n ** 3, lx, 5)
    du = to_dev(u)
    P.sem_gs(op.gs, du)
    torch.cuda.synchronize()
    assert rel_inf(du.cpu().numpy(), gs_ref(u, ids, nu)) <= 1e-15
    # float32 path
    d32 = to_dev(u, torch.float32)
    P.sem_gs(op.gs, d32)
    ref32 = gs_ref(u.astype(np.float32).astype(np.float64), ids, nu)
    assert rel_inf(d32.double().cpu().numpy(), ref32) <= 1e-6
    # gs(1) = multiplicity exactly
    one = torch.ones_like(du)
    P.sem_gs(op.gs, one)
    np.testing.assert_array_equal(one.cpu().numpy(), multiplicity(ids, nu))


def test_gs_arbitrary_ids(sem_ctx):
    """A general numbering (sparse, unordered ids) takes the relabelling path."""
    r = np.random.default_rng(3)
    ids = r.integers(0, 50, 2000) * 1_000_003 + 17
    plan = P.sem_gs_setup(sem_ctx, ids)
    u = r.standard_normal(2000)
    du = to_dev(u)
    P.sem_gs(plan, du)
    torch.cuda.synchronize()
    _, inv = np.unique(ids, return_inverse=True)
    ref = np.bincount(inv, weights=u)[inv]
    np.testing.assert_allclose(du.cpu().numpy(), ref, rtol=1e-14, atol=1e-14)
    plan.close()


def test_scatter_dtypes(sem_ctx):
    n, lx = 2, 4
    op = BoxOperator(sem_ctx, n, lx, 0.0, keep_coords=False)
    uu = synth.unique_normal(n_unique(n, lx), 9)
    ids = global_ids(n, lx)
    for dt in (torch.float64, torch.float32, torch.bfloat16):
        got = op.scatter(uu.astype(np.float32) if dt != torch.float64 else uu, dtype=dt)
        ref = torch.as_tensor(uu).to(dt).double().numpy()[ids]
        np.testing.assert_array_equal(got.double().cpu().numpy(), ref)


@pytest.mark.parametrize("lx", [2, 5, 8, 12])
def test_element_diagonal(sem_ctx, lx):
    nel = 6
    G, h1 = synth.random_spd_factors(nel, lx, 77)
    d = torch.empty((nel, lx, lx, lx), dtype=torch.float64, device="cuda")
    _, _, dx, _ = P.sem_gll(lx)
    P.sem_ax_diag(sem_ctx, d, to_dev(dx), to_dev(h1), *[to_dev(g) for g in G], nel, lx)
    torch.cuda.synchronize()
    Dh = deriv_matrix(gll_nodes_weights(lx - 1)[0])
    assert rel_inf(d.cpu().numpy(), element_diagonal(Dh, h1, G)) <= 1e-13


def test_fourier_rhs(sem_ctx):
    n, lx, amp = 2, 6, 0.1
    op = BoxOperator(sem_ctx, n, lx, amp)
    k, a, ph = synth.fourier_modes(2)
    f = torch.empty_like(op.x)
    P.sem_fourier(sem_ctx, f, op.x, op.y, op.z, op.bm, k, a, ph)
    torch.cuda.synchronize()
    x, y, z = box_coords(n, lx, amp)
    _, B, _ = geometric_factors(x, y, z, lx)
    ref = np.zeros_like(x)
    for m in range(len(a)):
        ref += a[m] * np.cos(2 * np.pi * (k[m, 0] * x + k[m, 1] * y + k[m, 2] * z) + ph[m])
    assert rel_inf(f.cpu().numpy(), B * ref) <= 1e-12


def test_convert_rounding(sem_ctx):
    r = np.random.default_rng(4)
    a = r.standard_normal(100000) * 10.0 ** r.integers(-6, 6, 100000)
    src = to_dev(a)
    b16 = torch.empty(a.shape, dtype=torch.bfloat16, device="cuda")
    f32 = torch.empty(a.shape, dtype=torch.float32, device="cuda")
    P.sem_convert(sem_ctx, b16, src)
    P.sem_convert(sem_ctx, f32, src)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(b16.double().cpu().numpy(), to_bf16(a))
    np.testing.assert_array_equal(f32.double().cpu().numpy(), a.astype(np.float32).astype(np.float64))


def test_config0_against_assembled_matrix(sem_ctx):
    """4^3 affine periodic box, lx = 8, h1 = 1, u_G ~ N(0, 1) (seed 0): one
    operator application plus gather-scatter equals Q (A_G u_G) with the
    assembled matrix built by the oracle."""
    n, lx = 4, 8
    nu = n_unique(n, lx)
    op = BoxOperator(sem_ctx, n, lx, 0.0, keep_coords=False)
    uu = synth.unique_normal(nu, 0)
    u = op.scatter(uu)
    w = torch.empty_like(u)
    op.apply(w, u)
    torch.cuda.synchronize()
    G, _, _ = geometric_factors(*box_coords(n, lx, 0.0), lx)
    ids = global_ids(n, lx)
    Dh = deriv_matrix(gll_nodes_weights(lx - 1)[0])
    AG = assembled_matrix(Dh, None, G, ids, nu)
    ref = (AG @ uu)[ids]
    assert rel_inf(w.cpu().numpy(), ref) <= 1e-12


@pytest.mark.parametrize("amp", [0.0, 0.1])
def test_config0_dirichlet_against_assembled_matrix(sem_ctx, amp):
    """The 4^3 box with u = 0 on the boundary (lx = 8, h1 = 1): one operator
    application plus the masked gather-scatter equals Q (A_G u_G) with the
    oracle's masked assembled matrix (the natural-boundary matrix with the
    boundary rows and columns deleted), and 0 on the Dirichlet nodes."""
    from oracle.mesh import global_ids_dirichlet, n_unique_dirichlet
    from oracle.gs import scatter
    n, lx = 4, 8
    nu = n_unique_dirichlet(n, lx)
    op = BoxOperator(sem_ctx, n, lx, amp, keep_coords=False, dirichlet=True)
    uu = synth.unique_normal(nu, 0)
    u = op.scatter(uu)
    w = torch.full_like(u, float("nan"))
    op.apply(w, u)
    torch.cuda.synchronize()
    G, _, _ = geometric_factors(*box_coords(n, lx, amp), lx)
    ids = global_ids_dirichlet(n, lx)
    Dh = deriv_matrix(gll_nodes_weights(lx - 1)[0])
    AG = assembled_matrix(Dh, None, G, ids, nu)
    ref = scatter(AG @ uu, ids)
    wl = w.cpu().numpy()
    assert np.all(wl[ids < 0] == 0.0)
    assert rel_inf(wl, ref) <= 1e-12
    op.gs.close()
