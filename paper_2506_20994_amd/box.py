"""Device-resident box problems (periodic, or with homogeneous Dirichlet
conditions on the whole boundary) assembled from the library's set-up calls
(mesh, geometry, gather-scatter plan, multiplicity).  Orchestration and
allocation only; every array is computed by libsem.so kernels."""
import numpy as np
import torch

from . import _binding as B


class BoxOperator:
    """n^3 box, lx GLL points per direction, sine deformation ``amp``;
    periodic, or with ``dirichlet`` u = 0 on the whole boundary (boundary
    nodes carry id -1 and are no unknowns).

    Attributes (all torch tensors on the current GPU, float64 unless noted):
      x, y, z          node coordinates, (nel, lx, lx, lx)
      ids              int64 global ids
      G                (g11, g22, g33, g12, g13, g23)
      bm               mass weights w_i w_j w_k |J|
      dx..dzt          the six lx*lx derivative matrices (Listing 1 layout)
      gs, mult         gather-scatter plan and multiplicities
      h1               None (h1 = 1) or the scattered coefficient
    """

    def __init__(self, ctx, n, lx, amp=0.0, h1_unique=None, keep_coords=True, dirichlet=False):
        self.ctx, self.n, self.lx, self.amp = ctx, n, lx, amp
        self.dirichlet = dirichlet
        self.nel = n ** 3
        self.n_local = self.nel * lx ** 3
        self.n_unique = max(n * (lx - 1) - 1, 0) ** 3 if dirichlet else (n * (lx - 1)) ** 3
        dev = torch.device("cuda", torch.cuda.current_device())
        shp = (self.nel, lx, lx, lx)
        f64 = dict(dtype=torch.float64, device=dev)
        self.x, self.y, self.z = (torch.empty(shp, **f64) for _ in range(3))
        self.ids = torch.empty(shp, dtype=torch.int64, device=dev)
        mesh = B.sem_box_mesh_dirichlet if dirichlet else B.sem_box_mesh
        mesh(ctx, n, lx, amp, self.x, self.y, self.z, self.ids)
        self.G = tuple(torch.empty(shp, **f64) for _ in range(6))
        self.bm = torch.empty(shp, **f64)
        self.min_detj = B.sem_geometry(ctx, self.x, self.y, self.z, self.nel, lx, *self.G, self.bm)
        _, _, dx, dxt = B.sem_gll(lx)
        self.dx = torch.from_numpy(dx).to(dev)
        self.dxt = torch.from_numpy(dxt).to(dev)
        self.dy, self.dz = self.dx.clone(), self.dx.clone()
        self.dyt, self.dzt = self.dxt.clone(), self.dxt.clone()
        torch.cuda.current_stream().synchronize()
        self.gs = B.sem_gs_setup(ctx, self.ids.cpu().numpy())
        self.mult = torch.empty(shp, **f64)
        B.sem_gs_mult(self.gs, self.mult)
        self.h1 = None
        if h1_unique is not None:
            self.h1 = torch.empty(shp, **f64)
            B.sem_scatter(ctx, self.h1, torch.as_tensor(np.asarray(h1_unique), **f64), self.ids)
        if not keep_coords:
            self.x = self.y = self.z = None

    @property
    def D(self):
        return (self.dx, self.dy, self.dz, self.dxt, self.dyt, self.dzt)

    def scatter(self, u_unique, dtype=torch.float64):
        out = torch.empty((self.nel, self.lx, self.lx, self.lx), dtype=dtype, device=self.ids.device)
        B.sem_scatter(self.ctx, out, torch.as_tensor(np.asarray(u_unique), dtype=dtype,
                                                     device=self.ids.device), self.ids)
        return out

    def ax(self, w, u):
        B.sem_ax(self.ctx, w, u, *self.D, self.h1, *self.G, self.nel, self.lx)

    def apply(self, w, u):
        """w = gs(Ax(u)): the assembled operator in the local layout."""
        self.ax(w, u)
        B.sem_gs(self.gs, w)

    def fourier_rhs(self, k, amp, phase, project=None):
        """Continuous right-hand side b = Q Q^T (B f) for the Fourier sum f at
        the node coordinates, minus its mean when ``project`` (default: on the
        periodic box, for the singular Poisson operator; pass False for a
        Helmholtz solve).  Needs keep_coords=True."""
        b = torch.empty_like(self.bm)
        B.sem_fourier(self.ctx, b, self.x, self.y, self.z, self.bm, k, amp, phase)
        B.sem_gs(self.gs, b)
        if (not self.dirichlet) if project is None else project:
            B.sem_remove_mean(self.gs, b)
        return b

    def solver(self, precision=0, h2b=None, **opts):
        """A solver for this operator; with ``h2b`` (h2 * bm, local layout) the
        Helmholtz operator A + h2 B."""
        return B.sem_cg_setup(self.ctx, self.gs, self.D, self.h1, self.G, self.nel, self.lx,
                              h2b=h2b, precision=precision, **opts)

    def bind(self, lp):
        """Bind a learned preconditioner to this operator."""
        B.sem_lp_bind(lp, self.D, self.h1, self.G, self.nel, self.lx, self.gs)

    def multigrid(self, h2=0.0, **opts):
        """The multigrid V-cycle of this box's operator (h1 = 1; with h2 > 0 the
        Helmholtz operator A + h2 B).  opts: see SemMgOpts."""
        h2b = h2 * self.bm if h2 > 0 else None
        return B.sem_mg_create(self.ctx, self.gs, self.D, self.G, self.nel, self.lx, self.n, self.amp,
                               dirichlet=self.dirichlet, h2=h2, h2b=h2b, **opts)
