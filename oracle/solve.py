"""Krylov solves around the operator, on unique (assembled) vectors.

The paper's operator is a component of a Poisson solve (Sec. 3) but the paper
names no solver.  The readings used here:
  * right-hand side: f(x) = sum_m a_m cos(2 pi k_m . x + phi_m) at the physical
    node coordinates, b_G = Q^T (B f) with B the mass weights; the periodic
    operator is singular with null space span{1}, so b_G is made consistent by
    subtracting its mean over unique nodes (1^T b_G = 0, exactly the solvability
    condition);
  * Jacobi-preconditioned CG: the textbook algorithm (Hestenes and Stiefel 1952;
    Saad, Iterative Methods for Sparse Linear Systems, 2nd ed., Alg. 9.1) with
    M = diag(A_G), x_0 = 0, stopped when ||b - A x||_2 <= tol ||b||_2 on the
    recursively updated residual, then the mean of x removed;
  * mixed-precision iterative refinement (Wilkinson; Carson and Higham 2018):
    float64 outer residual r = b - A x, an inner solve of A d = r / ||r|| with a
    reduced-precision operator, x += ||r|| d in float64, until the float64
    relative residual is <= tol;
  * flexible CG with one stored direction (Notay 2000, FCG(1));
  * the Dirichlet box (oracle.mesh.global_ids_dirichlet) has no null space:
    there the right-hand side is not projected and no mean is removed;
  * the Helmholtz problem (velocity-type solves): the operator A + h2 B with a
    constant h2 > 0 and the diagonal mass B (oracle.ax.ax_helmholtz); it is
    positive definite on either box, so nothing is projected either.
Pins: on tiny meshes PCG agrees with the pseudo-inverse solution; FCG with the
Jacobi preconditioner reproduces PCG's iterates; spectral convergence of a
manufactured solution (tests/test_oracle_solve.py).
"""
import numpy as np

from .gll import gll_nodes_weights, deriv_matrix
from .mesh import box_coords, global_ids, n_unique, global_ids_dirichlet, n_unique_dirichlet
from .geometry import geometric_factors
from .ax import ax_einsum, ax_helmholtz
from .gs import gather, scatter, multiplicity
from .assemble import element_diagonal


class BoxProblem:
    """n^3 box, lx points per direction, deformation amplitude a; periodic,
    or with homogeneous Dirichlet conditions on the whole boundary; Poisson,
    or Helmholtz with the constant h2 (operator A + h2 B)."""

    def __init__(self, n, lx, a=0.0, h1_unique=None, dirichlet=False, h2=None):
        self.n, self.lx, self.a = n, lx, a
        self.dirichlet = dirichlet
        # only the periodic Poisson operator is singular (null space: constants)
        self.project = not dirichlet and h2 is None
        xi, self.wgll = gll_nodes_weights(lx - 1)
        self.Dh = deriv_matrix(xi)
        self.dx = np.ascontiguousarray(self.Dh.T)
        self.dxt = np.ascontiguousarray(self.Dh)
        self.coords = box_coords(n, lx, a)
        self.G, self.B, self.detJ = geometric_factors(*self.coords, lx)
        self.ids = global_ids_dirichlet(n, lx) if dirichlet else global_ids(n, lx)
        self.nu = n_unique_dirichlet(n, lx) if dirichlet else n_unique(n, lx)
        self.mult = multiplicity(self.ids, self.nu)
        self.h1 = None if h1_unique is None else scatter(h1_unique, self.ids)
        self.h2b = None if h2 is None else h2 * self.B

    def ax_local(self, u_local):
        d, t = self.dx, self.dxt
        if self.h2b is not None:
            return ax_helmholtz(u_local, d, d, d, t, t, t, self.h1, *self.G, self.h2b)
        return ax_einsum(u_local, d, d, d, t, t, t, self.h1, *self.G)

    def apply(self, x_unique):
        """A_G x: scatter, element operator, gather."""
        return gather(self.ax_local(scatter(x_unique, self.ids)), self.ids, self.nu)

    def diagonal(self):
        d = element_diagonal(self.Dh, self.h1, self.G)
        if self.h2b is not None:
            d = d + self.h2b
        return gather(d, self.ids, self.nu)

    def fourier_rhs(self, k, amp, phase):
        """b_G for f = sum_m amp_m cos(2 pi k_m . x + phase_m), projected to
        1^T b_G = 0 for the periodic Poisson operator."""
        x, y, z = self.coords
        f = np.zeros_like(x)
        for m in range(len(amp)):
            f += amp[m] * np.cos(2.0 * np.pi * (k[m, 0] * x + k[m, 1] * y + k[m, 2] * z)
                                 + phase[m])
        b = gather(self.B * f, self.ids, self.nu)
        return b - b.mean() if self.project else b


def pcg(apply_A, b, Minv, tol=1e-10, maxit=10000, x0=None, project=True):
    """Preconditioned CG; returns (x, iterations, relres history).  With
    `project` (singular periodic operator) the mean of x is removed at the end."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_A(x) if x0 is not None else b.copy()
    bnorm = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / bnorm]
    if hist[-1] <= tol:
        return x, 0, hist
    z = Minv * r
    p = z.copy()
    rz = r @ z
    it = 0
    while it < maxit:
        w = apply_A(p)
        alpha = rz / (p @ w)
        x += alpha * p
        r -= alpha * w
        it += 1
        hist.append(np.linalg.norm(r) / bnorm)
        if hist[-1] <= tol:
            break
        z = Minv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return (x - x.mean() if project else x), it, hist


def fcg1(apply_A, b, precond, tol=1e-10, maxit=10000, project=True):
    """Flexible CG with one stored direction (Notay 2000).  ``precond(r)``
    returns z; it may change from one iteration to the next."""
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = np.linalg.norm(b)
    hist = [1.0]
    p_prev = w_prev = None
    pw_prev = None
    it = 0
    while it < maxit:
        z = precond(r)
        if p_prev is None:
            p = z
        else:
            p = z - ((z @ w_prev) / pw_prev) * p_prev
        w = apply_A(p)
        pw = p @ w
        alpha = (p @ r) / pw
        x += alpha * p
        r -= alpha * w
        it += 1
        hist.append(np.linalg.norm(r) / bnorm)
        if hist[-1] <= tol:
            break
        p_prev, w_prev, pw_prev = p, w, pw
    return (x - x.mean() if project else x), it, hist


def iterative_refinement(apply_A64, b, inner_solve, tol=1e-10, max_outer=50, project=True):
    """Float64 refinement around ``inner_solve(rhat) -> d`` (an approximate
    solution of A d = rhat with ||rhat|| = 1).  Returns (x, outer, relres)."""
    x = np.zeros_like(b)
    bnorm = np.linalg.norm(b)
    r = b.copy()
    relres = [1.0]
    for outer in range(1, max_outer + 1):
        rn = np.linalg.norm(r)
        d = inner_solve(r / rn)
        x += rn * d
        if project:
            x -= x.mean()
        r = b - apply_A64(x)
        if project:
            r -= r.mean()
        relres.append(np.linalg.norm(r) / bnorm)
        if relres[-1] <= tol:
            return x, outer, relres
    return x, max_outer, relres
