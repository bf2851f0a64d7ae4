"""Multigrid preconditioner for the box solves: one symmetric V-cycle over a
hierarchy of re-discretised box operators with Chebyshev-Jacobi smoothing.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper's Poisson solve (Sec. 3) is preconditioned here by the classical
spectral-element preconditioner, the comparison the learned one needs: the
paper itself stops at the operator and its gather-scatter (Sec. 2.1, 4.2).
Sources: p-multigrid for spectral elements (Ronquist and Patera 1987),
Chebyshev polynomial smoothing (Adams, Brezina, Hu and Tuminaro 2003), the
Chebyshev semi-iteration (Saad 2003, Alg. 12.1), trilinear h-coarsening.
Readings taken (none is fixed by the paper):
  * levels: the fine (n, lx), then lx -> max(2, lx // 2) on the same elements
    down to lx = 2, then the lx = 2 box of n^3 elements -> (n/2)^3 while n is
    even and n/2 >= n_coarse; the last level is solved exactly;
  * each level's operator is re-discretised on the same deformed box
    (oracle.solve.BoxProblem at that n and lx; h1 = 1, Helmholtz h2 B_l);
    where a coarse level's isoparametric geometry folds (det J <= 0 at some
    node: coarse trilinear elements resolve the sine map poorly, e.g. at
    amplitude 0.15), that level takes the amplitude halved until it does not
    (``level_amplitude``) -- any positive definite coarse operator keeps the
    V-cycle a valid preconditioner;
  * transfer P: the coarse level's continuous field evaluated at the fine
    level's nodes -- p: the coarse Lagrange basis at the fine GLL points of
    the same element; h: the parent element's trilinear basis at the child's
    vertices (reference coordinate -1 + parity + i); restriction P^T;
  * smoother: k steps of the Chebyshev semi-iteration in D^-1 A (D the
    assembled diagonal) for the interval [lo lmax, hi lmax], lmax the largest
    eigenvalue of D^-1 A (exact here; estimated by the library);
  * Galerkin option: every lx = 2 level below the first takes A_c = P^T A_f P
    (A_f the level above it, with its mass term) instead of a re-discretised
    operator, so it needs no geometry of its own (its amplitude is reported as
    0); on strongly deformed boxes this keeps the coarse correction an
    A-orthogonal projection where the halved-amplitude coarse boxes of the
    re-discretised hierarchy approximate the operator poorly (Galerkin coarse
    operators: Trottenberg, Oosterlee and Schueller 2001);
  * coarsest level: (A + c 1 1^T)^-1 on the singular periodic box (c = mean
    diagonal / n_unique; on mean-free right-hand sides this is the
    pseudo-inverse), A^-1 otherwise;
  * V-cycle(b): x = S(b, 0); x += P V(P^T (b - A x)); x = S(b, x).
Pins (tests/test_oracle_mg.py): P reproduces coarse polynomials (p) and the
trilinear interpolant at vertices, edge, face and cell midpoints (h); P 1 = 1;
the Chebyshev steps equal the closed-form polynomial T_k((theta - D^-1 A) /
delta) / T_k(theta / delta) acting on the error; the two-level V-cycle's
error propagator equals S (I - P A_c^-1 P^T A) S from dense algebra; the
V-cycle is a symmetric positive definite preconditioner; preconditioned CG
needs about as many iterations on 8^3 as on 4^3 elements; with Galerkin
levels the two-grid coarse correction I - P A_c^-1 P^T A is idempotent and
A-self-adjoint (it is not with re-discretised levels), constants stay in the
null space of the periodic Poisson levels, and the solve on a folding box
needs fewer iterations than with re-discretised levels.
"""
import numpy as np
import scipy.sparse as sp

from .gll import gll_nodes_weights, lagrange_basis
from .solve import BoxProblem


def level_shapes(n, lx, n_coarse=2):
    """[(n_l, lx_l, kind_of_transfer_to_the_next)], finest first."""
    out = []
    while lx > 2:
        out.append((n, lx, "p"))
        lx = max(2, lx // 2)
    while n % 2 == 0 and n // 2 >= n_coarse:
        out.append((n, 2, "h"))
        n //= 2
    out.append((n, lx, None))
    return out


def level_amplitude(n, lx, a, dirichlet=False, max_halvings=20):
    """The largest a / 2^m (m >= 0) whose box of n^3 elements at lx has det J >
    0 at every node (0 after max_halvings)."""
    from .mesh import box_coords
    from .geometry import geometric_factors
    for _ in range(max_halvings + 1):
        _, _, dj = geometric_factors(*box_coords(n, lx, a), lx)
        if np.min(dj) > 0.0:
            return a
        a *= 0.5
    return 0.0


def p_matrix(lx_f, lx_c):
    """J[i, a] = l_a(xi_i): coarse basis a at fine GLL point i, (lx_f, lx_c)."""
    xf, _ = gll_nodes_weights(lx_f - 1)
    xc, _ = gll_nodes_weights(lx_c - 1)
    return lagrange_basis(xc, xf)


def h_matrix(parity):
    """J_p[i, a] = phi_a(-1 + p + i), phi_0 = (1 - eta) / 2, phi_1 = (1 + eta) / 2."""
    eta = -1.0 + parity + np.arange(2)
    return np.stack([(1 - eta) / 2, (1 + eta) / 2], axis=1)


def prolongation(fine, coarse, kind):
    """Sparse P (fine unique x coarse unique).  fine, coarse: BoxProblem."""
    nf = fine.n
    P = {}
    for e in range(nf ** 3):
        ex, ey, ez = e % nf, (e // nf) % nf, e // (nf * nf)
        if kind == "p":
            E = e
            Jx = Jy = Jz = p_matrix(fine.lx, coarse.lx)
        else:
            nc = coarse.n
            E = ex // 2 + nc * (ey // 2 + nc * (ez // 2))
            Jx, Jy, Jz = h_matrix(ex % 2), h_matrix(ey % 2), h_matrix(ez % 2)
        ids_f, ids_c = fine.ids[e], coarse.ids[E]
        for k, j, i in np.ndindex(*ids_f.shape):
            f = ids_f[k, j, i]
            if f < 0:
                continue
            for c, b, a in np.ndindex(*ids_c.shape):
                g = ids_c[c, b, a]
                w = Jz[k, c] * Jy[j, b] * Jx[i, a]
                if g < 0 or w == 0.0:
                    continue
                if (f, g) in P:     # the same interpolant seen from another element
                    assert abs(P[f, g] - w) <= 1e-13, (f, g, P[f, g], w)
                P[f, g] = w
    keys = np.array(list(P.keys()), dtype=np.int64).reshape(-1, 2)
    vals = np.array(list(P.values()))
    return sp.csr_matrix((vals, (keys[:, 0], keys[:, 1])), shape=(fine.nu, coarse.nu))


def chebyshev(apply_A, dinv, b, x, k, lo, hi):
    """k steps of the Chebyshev semi-iteration for A x = b, preconditioned by
    D^-1 (dinv), for the eigenvalue interval [lo, hi] of D^-1 A, from x (None:
    0).  theta = (hi + lo) / 2, delta = (hi - lo) / 2, sigma = theta / delta;
    d_0 = D^-1 r_0 / theta; rho_0 = 1 / sigma; rho_m = 1 / (2 sigma - rho_{m-1}),
    d_m = rho_m rho_{m-1} d_{m-1} + (2 rho_m / delta) D^-1 r_m; x += d_m."""
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    sigma = theta / delta
    if x is None:
        x = np.zeros_like(b)
        r = b.copy()
    else:
        x = x.copy()
        r = b - apply_A(x)
    rho = 1.0 / sigma
    d = dinv * r / theta
    x += d
    for _ in range(1, k):
        r = r - apply_A(d)
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (dinv * r)
        rho = rho_new
        x += d
    return x


class Hierarchy:
    """Levels of the box (n, lx, amplitude a; periodic or Dirichlet; h2 for
    the Helmholtz form) with their assembled matrices, diagonals, transfers
    and the exact lmax of D^-1 A (replace by ``set_lmax`` to reproduce a
    caller's estimates).  galerkin: the lx = 2 levels below the first are
    P^T A P of the level above."""

    def __init__(self, n, lx, a, dirichlet=False, h2=None, n_coarse=2, degree=2, lo=0.3, hi=1.1,
                 galerkin=False):
        from .assemble import assembled_matrix
        self.shapes = level_shapes(n, lx, n_coarse)
        self.degree, self.lo, self.hi = degree, lo, hi
        self.boxes, self.A, self.dinv, self.P, self.lmax, self.amps = [], [], [], [], [], []
        # Galerkin levels: every lx = 2 level below the first (no geometry: amplitude 0)
        self.galerkin = [galerkin and q > 0 and lxl == 2 for q, (_, lxl, _) in enumerate(self.shapes)]
        for q, (nl, lxl, _) in enumerate(self.shapes):
            if self.galerkin[q]:
                al = 0.0
            else:
                al = a if q == 0 else level_amplitude(nl, lxl, a, dirichlet)
            self.amps.append(al)
            self.boxes.append(BoxProblem(nl, lxl, al, dirichlet=dirichlet, h2=h2))
        for q, (_, _, kind) in enumerate(self.shapes[:-1]):
            self.P.append(prolongation(self.boxes[q], self.boxes[q + 1], kind))
        for q, B in enumerate(self.boxes):
            if self.galerkin[q]:
                A = self.P[q - 1].T @ self.A[q - 1] @ self.P[q - 1]
            else:
                A = assembled_matrix(B.Dh, None, B.G, B.ids, B.nu)
                if h2 is not None:
                    from .gs import gather
                    A = A + sp.diags(gather(h2 * B.B, B.ids, B.nu))
            self.A.append(A.tocsr())
            self.dinv.append(1.0 / A.diagonal())
        for q in range(len(self.shapes) - 1):
            Dm = sp.diags(np.sqrt(self.dinv[q]))
            M = Dm @ self.A[q] @ Dm
            if M.shape[0] <= 3000:
                self.lmax.append(float(np.linalg.eigvalsh(M.toarray())[-1]))
            else:                      # Lanczos, converged to rounding
                from scipy.sparse.linalg import eigsh
                self.lmax.append(float(eigsh(M, k=1, which="LA", tol=1e-12)[0][0]))
        Ac = self.A[-1].toarray()
        self.singular = self.boxes[-1].project
        if self.singular:
            nc = Ac.shape[0]
            Ac = Ac + np.mean(np.diag(Ac)) / nc * np.ones((nc, nc))
        self.coarse_inv = np.linalg.inv(Ac)

    def set_lmax(self, lmax):
        self.lmax = [float(v) for v in lmax]

    def smooth(self, q, b, x):
        lm = self.lmax[q]
        return chebyshev(lambda v: self.A[q] @ v, self.dinv[q], b, x, self.degree, self.lo * lm, self.hi * lm)

    def vcycle(self, b, q=0):
        """z = V(b) on level q (unique vectors of that level's box)."""
        if q == len(self.shapes) - 1:
            return self.coarse_inv @ b
        x = self.smooth(q, b, None)
        r = b - self.A[q] @ x
        x = x + self.P[q] @ self.vcycle(self.P[q].T @ r, q + 1)
        return self.smooth(q, b, x)

    def matrix(self):
        """The V-cycle as a dense matrix (columns V(e_j)) on the finest level."""
        nu = self.boxes[0].nu
        return np.stack([self.vcycle(np.eye(nu)[j]) for j in range(nu)], axis=1)
