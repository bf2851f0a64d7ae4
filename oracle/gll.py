"""Gauss-Lobatto-Legendre points, weights, Lagrange basis and derivative matrix.

Paper Sec. 3 (Eq. 2): the basis is the N-th order Lagrange interpolant through
the N+1 GLL points of [-1, 1].  Eq. 2 is printed garbled (a derivative and a
parenthesis are lost); the reading used here is the standard one,
    l_i(xi) = (xi^2 - 1) L_N'(xi) / (N (N+1) L_N(xi_i) (xi - xi_i)),
which satisfies l_i(xi_j) = delta_ij.

Pins (tests/test_oracle_gll.py): closed-form nodes and weights for N = 2, 3, 4;
tabulated N = 7 nodes (tests/golden/gll_n7.txt); sum of weights = 2; exact
quadrature to degree 2N - 1; D applied to 1 and to xi; exactness of D on
polynomials of degree <= N; corner entries -N(N+1)/4 and N(N+1)/4.
"""
import numpy as np


def legendre(n, x):
    """(L_n(x), L_{n-1}(x)) by the three-term recurrence
    (m+1) L_{m+1} = (2m+1) x L_m - m L_{m-1}."""
    x = np.asarray(x, dtype=np.float64)
    p_prev = np.ones_like(x)
    if n == 0:
        return p_prev, np.zeros_like(x)
    p = x.copy()
    for m in range(1, n):
        p_prev, p = p, ((2 * m + 1) * x * p - m * p_prev) / (m + 1)
    return p, p_prev


def legendre_derivs(n, x):
    """L_n, L_n' and L_n'' at interior points |x| < 1.

    L_n' = n (x L_n - L_{n-1}) / (x^2 - 1); L_n'' from Legendre's equation
    (1 - x^2) L'' - 2 x L' + n (n+1) L = 0.
    """
    p, pm1 = legendre(n, x)
    dp = n * (x * p - pm1) / (x * x - 1.0)
    d2p = (2.0 * x * dp - n * (n + 1) * p) / (1.0 - x * x)
    return p, dp, d2p


def gll_nodes_weights(N):
    """GLL nodes xi_0 = -1 < ... < xi_N = 1 and weights for order N >= 1.

    Interior nodes are the roots of L_N', found by Newton's method from the
    Chebyshev-Gauss-Lobatto guesses -cos(pi i / N), then symmetrised.
    Weights w_i = 2 / (N (N+1) L_N(xi_i)^2).
    """
    if N < 1:
        raise ValueError("N must be >= 1")
    xi = -np.cos(np.pi * np.arange(N + 1) / N)
    xi[0], xi[N] = -1.0, 1.0
    if N >= 2:
        x = xi[1:N].copy()
        for _ in range(100):
            _, dp, d2p = legendre_derivs(N, x)
            dx = dp / d2p
            x -= dx
            if np.max(np.abs(dx)) < 1e-16:
                break
        # one more step to settle on the root after the stopping test
        _, dp, d2p = legendre_derivs(N, x)
        x -= dp / d2p
        xi[1:N] = x
    xi = 0.5 * (xi - xi[::-1])          # exact antisymmetry xi_{N-i} = -xi_i
    if N % 2 == 0:
        xi[N // 2] = 0.0
    LN, _ = legendre(N, xi)
    w = 2.0 / (N * (N + 1) * LN * LN)
    return xi, w


def lagrange_basis(xi_nodes, x):
    """Values l_i(x) of the Lagrange interpolants through ``xi_nodes`` (Eq. 2
    read as above), shape (len(x), N+1), via the product formula."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(xi_nodes)
    out = np.ones((len(x), n))
    for i in range(n):
        for m in range(n):
            if m != i:
                out[:, i] *= (x - xi_nodes[m]) / (xi_nodes[i] - xi_nodes[m])
    return out


def lagrange_eq2(N, xi_nodes, x):
    """l_i(x) from the closed form of Eq. 2 (read as in the module docstring),
    for x not equal to a node.  Shape (len(x), N+1)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    p, pm1 = legendre(N, x)
    dp = N * (x * p - pm1) / (x * x - 1.0)
    LNi, _ = legendre(N, xi_nodes)
    return ((x * x - 1.0)[:, None] * dp[:, None]
            / (N * (N + 1) * LNi[None, :] * (x[:, None] - xi_nodes[None, :])))


def deriv_matrix(xi):
    """Dhat[i, l] = l_l'(xi_i): derivative at node i of the l-th basis function.

    Off-diagonal: L_N(xi_i) / (L_N(xi_l) (xi_i - xi_l)); diagonal from the
    row-sum rule Dhat[i, i] = -sum_{l != i} Dhat[i, l] (derivative of a
    constant vanishes).
    """
    N = len(xi) - 1
    LN, _ = legendre(N, xi)
    D = np.zeros((N + 1, N + 1))
    for i in range(N + 1):
        for l in range(N + 1):
            if i != l:
                D[i, l] = LN[i] / (LN[l] * (xi[i] - xi[l]))
    for i in range(N + 1):
        D[i, i] = -np.sum(D[i, :i]) - np.sum(D[i, i + 1:])
    return D


def listing_matrices(lx):
    """The six lx*lx arrays of the operator's argument list (Listing 1/2).

    Listing 2 contracts ``dxd[l, i] * ud[..., l]`` into the r-derivative at i,
    so dxd[l, i] = Dhat[i, l] (dxd = Dhat^T as a row-major array); the
    transposed pass uses dxtd[l, i] = Dhat[l, i] (dxtd = Dhat).  The box is
    isotropic, so dy = dz = dx and dyt = dzt = dxt.
    Returns (dx, dy, dz, dxt, dyt, dzt), each C-contiguous float64 (lx, lx).
    """
    xi, _ = gll_nodes_weights(lx - 1)
    Dh = deriv_matrix(xi)
    dx = np.ascontiguousarray(Dh.T)
    dxt = np.ascontiguousarray(Dh)
    return dx, dx.copy(), dx.copy(), dxt, dxt.copy(), dxt.copy()
