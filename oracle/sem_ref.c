/* Plain C statement of the spectral-element Poisson path: box mesh, geometry,
 * element operator, Jacobi diagonal, gather, Fourier source and Jacobi-PCG.
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
 * CPU-baseline leg call it (through oracle/cref.py); the HIP library shares no
 * code with it.  It exists because the numpy oracle is too slow for reference
 * solutions on 32^3 boxes; every function here is pinned against the numpy
 * oracle on small cases (tests/test_oracle_cref.py).
 *
 * Conventions.
 *   Element-local arrays are [e][k][j][i] with i fastest, n3 = lx^3 entries
 *   per element.  Dh[a * lx + b] = l_b'(xi_a): the derivative, at GLL node a,
 *   of the Lagrange polynomial of node b (Sec. 3, Eq. 2-3).  w: GLL weights.
 *   g11 .. g23 are the geometric factors of the weak form of Eq. 1 with the
 *   quadrature weights and |J| folded in:
 *       g_ab = w_i w_j w_k |J| sum_c (dr_a/dx_c)(dr_b/dx_c),  1 = r, 2 = s, 3 = t.
 *   ids[L] is the unique (global) node of local node L, negative for a node
 *   held at zero (homogeneous Dirichlet).
 *
 * Nothing is blocked or fused beyond a per-element loop; elements (and unique
 * nodes in the gather) are split across OpenMP threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IDX(k, j, i) (((k) * lx + (j)) * lx + (i))

/* Undeformed position (ex + (1 + xi_i)/2) / n of the nodes of the periodic
 * unit-cube box of n^3 elements (numbered e = ex + n (ey + n ez)), then the
 * cyclic sine map x = X + amp sin(2 pi Y) sin(2 pi Z) (y, z cyclically). */
void oracle_box_coords(int n, int lx, double amp, const double* xi,
                       double* x, double* y, double* z)
{
    const int64_t nel = (int64_t)n * n * n, n3 = (int64_t)lx * lx * lx;
    const double tp = 2.0 * M_PI;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < nel; ++e) {
        const int ex = (int)(e % n), ey = (int)((e / n) % n), ez = (int)(e / ((int64_t)n * n));
        for (int k = 0; k < lx; ++k)
            for (int j = 0; j < lx; ++j)
                for (int i = 0; i < lx; ++i) {
                    const double X = (ex + 0.5 * (1.0 + xi[i])) / n;
                    const double Y = (ey + 0.5 * (1.0 + xi[j])) / n;
                    const double Z = (ez + 0.5 * (1.0 + xi[k])) / n;
                    const int64_t L = e * n3 + IDX(k, j, i);
                    x[L] = X + amp * sin(tp * Y) * sin(tp * Z);
                    y[L] = Y + amp * sin(tp * Z) * sin(tp * X);
                    z[L] = Z + amp * sin(tp * X) * sin(tp * Y);
                }
    }
}

/* Isoparametric geometry: J[c][a] = dx_c/dr_a is Dh applied along reference
 * direction a to coordinate c; g_ab and the mass weight B = w_i w_j w_k |J|.
 * Returns the minimum det J over all nodes. */
double oracle_geometry(const double* x, const double* y, const double* z, int64_t nel, int lx,
                       const double* Dh, const double* w,
                       double* g11, double* g22, double* g33,
                       double* g12, double* g13, double* g23, double* B)
{
    const int64_t n3 = (int64_t)lx * lx * lx;
    double dmin = INFINITY;
#pragma omp parallel for schedule(static) reduction(min : dmin)
    for (int64_t e = 0; e < nel; ++e) {
        const double* C[3] = {x + e * n3, y + e * n3, z + e * n3};
        for (int k = 0; k < lx; ++k)
            for (int j = 0; j < lx; ++j)
                for (int i = 0; i < lx; ++i) {
                    double J[3][3];
                    for (int c = 0; c < 3; ++c) {
                        double dr = 0.0, ds = 0.0, dt = 0.0;
                        for (int b = 0; b < lx; ++b) {
                            dr += Dh[i * lx + b] * C[c][IDX(k, j, b)];
                            ds += Dh[j * lx + b] * C[c][IDX(k, b, i)];
                            dt += Dh[k * lx + b] * C[c][IDX(b, j, i)];
                        }
                        J[c][0] = dr;
                        J[c][1] = ds;
                        J[c][2] = dt;
                    }
                    /* inverse by cofactors: Ji[a][c] = dr_a/dx_c */
                    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
                                     - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
                                     + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
                    double Ji[3][3];
                    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
                    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
                    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
                    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
                    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
                    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
                    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
                    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
                    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
                    const double W = w[i] * w[j] * w[k] * det;
                    double M[3][3];
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b)
                            M[a][b] = W * (Ji[a][0] * Ji[b][0] + Ji[a][1] * Ji[b][1] + Ji[a][2] * Ji[b][2]);
                    const int64_t L = e * n3 + IDX(k, j, i);
                    g11[L] = M[0][0]; g22[L] = M[1][1]; g33[L] = M[2][2];
                    g12[L] = M[0][1]; g13[L] = M[0][2]; g23[L] = M[1][2];
                    if (B) B[L] = W;
                    if (det < dmin) dmin = det;
                }
    }
    return dmin;
}

/* Element operator of Sec. 4.2, written as a loop over quadrature points:
 * w_e = sum_{a,b} D_a^T diag(h1 g_ab) D_b u_e.  At every node m the reference
 * gradient (D_b u)(m) is formed along the three grid lines through m, the
 * flux q_a = h1 sum_b g_ab (D_b u)(m) is taken, and q_a is spread back along
 * the same lines with the transposed derivative weights (w_n += Dh[m_a, n_a]
 * q_a for the nodes n on the line through m in direction a).  h1 may be NULL
 * (h1 = 1).  With h2b non-NULL the Helmholtz form adds the diagonal mass term
 * h2b_n u_n (h2b = h2 w_i w_j w_k |J| per node). */
void oracle_ax(double* w, const double* u, const double* Dh, const double* h1,
               const double* g11, const double* g22, const double* g33,
               const double* g12, const double* g13, const double* g23,
               const double* h2b, int64_t nel, int lx)
{
    const int64_t n3 = (int64_t)lx * lx * lx;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < nel; ++e) {
        const double* ue = u + e * n3;
        double* we = w + e * n3;
        memset(we, 0, sizeof(double) * n3);
        for (int k = 0; k < lx; ++k)
            for (int j = 0; j < lx; ++j)
                for (int i = 0; i < lx; ++i) {
                    double gr = 0.0, gs = 0.0, gt = 0.0;
                    for (int b = 0; b < lx; ++b) {
                        gr += Dh[i * lx + b] * ue[IDX(k, j, b)];
                        gs += Dh[j * lx + b] * ue[IDX(k, b, i)];
                        gt += Dh[k * lx + b] * ue[IDX(b, j, i)];
                    }
                    const int64_t L = e * n3 + IDX(k, j, i);
                    const double h = h1 ? h1[L] : 1.0;
                    const double qr = h * (g11[L] * gr + g12[L] * gs + g13[L] * gt);
                    const double qs = h * (g12[L] * gr + g22[L] * gs + g23[L] * gt);
                    const double qt = h * (g13[L] * gr + g23[L] * gs + g33[L] * gt);
                    for (int b = 0; b < lx; ++b) {
                        we[IDX(k, j, b)] += Dh[i * lx + b] * qr;
                        we[IDX(k, b, i)] += Dh[j * lx + b] * qs;
                        we[IDX(b, j, i)] += Dh[k * lx + b] * qt;
                    }
                }
        if (h2b)
            for (int64_t p = 0; p < n3; ++p) we[p] += h2b[e * n3 + p] * ue[p];
    }
}

/* Diagonal of the element matrices above: at node n = (i, j, k),
 *   d_n = sum_m sum_{a,b} (D_a)_{mn} h1 g_ab(m) (D_b)_{mn};
 * (D_r)_{mn} is nonzero only for m on the r-line through n, where it is
 * Dh[m_i, i], so the pure terms run along one line each and the mixed terms
 * only see m = n.  The Helmholtz mass term h2b (may be NULL) adds to it. */
void oracle_diag(double* d, const double* Dh, const double* h1,
                 const double* g11, const double* g22, const double* g33,
                 const double* g12, const double* g13, const double* g23,
                 const double* h2b, int64_t nel, int lx)
{
    const int64_t n3 = (int64_t)lx * lx * lx;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < nel; ++e) {
        const int64_t o = e * n3;
#define V(g, p) ((h1 ? h1[o + (p)] : 1.0) * g[o + (p)])
        for (int k = 0; k < lx; ++k)
            for (int j = 0; j < lx; ++j)
                for (int i = 0; i < lx; ++i) {
                    double s = 0.0;
                    for (int m = 0; m < lx; ++m) {
                        const double dr = Dh[m * lx + i], ds = Dh[m * lx + j], dt = Dh[m * lx + k];
                        s += dr * dr * V(g11, IDX(k, j, m));
                        s += ds * ds * V(g22, IDX(k, m, i));
                        s += dt * dt * V(g33, IDX(m, j, i));
                    }
                    const int p = IDX(k, j, i);
                    const double di = Dh[i * lx + i], dj = Dh[j * lx + j], dk = Dh[k * lx + k];
                    s += 2.0 * di * dj * V(g12, p) + 2.0 * di * dk * V(g13, p) + 2.0 * dj * dk * V(g23, p);
                    d[o + p] = s + (h2b ? h2b[o + p] : 0.0);
                }
#undef V
    }
}

/* f_L = sum_m amp_m cos(2 pi k_m . x_L + phase_m) */
void oracle_fourier(double* f, const double* x, const double* y, const double* z, int64_t n,
                    const int64_t* k, const double* amp, const double* phase, int nmodes)
{
    const double tp = 2.0 * M_PI;
#pragma omp parallel for schedule(static)
    for (int64_t L = 0; L < n; ++L) {
        double s = 0.0;
        for (int m = 0; m < nmodes; ++m)
            s += amp[m] * cos(tp * (k[3 * m] * x[L] + k[3 * m + 1] * y[L] + k[3 * m + 2] * z[L]) + phase[m]);
        f[L] = s;
    }
}

/* out = Q^T in: the sum of the local copies of every unique node (serial, in
 * increasing local index). */
void oracle_gather(double* out, const double* in, const int64_t* ids, int64_t n_local, int64_t n_unique)
{
    memset(out, 0, sizeof(double) * n_unique);
    for (int64_t L = 0; L < n_local; ++L)
        if (ids[L] >= 0) out[ids[L]] += in[L];
}

/* ------------------------------------------------------------- Jacobi-PCG */

typedef struct {
    const int64_t* ids;
    int64_t nel, n_local, n_unique;
    int lx;
    const double *Dh, *h1, *g[6], *h2b;
    int64_t* off;      /* CSR of the local copies of every unique node */
    int64_t* loc;
    double *ul, *wl;   /* local-layout work fields */
} Problem;

static void scatter(const Problem* P, double* ul, const double* xu)
{
#pragma omp parallel for schedule(static)
    for (int64_t L = 0; L < P->n_local; ++L) ul[L] = P->ids[L] >= 0 ? xu[P->ids[L]] : 0.0;
}

static void gather_csr(const Problem* P, double* yu, const double* wl)
{
#pragma omp parallel for schedule(static)
    for (int64_t u = 0; u < P->n_unique; ++u) {
        double s = 0.0;
        for (int64_t q = P->off[u]; q < P->off[u + 1]; ++q) s += wl[P->loc[q]];
        yu[u] = s;
    }
}

/* y = A_G x = Q^T A_e Q x on unique vectors */
static void apply_assembled(const Problem* P, double* yu, const double* xu)
{
    scatter(P, P->ul, xu);
    oracle_ax(P->wl, P->ul, P->Dh, P->h1, P->g[0], P->g[1], P->g[2], P->g[3], P->g[4], P->g[5],
              P->h2b, P->nel, P->lx);
    gather_csr(P, yu, P->wl);
}

static double dot(const double* a, const double* b, int64_t n)
{
    double s = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : s)
    for (int64_t q = 0; q < n; ++q) s += a[q] * b[q];
    return s;
}

/* Solve A_G x = b by Jacobi-preconditioned CG (Hestenes and Stiefel 1952;
 * Saad 2003, Alg. 9.1), M = diag(A_G), x_0 = 0, stopping when the recursively
 * updated residual satisfies ||r||_2 <= tol ||b||_2 or after maxit
 * iterations.  With `project` (the periodic operator, singular with the
 * constants as null space; b must then sum to zero) the mean of x is removed
 * at the end.  h2b (may be NULL): the Helmholtz operator A + h2 B.  x, b: unique vectors of n_unique entries.  *relres receives
 * the true ||b - A x||_2 / ||b||_2.  Returns the number of iterations, or -1
 * when memory runs out. */
int oracle_pcg(double* x, const double* b, const int64_t* ids, int64_t nel, int lx, int64_t n_unique,
               const double* Dh, const double* h1,
               const double* g11, const double* g22, const double* g33,
               const double* g12, const double* g13, const double* g23, const double* h2b,
               double tol, int maxit, int project, double* relres)
{
    Problem P = {0};
    P.ids = ids; P.nel = nel; P.lx = lx; P.n_unique = n_unique;
    P.n_local = nel * lx * lx * lx;
    P.Dh = Dh; P.h1 = h1;
    P.g[0] = g11; P.g[1] = g22; P.g[2] = g33; P.g[3] = g12; P.g[4] = g13; P.g[5] = g23;
    P.h2b = h2b;
    P.off = calloc((size_t)n_unique + 1, sizeof(int64_t));
    P.loc = malloc(sizeof(int64_t) * (size_t)P.n_local);
    P.ul = malloc(sizeof(double) * (size_t)P.n_local);
    P.wl = malloc(sizeof(double) * (size_t)P.n_local);
    double* r = malloc(sizeof(double) * (size_t)n_unique);
    double* z = malloc(sizeof(double) * (size_t)n_unique);
    double* p = malloc(sizeof(double) * (size_t)n_unique);
    double* q = malloc(sizeof(double) * (size_t)n_unique);
    double* minv = malloc(sizeof(double) * (size_t)n_unique);
    int it = -1;
    if (!P.off || !P.loc || !P.ul || !P.wl || !r || !z || !p || !q || !minv) goto out;
    /* CSR of copies by counting */
    for (int64_t L = 0; L < P.n_local; ++L)
        if (ids[L] >= 0) ++P.off[ids[L] + 1];
    for (int64_t u = 0; u < n_unique; ++u) P.off[u + 1] += P.off[u];
    {
        int64_t* fill = malloc(sizeof(int64_t) * (size_t)n_unique);
        if (!fill) goto out;
        memcpy(fill, P.off, sizeof(int64_t) * (size_t)n_unique);
        for (int64_t L = 0; L < P.n_local; ++L)
            if (ids[L] >= 0) P.loc[fill[ids[L]]++] = L;
        free(fill);
    }
    /* Jacobi: the assembled diagonal */
    oracle_diag(P.wl, Dh, h1, g11, g22, g33, g12, g13, g23, h2b, nel, lx);
    gather_csr(&P, minv, P.wl);
    for (int64_t u = 0; u < n_unique; ++u) minv[u] = 1.0 / minv[u];

    const double bnorm = sqrt(dot(b, b, n_unique));
    for (int64_t u = 0; u < n_unique; ++u) {
        x[u] = 0.0;
        r[u] = b[u];
        z[u] = minv[u] * r[u];
        p[u] = z[u];
    }
    double rz = dot(r, z, n_unique);
    it = 0;
    if (bnorm > 0.0 && sqrt(dot(r, r, n_unique)) > tol * bnorm) {
        while (it < maxit) {
            apply_assembled(&P, q, p);
            const double alpha = rz / dot(p, q, n_unique);
#pragma omp parallel for schedule(static)
            for (int64_t u = 0; u < n_unique; ++u) {
                x[u] += alpha * p[u];
                r[u] -= alpha * q[u];
            }
            ++it;
            if (sqrt(dot(r, r, n_unique)) <= tol * bnorm) break;
#pragma omp parallel for schedule(static)
            for (int64_t u = 0; u < n_unique; ++u) z[u] = minv[u] * r[u];
            const double rz_new = dot(r, z, n_unique);
            const double beta = rz_new / rz;
            rz = rz_new;
#pragma omp parallel for schedule(static)
            for (int64_t u = 0; u < n_unique; ++u) p[u] = z[u] + beta * p[u];
        }
    }
    if (project) {
        double s = 0.0;
        for (int64_t u = 0; u < n_unique; ++u) s += x[u];
        s /= (double)n_unique;
        for (int64_t u = 0; u < n_unique; ++u) x[u] -= s;
    }
    /* true residual */
    apply_assembled(&P, q, x);
    for (int64_t u = 0; u < n_unique; ++u) q[u] = b[u] - q[u];
    if (relres) *relres = bnorm > 0.0 ? sqrt(dot(q, q, n_unique)) / bnorm : 0.0;
out:
    free(P.off); free(P.loc); free(P.ul); free(P.wl);
    free(r); free(z); free(p); free(q); free(minv);
    return it;
}

/* y = A_G x on unique vectors (the assembled operator of the PCG above), for
 * residual checks of solutions computed elsewhere.  Returns -1 when memory
 * runs out. */
int oracle_apply_assembled(double* y, const double* x, const int64_t* ids, int64_t nel, int lx,
                           int64_t n_unique, const double* Dh, const double* h1,
                           const double* g11, const double* g22, const double* g33,
                           const double* g12, const double* g13, const double* g23,
                           const double* h2b)
{
    const int64_t n_local = nel * lx * lx * lx;
    double* ul = malloc(sizeof(double) * (size_t)n_local);
    double* wl = malloc(sizeof(double) * (size_t)n_local);
    if (!ul || !wl) {
        free(ul);
        free(wl);
        return -1;
    }
#pragma omp parallel for schedule(static)
    for (int64_t L = 0; L < n_local; ++L) ul[L] = ids[L] >= 0 ? x[ids[L]] : 0.0;
    oracle_ax(wl, ul, Dh, h1, g11, g22, g33, g12, g13, g23, h2b, nel, lx);
    oracle_gather(y, wl, ids, n_local, n_unique);
    free(ul);
    free(wl);
    return 0;
}

/* Threads of the OpenMP loops above (n <= 0 leaves the setting alone). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_num_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp master
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            n = omp_get_num_threads();
#endif
        }
    }
    return n;
}
