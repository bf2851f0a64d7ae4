/* Plain C statement of the element operator, for timing the CPU baseline.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  The loop nest follows the
 * paper's Listing 2 (Sec. 4.2): for each element, three derivative sums per
 * node, the pointwise h1 * G multiply, then three transposed sums.  The six
 * temporaries are per element (lx^3 each) instead of full size; nothing else
 * is blocked, fused or reordered.  Elements are split across OpenMP threads.
 * Arrays are [e][k][j][i] with i fastest; dx[l*lx+i] multiplies u[..., l] into
 * the r-derivative at i, dxt[l*lx+i] multiplies the r-flux at l into w at i.
 */
#include <stdlib.h>
#include <stdint.h>

void oracle_ax_ref(double* w, const double* u,
                   const double* dx, const double* dy, const double* dz,
                   const double* dxt, const double* dyt, const double* dzt,
                   const double* h1, const double* g11, const double* g22,
                   const double* g33, const double* g12, const double* g13,
                   const double* g23, int64_t nel, int lx)
{
    const int64_t n3 = (int64_t)lx * lx * lx;
#pragma omp parallel
    {
        double* ur = (double*)malloc(sizeof(double) * 6 * n3);
        double* us = ur + n3;
        double* ut = us + n3;
        double* vr = ut + n3;
        double* vs = vr + n3;
        double* vt = vs + n3;
#pragma omp for schedule(static)
        for (int64_t e = 0; e < nel; ++e) {
            const double* ue = u + e * n3;
            const int64_t o = e * n3;
            for (int k = 0; k < lx; ++k)
                for (int j = 0; j < lx; ++j)
                    for (int i = 0; i < lx; ++i) {
                        const int p = (k * lx + j) * lx + i;
                        double r = 0.0, s = 0.0, t = 0.0;
                        for (int l = 0; l < lx; ++l) {
                            r += dx[l * lx + i] * ue[(k * lx + j) * lx + l];
                            s += dy[l * lx + j] * ue[(k * lx + l) * lx + i];
                            t += dz[l * lx + k] * ue[(l * lx + j) * lx + i];
                        }
                        const double H = h1 ? h1[o + p] : 1.0;
                        vr[p] = H * (g11[o + p] * r + g12[o + p] * s + g13[o + p] * t);
                        vs[p] = H * (g12[o + p] * r + g22[o + p] * s + g23[o + p] * t);
                        vt[p] = H * (g13[o + p] * r + g23[o + p] * s + g33[o + p] * t);
                    }
            for (int k = 0; k < lx; ++k)
                for (int j = 0; j < lx; ++j)
                    for (int i = 0; i < lx; ++i) {
                        double acc = 0.0;
                        for (int l = 0; l < lx; ++l) {
                            acc += dxt[l * lx + i] * vr[(k * lx + j) * lx + l];
                            acc += dyt[l * lx + j] * vs[(k * lx + l) * lx + i];
                            acc += dzt[l * lx + k] * vt[(l * lx + j) * lx + i];
                        }
                        w[o + (k * lx + j) * lx + i] = acc;
                    }
        }
        free(ur);
    }
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
