// Set-up steps: GLL quantities (host), box mesh, isoparametric geometric
// factors, scatter, element diagonal, Fourier right-hand sides, conversions.
#include <cmath>
#include <vector>

#include "sem_internal.h"

namespace sem {

// GLL points as the zeros of q = L_{N+1} - L_{N-1} (proportional to
// (1 - x^2) L_N'), found by Newton's method with q' = (2N + 1) L_N; weights
// 2 / (N (N+1) L_N^2); derivative matrix in barycentric form
// D[i][l] = (b_l / b_i) / (x_i - x_l), diagonal by the negative row sum.
void gll_host(int lx, double* xi, double* w, double* dhat) {
    const int N = lx - 1;
    std::vector<double> x(lx);
    // L_{n-1}, L_n and L_{n+1} at t by the three-term recurrence (n >= 1)
    auto legendre = [](int n, double t, double* Ln, double* Lnm1, double* Lnp1) {
        double a = 1.0, b = t;
        for (int m = 1; m < n; ++m) {
            const double c = ((2.0 * m + 1.0) * t * b - m * a) / (m + 1.0);
            a = b;
            b = c;
        }
        *Lnm1 = a;
        *Ln = b;
        *Lnp1 = ((2.0 * n + 1.0) * t * b - n * a) / (n + 1.0);
    };
    x[0] = -1.0; x[N] = 1.0;
    for (int j = 1; j < N; ++j) {
        double t = -std::cos(M_PI * j / N);
        for (int it = 0; it < 60; ++it) {
            double Ln, Lm, Lp;
            legendre(N, t, &Ln, &Lm, &Lp);
            double dt = (Lp - Lm) / ((2.0 * N + 1.0) * Ln);
            t -= dt;
            if (std::fabs(dt) < 1e-17) break;
        }
        x[j] = t;
    }
    for (int j = 0; j <= N / 2; ++j) {      // enforce x_{N-j} = -x_j
        double s = 0.5 * (x[N - j] - x[j]);
        x[j] = -s; x[N - j] = s;
    }
    if (N % 2 == 0) x[N / 2] = 0.0;
    if (xi) for (int j = 0; j < lx; ++j) xi[j] = x[j];
    if (w) {
        for (int j = 0; j < lx; ++j) {
            double Ln, Lm, Lp;
            legendre(N, x[j], &Ln, &Lm, &Lp);
            w[j] = 2.0 / (N * (N + 1.0) * Ln * Ln);
        }
    }
    if (dhat) {
        std::vector<double> bw(lx, 1.0);
        for (int j = 0; j < lx; ++j)
            for (int k = 0; k < lx; ++k)
                if (k != j) bw[j] /= (x[j] - x[k]);
        for (int i = 0; i < lx; ++i) {
            double s = 0.0;
            for (int l = 0; l < lx; ++l) {
                if (l == i) continue;
                double v = (bw[l] / bw[i]) / (x[i] - x[l]);
                dhat[i * lx + l] = v;
                s += v;
            }
            dhat[i * lx + i] = -s;
        }
    }
}

}  // namespace sem

extern "C" int sem_gll(int lx, double* xi, double* w, double* dx, double* dxt) {
    if (!sem::lx_ok(lx)) return sem::fail(nullptr, SEM_EUNSUPPORTED_LX, "sem_gll: lx=%d outside [2,12]", lx);
    double D[SEM_LX_MAX * SEM_LX_MAX];
    sem::gll_host(lx, xi, w, D);
    for (int i = 0; i < lx; ++i)
        for (int l = 0; l < lx; ++l) {
            if (dx) dx[l * lx + i] = D[i * lx + l];
            if (dxt) dxt[l * lx + i] = D[l * lx + i];
        }
    return SEM_OK;
}

namespace {

struct GllArgs {
    double xi[SEM_LX_MAX];
    double w[SEM_LX_MAX];
    double D[SEM_LX_MAX * SEM_LX_MAX];   // D[i*lx + l] = l_l'(xi_i)
};

GllArgs make_gll(int lx) {
    GllArgs g{};
    sem::gll_host(lx, g.xi, g.w, g.D);
    return g;
}

constexpr int kBlock = 256;

inline unsigned grid_for(int64_t n, int64_t cap = 1 << 20) {
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (unsigned)b;
}

// ids: periodic lattice position, or (dirichlet) -1 on the box boundary and
// the position on the (M - 1)^3 lattice of interior points
__global__ void box_mesh_kernel(int n, int lx, double amp, GllArgs g, int64_t n_local,
                                double* __restrict__ x, double* __restrict__ y,
                                double* __restrict__ z, int64_t* __restrict__ ids, bool dirichlet) {
    const int N = lx - 1;
    const int64_t M = (int64_t)n * N;
    const int64_t l3 = (int64_t)lx * lx * lx;
    const double tp = 2.0 * M_PI;
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n_local;
         L += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = L / l3;
        const int r = (int)(L - e * l3);
        const int i = r % lx, j = (r / lx) % lx, k = r / (lx * lx);
        const int64_t ex = e % n, ey = (e / n) % n, ez = e / ((int64_t)n * n);
        if (x || y || z) {
            const double X = (ex + 0.5 * (1.0 + g.xi[i])) / n;
            const double Y = (ey + 0.5 * (1.0 + g.xi[j])) / n;
            const double Z = (ez + 0.5 * (1.0 + g.xi[k])) / n;
            const double sx = sin(tp * X), sy = sin(tp * Y), sz = sin(tp * Z);
            if (x) x[L] = X + amp * sy * sz;
            if (y) y[L] = Y + amp * sz * sx;
            if (z) z[L] = Z + amp * sx * sy;
        }
        if (ids && dirichlet) {
            const int64_t I = ex * N + i, J = ey * N + j, K = ez * N + k;
            const bool inside = I > 0 && I < M && J > 0 && J < M && K > 0 && K < M;
            ids[L] = inside ? ((K - 1) * (M - 1) + (J - 1)) * (M - 1) + (I - 1) : -1;
        } else if (ids) {
            const int64_t gi = (ex * N + i) % M, gj = (ey * N + j) % M, gk = (ez * N + k) % M;
            ids[L] = (gk * M + gj) * M + gi;
        }
    }
}

__device__ inline void atomic_min_double(double* addr, double v) {
    unsigned long long* a = reinterpret_cast<unsigned long long*>(addr);
    unsigned long long old = *a, assumed;
    do {
        assumed = old;
        if (__longlong_as_double(assumed) <= v) break;
        old = atomicCAS(a, assumed, __double_as_longlong(v));
    } while (assumed != old);
}

__global__ void geometry_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                const double* __restrict__ z, int64_t n_local, int lx, GllArgs g,
                                double* __restrict__ g11, double* __restrict__ g22,
                                double* __restrict__ g33, double* __restrict__ g12,
                                double* __restrict__ g13, double* __restrict__ g23,
                                double* __restrict__ bm, double* __restrict__ detmin) {
    __shared__ double smin[kBlock];
    const int64_t l3 = (int64_t)lx * lx * lx;
    const int64_t l2 = (int64_t)lx * lx;
    double mymin = 1e300;
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n_local;
         L += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = L / l3;
        const int r = (int)(L - e * l3);
        const int i = r % lx, j = (r / lx) % lx, k = r / (lx * lx);
        const int64_t b0 = e * l3;
        // J[c][a] = d x_c / d r_a
        double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        const double* X[3] = {x, y, z};
        for (int l = 0; l < lx; ++l) {
            const double di = g.D[i * lx + l], dj = g.D[j * lx + l], dk = g.D[k * lx + l];
            const int64_t pr = b0 + k * l2 + j * lx + l;
            const int64_t ps = b0 + k * l2 + l * lx + i;
            const int64_t pt = b0 + l * l2 + j * lx + i;
            for (int c = 0; c < 3; ++c) {
                J[c][0] += di * X[c][pr];
                J[c][1] += dj * X[c][ps];
                J[c][2] += dk * X[c][pt];
            }
        }
        // cofactors: inverse(J)[a][c] = cof[c][a] / det
        const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        const double c10 = J[0][2] * J[2][1] - J[0][1] * J[2][2];
        const double c11 = J[0][0] * J[2][2] - J[0][2] * J[2][0];
        const double c12 = J[0][1] * J[2][0] - J[0][0] * J[2][1];
        const double c20 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
        const double c21 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
        const double c22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        mymin = fmin(mymin, det);
        // Jinv[a][c] = cof[c][a] / det, so G_ab = W sum_c cof[c][a] cof[c][b] / det^2
        const double W = g.w[i] * g.w[j] * g.w[k] * det;
        const double s = W / (det * det);
        const double cof[3][3] = {{c00, c01, c02}, {c10, c11, c12}, {c20, c21, c22}};
        double Gm[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = a; b < 3; ++b)
                Gm[a][b] = s * (cof[0][a] * cof[0][b] + cof[1][a] * cof[1][b] + cof[2][a] * cof[2][b]);
        g11[L] = Gm[0][0]; g22[L] = Gm[1][1]; g33[L] = Gm[2][2];
        g12[L] = Gm[0][1]; g13[L] = Gm[0][2]; g23[L] = Gm[1][2];
        if (bm) bm[L] = W;
    }
    smin[threadIdx.x] = mymin;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomic_min_double(detmin, smin[0]);
}

template <typename T>
__global__ void scatter_kernel(T* __restrict__ out, const T* __restrict__ in,
                               const int64_t* __restrict__ ids, int64_t n) {
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n;
         L += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g = ids[L];
        out[L] = g >= 0 ? in[g] : T(0);          // negative id: Dirichlet node, 0
    }
}

__global__ void ax_diag_kernel(double* __restrict__ d, const double* __restrict__ dx,
                               const double* __restrict__ h1, const double* __restrict__ g11,
                               const double* __restrict__ g22, const double* __restrict__ g33,
                               const double* __restrict__ g12, const double* __restrict__ g13,
                               const double* __restrict__ g23, int64_t n_local, int lx) {
    const int64_t l3 = (int64_t)lx * lx * lx;
    const int64_t l2 = (int64_t)lx * lx;
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n_local;
         L += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = L / l3;
        const int r = (int)(L - e * l3);
        const int i = r % lx, j = (r / lx) % lx, k = r / (lx * lx);
        const int64_t b0 = e * l3;
        // Dhat_ab = dx[b*lx + a]
        double acc = 0.0;
        for (int l = 0; l < lx; ++l) {
            const double a = dx[i * lx + l], b = dx[j * lx + l], c = dx[k * lx + l];
            const int64_t pr = b0 + k * l2 + j * lx + l;
            const int64_t ps = b0 + k * l2 + l * lx + i;
            const int64_t pt = b0 + l * l2 + j * lx + i;
            const double hr = h1 ? h1[pr] : 1.0, hs = h1 ? h1[ps] : 1.0, ht = h1 ? h1[pt] : 1.0;
            acc += a * a * hr * g11[pr] + b * b * hs * g22[ps] + c * c * ht * g33[pt];
        }
        const double di = dx[i * lx + i], dj = dx[j * lx + j], dk = dx[k * lx + k];
        const double h = h1 ? h1[L] : 1.0;
        acc += 2.0 * h * (di * dj * g12[L] + di * dk * g13[L] + dj * dk * g23[L]);
        d[L] = acc;
    }
}

struct Modes {
    int nm;
    int k[64][3];
    double amp[64];
    double phase[64];
};

__global__ void fourier_kernel(double* __restrict__ f, const double* __restrict__ x,
                               const double* __restrict__ y, const double* __restrict__ z,
                               const double* __restrict__ scale, int64_t n, Modes m) {
    const double tp = 2.0 * M_PI;
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n;
         L += (int64_t)gridDim.x * blockDim.x) {
        const double px = x[L], py = y[L], pz = z[L];
        double s = 0.0;
        for (int q = 0; q < m.nm; ++q)
            s += m.amp[q] * cos(tp * (m.k[q][0] * px + m.k[q][1] * py + m.k[q][2] * pz) + m.phase[q]);
        f[L] = scale ? scale[L] * s : s;
    }
}

__device__ inline uint16_t f32_to_bf16_rne(float f) {
    uint32_t b = __float_as_uint(f);
    if ((b & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((b >> 16) | 0x40u);
    b += 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

template <typename TD, typename TS>
__device__ inline TD conv(TS v);
template <> __device__ inline double conv<double, double>(double v) { return v; }
template <> __device__ inline float conv<float, double>(double v) { return (float)v; }
template <> __device__ inline uint16_t conv<uint16_t, double>(double v) { return f32_to_bf16_rne((float)v); }
template <> __device__ inline double conv<double, float>(float v) { return (double)v; }
template <> __device__ inline float conv<float, float>(float v) { return v; }
template <> __device__ inline uint16_t conv<uint16_t, float>(float v) { return f32_to_bf16_rne(v); }
template <> __device__ inline double conv<double, uint16_t>(uint16_t v) { return (double)bf16_to_f32(v); }
template <> __device__ inline float conv<float, uint16_t>(uint16_t v) { return bf16_to_f32(v); }
template <> __device__ inline uint16_t conv<uint16_t, uint16_t>(uint16_t v) { return v; }

template <typename TD, typename TS>
__global__ void convert_kernel(TD* __restrict__ dst, const TS* __restrict__ src, int64_t n) {
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n;
         L += (int64_t)gridDim.x * blockDim.x)
        dst[L] = conv<TD, TS>(src[L]);
}

}  // namespace

namespace {

int box_mesh(sem_ctx_t ctx, const char* name, int n, int lx, double amp, double* x, double* y, double* z,
             int64_t* ids, bool dirichlet) {
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (!sem::lx_ok(lx)) return sem::fail(ctx, SEM_EUNSUPPORTED_LX, "%s: lx=%d", name, lx);
    if (n < 1) return sem::fail(ctx, SEM_EINVAL, "%s: n=%d < 1", name, n);
    const int64_t n_local = (int64_t)n * n * n * lx * lx * lx;
    GllArgs g = make_gll(lx);
    box_mesh_kernel<<<grid_for(n_local), kBlock, 0, ctx->stream>>>(n, lx, amp, g, n_local, x, y, z, ids,
                                                                   dirichlet);
    SEM_LAUNCH_CHECK(ctx);
    return SEM_OK;
}

}  // namespace

extern "C" int sem_box_mesh(sem_ctx_t ctx, int n, int lx, double amp, double* x, double* y,
                            double* z, int64_t* ids) {
    return box_mesh(ctx, "sem_box_mesh", n, lx, amp, x, y, z, ids, false);
}

extern "C" int sem_box_mesh_dirichlet(sem_ctx_t ctx, int n, int lx, double amp, double* x, double* y,
                                      double* z, int64_t* ids) {
    return box_mesh(ctx, "sem_box_mesh_dirichlet", n, lx, amp, x, y, z, ids, true);
}

extern "C" int sem_geometry(sem_ctx_t ctx, const double* x, const double* y, const double* z,
                            int64_t nel, int lx, double* g11, double* g22, double* g33,
                            double* g12, double* g13, double* g23, double* bm, double* min_detj) {
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (!sem::lx_ok(lx)) return sem::fail(ctx, SEM_EUNSUPPORTED_LX, "sem_geometry: lx=%d", lx);
    if (nel < 0) return sem::fail(ctx, SEM_EINVAL, "sem_geometry: nel < 0");
    if (!x || !y || !z || !g11 || !g22 || !g33 || !g12 || !g13 || !g23)
        return sem::fail(ctx, SEM_EINVAL, "sem_geometry: null pointer");
    const int64_t n_local = nel * lx * lx * lx;
    if (n_local == 0) { if (min_detj) *min_detj = 0.0; return SEM_OK; }
    GllArgs g = make_gll(lx);
    ctx->host_pinned[0] = 1e300;
    SEM_HIP(ctx, hipMemcpyAsync(ctx->red, ctx->host_pinned, sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    geometry_kernel<<<grid_for(n_local, 4096), kBlock, 0, ctx->stream>>>(
        x, y, z, n_local, lx, g, g11, g22, g33, g12, g13, g23, bm, ctx->red);
    SEM_LAUNCH_CHECK(ctx);
    SEM_HIP(ctx, hipMemcpyAsync(ctx->host_pinned, ctx->red, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    SEM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const double dmin = ctx->host_pinned[0];
    if (min_detj) *min_detj = dmin;
    if (!(dmin > 0.0)) return sem::fail(ctx, SEM_EGEOMETRY, "sem_geometry: folded mesh, min det J = %g", dmin);
    return SEM_OK;
}

extern "C" int sem_scatter(sem_ctx_t ctx, void* out, const void* in, const int64_t* ids,
                           int64_t n_local, sem_dtype_t dtype) {
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (n_local < 0) return sem::fail(ctx, SEM_EINVAL, "sem_scatter: n_local < 0");
    if (n_local == 0) return SEM_OK;
    if (!out || !in || !ids) return sem::fail(ctx, SEM_EINVAL, "sem_scatter: null pointer");
    const unsigned grid = grid_for(n_local);
    switch (dtype) {
        case SEM_F64: scatter_kernel<double><<<grid, kBlock, 0, ctx->stream>>>((double*)out, (const double*)in, ids, n_local); break;
        case SEM_F32: scatter_kernel<float><<<grid, kBlock, 0, ctx->stream>>>((float*)out, (const float*)in, ids, n_local); break;
        case SEM_BF16: scatter_kernel<uint16_t><<<grid, kBlock, 0, ctx->stream>>>((uint16_t*)out, (const uint16_t*)in, ids, n_local); break;
        default: return sem::fail(ctx, SEM_EINVAL, "sem_scatter: bad dtype %d", (int)dtype);
    }
    SEM_LAUNCH_CHECK(ctx);
    return SEM_OK;
}

extern "C" int sem_ax_diag(sem_ctx_t ctx, double* d, const double* dx, const double* h1,
                           const double* g11, const double* g22, const double* g33,
                           const double* g12, const double* g13, const double* g23,
                           int64_t nel, int lx) {
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (!sem::lx_ok(lx)) return sem::fail(ctx, SEM_EUNSUPPORTED_LX, "sem_ax_diag: lx=%d", lx);
    if (nel < 0) return sem::fail(ctx, SEM_EINVAL, "sem_ax_diag: nel < 0");
    if (nel == 0) return SEM_OK;
    if (!d || !dx || !g11 || !g22 || !g33 || !g12 || !g13 || !g23)
        return sem::fail(ctx, SEM_EINVAL, "sem_ax_diag: null pointer");
    const int64_t n_local = nel * lx * lx * lx;
    ax_diag_kernel<<<grid_for(n_local), kBlock, 0, ctx->stream>>>(d, dx, h1, g11, g22, g33, g12, g13, g23, n_local, lx);
    SEM_LAUNCH_CHECK(ctx);
    return SEM_OK;
}

extern "C" int sem_fourier(sem_ctx_t ctx, double* f, const double* x, const double* y,
                           const double* z, const double* scale, int64_t n_local,
                           const int64_t* k, const double* amp, const double* phase, int nmodes) {
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (nmodes < 0 || nmodes > 64) return sem::fail(ctx, SEM_EINVAL, "sem_fourier: nmodes=%d not in [0,64]", nmodes);
    if (n_local < 0) return sem::fail(ctx, SEM_EINVAL, "sem_fourier: n_local < 0");
    if (n_local == 0) return SEM_OK;
    if (!f || !x || !y || !z || (nmodes > 0 && (!k || !amp || !phase)))
        return sem::fail(ctx, SEM_EINVAL, "sem_fourier: null pointer");
    Modes m{};
    m.nm = nmodes;
    for (int q = 0; q < nmodes; ++q) {
        for (int c = 0; c < 3; ++c) m.k[q][c] = (int)k[3 * q + c];
        m.amp[q] = amp[q];
        m.phase[q] = phase[q];
    }
    fourier_kernel<<<grid_for(n_local), kBlock, 0, ctx->stream>>>(f, x, y, z, scale, n_local, m);
    SEM_LAUNCH_CHECK(ctx);
    return SEM_OK;
}

extern "C" int sem_convert(sem_ctx_t ctx, void* dst, sem_dtype_t dt, const void* src,
                           sem_dtype_t st, int64_t n) {
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (n < 0) return sem::fail(ctx, SEM_EINVAL, "sem_convert: n < 0");
    if (n == 0) return SEM_OK;
    if (!dst || !src) return sem::fail(ctx, SEM_EINVAL, "sem_convert: null pointer");
    const unsigned grid = grid_for(n);
    hipStream_t s = ctx->stream;
#define SEM_CONV(TD, TS) convert_kernel<TD, TS><<<grid, kBlock, 0, s>>>((TD*)dst, (const TS*)src, n)
    if (dt == SEM_F64 && st == SEM_F64) SEM_CONV(double, double);
    else if (dt == SEM_F32 && st == SEM_F64) SEM_CONV(float, double);
    else if (dt == SEM_BF16 && st == SEM_F64) SEM_CONV(uint16_t, double);
    else if (dt == SEM_F64 && st == SEM_F32) SEM_CONV(double, float);
    else if (dt == SEM_F32 && st == SEM_F32) SEM_CONV(float, float);
    else if (dt == SEM_BF16 && st == SEM_F32) SEM_CONV(uint16_t, float);
    else if (dt == SEM_F64 && st == SEM_BF16) SEM_CONV(double, uint16_t);
    else if (dt == SEM_F32 && st == SEM_BF16) SEM_CONV(float, uint16_t);
    else if (dt == SEM_BF16 && st == SEM_BF16) SEM_CONV(uint16_t, uint16_t);
    else return sem::fail(ctx, SEM_EINVAL, "sem_convert: bad dtype pair %d <- %d", (int)dt, (int)st);
#undef SEM_CONV
    SEM_LAUNCH_CHECK(ctx);
    return SEM_OK;
}
