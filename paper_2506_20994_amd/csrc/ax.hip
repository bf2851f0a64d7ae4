// The element-local stiffness operator w = A_e u (paper Sec. 4.2, Listing 2).
//
// Work decomposition (gfx950, wave64): a workgroup holds EPB elements; each
// element is owned by lx*lx threads, thread (i, j) owning the column
// u[e][0..lx)[j][i].  The column lives in registers, so the t-derivative is a
// register-only sum, and the t-flux of each slice is folded into the
// transposed t-sum as soon as it is formed.  The r- and s-derivatives need the
// rows of a k-slice, so the element is staged once in LDS; the r/s fluxes are
// staged in LDS for the transposed pass.
// The streamed arrays (u, w, h1, g11..g23) are read and written exactly once,
// with consecutive threads on consecutive addresses.
//
// Storage type TS (u, h1, G) and compute type TC:
//   double / double   (SEM_F64)
//   float  / float    (SEM_F32)
//   bf16   / float    (SEM_BF16, bf16 stored as uint16_t bit patterns)
#include "sem_internal.h"

namespace {

template <typename T> struct Load;
template <> struct Load<double> { __device__ static double get(const double* p, int64_t o) { return p[o]; } };
template <> struct Load<float> { __device__ static float get(const float* p, int64_t o) { return p[o]; } };
template <> struct Load<uint16_t> {
    __device__ static float get(const uint16_t* p, int64_t o) { return __uint_as_float((uint32_t)p[o] << 16); }
};

template <int LX> struct Shape;
// elements per workgroup: keep the workgroup near a whole number of waves and
// the three LDS element buffers of float64 within about 64 KiB.
template <> struct Shape<2>  { static constexpr int EPB = 64; };
template <> struct Shape<3>  { static constexpr int EPB = 28; };
template <> struct Shape<4>  { static constexpr int EPB = 16; };
template <> struct Shape<5>  { static constexpr int EPB = 10; };
template <> struct Shape<6>  { static constexpr int EPB = 7; };
template <> struct Shape<7>  { static constexpr int EPB = 5; };
template <> struct Shape<8>  { static constexpr int EPB = 4; };
template <> struct Shape<9>  { static constexpr int EPB = 3; };
template <> struct Shape<10> { static constexpr int EPB = 2; };
template <> struct Shape<11> { static constexpr int EPB = 2; };
template <> struct Shape<12> { static constexpr int EPB = 1; };

template <int LX, int EPB, typename TS, typename TC, typename TW>
__global__ void __launch_bounds__(EPB * LX * LX)
ax_kernel(TW* __restrict__ w, const TS* __restrict__ u,
          const TC* __restrict__ dx, const TC* __restrict__ dy, const TC* __restrict__ dz,
          const TC* __restrict__ dxt, const TC* __restrict__ dyt, const TC* __restrict__ dzt,
          const TS* __restrict__ h1, const TS* __restrict__ g11, const TS* __restrict__ g22,
          const TS* __restrict__ g33, const TS* __restrict__ g12, const TS* __restrict__ g13,
          const TS* __restrict__ g23, int64_t nel) {
    constexpr int L2 = LX * LX;
    constexpr int L3 = L2 * LX;
    __shared__ TC s_u[EPB * L3];   // the element's u
    __shared__ TC s_r[EPB * L3];   // r-flux
    __shared__ TC s_s[EPB * L3];   // s-flux
    __shared__ TC s_d[6 * L2];     // dx, dy, dz, dxt, dyt, dzt

    const int tid = threadIdx.x;
    const int el = tid / L2;
    const int ij = tid - el * L2;
    const int i = ij % LX;
    const int j = ij / LX;
    const int64_t e = (int64_t)blockIdx.x * EPB + el;
    const bool live = e < nel;
    const int64_t base = e * L3 + ij;
    TC* su = s_u + el * L3;
    TC* sr = s_r + el * L3;
    TC* ss = s_s + el * L3;
    const TC* sdx = s_d;
    const TC* sdy = s_d + L2;
    const TC* sdz = s_d + 2 * L2;
    const TC* sdxt = s_d + 3 * L2;
    const TC* sdyt = s_d + 4 * L2;
    const TC* sdzt = s_d + 5 * L2;

    for (int q = tid; q < L2; q += EPB * L2) {
        s_d[q] = dx[q];
        s_d[L2 + q] = dy[q];
        s_d[2 * L2 + q] = dz[q];
        s_d[3 * L2 + q] = dxt[q];
        s_d[4 * L2 + q] = dyt[q];
        s_d[5 * L2 + q] = dzt[q];
    }

    // the thread's column of u, kept in registers for the t-derivative
    TC uc[LX];
#pragma unroll
    for (int k = 0; k < LX; ++k) {
        uc[k] = live ? (TC)Load<TS>::get(u, base + k * L2) : TC(0);
        su[k * L2 + ij] = uc[k];
    }
    __syncthreads();

    TC di[LX], dj[LX];
#pragma unroll
    for (int l = 0; l < LX; ++l) {
        di[l] = sdx[l * LX + i];
        dj[l] = sdy[l * LX + j];
    }

    // forward passes slice by slice; the t-flux of slice k is folded straight
    // into the transposed t-pass: wt[m] += dzt[k, m] * vt_k
    TC wt[LX];
#pragma unroll
    for (int m = 0; m < LX; ++m) wt[m] = 0;
#pragma unroll 1
    for (int k = 0; k < LX; ++k) {
        TC r = 0, s = 0, t = 0;
#pragma unroll
        for (int l = 0; l < LX; ++l) {
            r += di[l] * su[k * L2 + j * LX + l];
            s += dj[l] * su[k * L2 + l * LX + i];
            t += sdz[l * LX + k] * uc[l];
        }
        const int64_t o = base + k * L2;
        TC G11 = 0, G22 = 0, G33 = 0, G12 = 0, G13 = 0, G23 = 0, H = 1;
        if (live) {
            G11 = Load<TS>::get(g11, o); G22 = Load<TS>::get(g22, o); G33 = Load<TS>::get(g33, o);
            G12 = Load<TS>::get(g12, o); G13 = Load<TS>::get(g13, o); G23 = Load<TS>::get(g23, o);
            if (h1) H = Load<TS>::get(h1, o);
        }
        sr[k * L2 + ij] = H * (G11 * r + G12 * s + G13 * t);
        ss[k * L2 + ij] = H * (G12 * r + G22 * s + G23 * t);
        const TC vt = H * (G13 * r + G23 * s + G33 * t);
#pragma unroll
        for (int m = 0; m < LX; ++m) wt[m] += sdzt[k * LX + m] * vt;
    }
    __syncthreads();

#pragma unroll
    for (int l = 0; l < LX; ++l) {
        di[l] = sdxt[l * LX + i];
        dj[l] = sdyt[l * LX + j];
    }
#pragma unroll
    for (int k = 0; k < LX; ++k) {
        TC acc = wt[k];
#pragma unroll
        for (int l = 0; l < LX; ++l) {
            acc += di[l] * sr[k * L2 + j * LX + l];
            acc += dj[l] * ss[k * L2 + l * LX + i];
        }
        if (live) w[base + k * L2] = (TW)acc;
    }
}

template <int LX, typename TS, typename TC, typename TW>
int launch_lx(sem_ctx_t ctx, void* w, const void* u, const void* const* D, const void* h1,
              const void* const* G, int64_t nel) {
    constexpr int EPB = Shape<LX>::EPB;
    const int64_t blocks = (nel + EPB - 1) / EPB;
    if (blocks > 0x7fffffff) return sem::fail(ctx, SEM_EINVAL, "sem_ax: nel too large");
    ax_kernel<LX, EPB, TS, TC, TW><<<(unsigned)blocks, EPB * LX * LX, 0, ctx->stream>>>(
        (TW*)w, (const TS*)u, (const TC*)D[0], (const TC*)D[1], (const TC*)D[2],
        (const TC*)D[3], (const TC*)D[4], (const TC*)D[5], (const TS*)h1,
        (const TS*)G[0], (const TS*)G[1], (const TS*)G[2], (const TS*)G[3], (const TS*)G[4],
        (const TS*)G[5], nel);
    SEM_LAUNCH_CHECK(ctx);
    return SEM_OK;
}

template <typename TS, typename TC, typename TW>
int dispatch(sem_ctx_t ctx, int lx, void* w, const void* u, const void* const* D,
             const void* h1, const void* const* G, int64_t nel) {
    switch (lx) {
        case 2: return launch_lx<2, TS, TC, TW>(ctx, w, u, D, h1, G, nel);
        case 3: return launch_lx<3, TS, TC, TW>(ctx, w, u, D, h1, G, nel);
        case 4: return launch_lx<4, TS, TC, TW>(ctx, w, u, D, h1, G, nel);
        case 5: return launch_lx<5, TS, TC, TW>(ctx, w, u, D, h1, G, nel);
        case 6: return launch_lx<6, TS, TC, TW>(ctx, w, u, D, h1, G, nel);
        case 7: return launch_lx<7, TS, TC, TW>(ctx, w, u, D, h1, G, nel);
        case 8: return launch_lx<8, TS, TC, TW>(ctx, w, u, D, h1, G, nel);
        case 9: return launch_lx<9, TS, TC, TW>(ctx, w, u, D, h1, G, nel);
        case 10: return launch_lx<10, TS, TC, TW>(ctx, w, u, D, h1, G, nel);
        case 11: return launch_lx<11, TS, TC, TW>(ctx, w, u, D, h1, G, nel);
        case 12: return launch_lx<12, TS, TC, TW>(ctx, w, u, D, h1, G, nel);
        default: return sem::fail(ctx, SEM_EUNSUPPORTED_LX, "sem_ax: lx=%d outside [2,12]", lx);
    }
}

size_t dsize(sem_dtype_t t) { return t == SEM_F64 ? 8 : t == SEM_F32 ? 4 : 2; }

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    if (!a || !b) return false;
    const char* pa = (const char*)a;
    const char* pb = (const char*)b;
    return pa < pb + nb && pb < pa + na;
}

}  // namespace

extern "C" int sem_ax(sem_ctx_t ctx, void* w, const void* u, const void* dx, const void* dy,
                      const void* dz, const void* dxt, const void* dyt, const void* dzt,
                      const void* h1, const void* g11, const void* g22, const void* g33,
                      const void* g12, const void* g13, const void* g23, int64_t nel, int lx,
                      sem_dtype_t field_dtype, sem_dtype_t out_dtype) {
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (!sem::lx_ok(lx)) return sem::fail(ctx, SEM_EUNSUPPORTED_LX, "sem_ax: lx=%d outside [2,12]", lx);
    if (nel < 0) return sem::fail(ctx, SEM_EINVAL, "sem_ax: nel=%lld < 0", (long long)nel);
    if (nel == 0) return SEM_OK;
    const void* D[6] = {dx, dy, dz, dxt, dyt, dzt};
    const void* G[6] = {g11, g22, g33, g12, g13, g23};
    if (!w || !u) return sem::fail(ctx, SEM_EINVAL, "sem_ax: null w or u");
    for (int q = 0; q < 6; ++q)
        if (!D[q] || !G[q]) return sem::fail(ctx, SEM_EINVAL, "sem_ax: null derivative or geometric-factor pointer");
    const bool f64 = field_dtype == SEM_F64;
    if (field_dtype != SEM_F64 && field_dtype != SEM_F32 && field_dtype != SEM_BF16)
        return sem::fail(ctx, SEM_EINVAL, "sem_ax: bad field dtype %d", (int)field_dtype);
    if (!(out_dtype == SEM_F32 || (out_dtype == SEM_F64 && f64)))
        return sem::fail(ctx, SEM_EINVAL, "sem_ax: unsupported out dtype %d for field dtype %d",
                         (int)out_dtype, (int)field_dtype);
    const int64_t n = nel * lx * lx * lx;
    const size_t nw = (size_t)n * dsize(out_dtype), nf = (size_t)n * dsize(field_dtype);
    const size_t nd = (size_t)lx * lx * (f64 ? 8 : 4);
    bool alias = overlaps(w, nw, u, nf) || overlaps(w, nw, h1, nf);
    for (int q = 0; q < 6; ++q) alias = alias || overlaps(w, nw, G[q], nf) || overlaps(w, nw, D[q], nd);
    if (alias) return sem::fail(ctx, SEM_EINVAL, "sem_ax: output overlaps an input");
    if (f64) return dispatch<double, double, double>(ctx, lx, w, u, D, h1, G, nel);
    if (field_dtype == SEM_F32) return dispatch<float, float, float>(ctx, lx, w, u, D, h1, G, nel);
    return dispatch<uint16_t, float, float>(ctx, lx, w, u, D, h1, G, nel);
}
