// Krylov solves around the assembled operator y = gs(Ax(x)).
//
//  * Jacobi-preconditioned CG (Hestenes-Stiefel; Saad, Alg. 9.1), M = diag(A_G),
//    x_0 = 0, stopped on the recursively updated residual.
//  * Float64 iterative refinement (Wilkinson; Carson and Higham 2018) around
//    inner PCG solves whose vectors are float32 and whose operator is the
//    float32 or the bfloat16-factor form of the element operator; dot products
//    are always accumulated in float64.
//
// Krylov vectors live on the unique (assembled) nodes, numbered densely by
// the gather-scatter plan: the operator reads p[lid[L]] for every local node L
// and writes its element-local output w_L in the local layout (coalesced);
// the update kernel assembles w_u = sum of the local copies of u, read
// through the plan's CSR lists, on the fly, so no separate gather-scatter
// pass and no duplicated vector traffic remain.
// p^T A p is the element-local sum of p_L w_L taken in the operator's
// epilogue.  Everything stays on the device: scalars (alpha, beta, r.z, ...)
// live in a small device struct, a `done` flag turns every later kernel of a
// converged solve into an early return, and the host reads the flag once
// every `check_every` iterations.  Reductions are two-stage with a fixed
// number of partials and a fixed summation order: results are bitwise
// reproducible.
#include <cmath>
#include <mutex>
#include <vector>

#include "sem_internal.h"

namespace {

constexpr int kBlock = 256;
// vector kernels run on a fixed grid (fixed partial count, deterministic
// reductions): 8192 blocks for float64 vectors, 2048 for float32 ones, whose
// lighter per-node traffic is better served by more nodes per thread and
// shorter single-block finalisers (measured at 32^3, lx = 8)
constexpr int kGrid = 8192;
constexpr int kGrid32 = 2048;
constexpr int kFinal = 1024;          // threads of the single-block finalisers

struct Scal {
    double rz, pAp, alpha, beta, rr, bb, tol2, mean, pw_prev;
    int done, it, breakdown, maxit;
    int usej, njac, fallback;   // flexible CG: Jacobi this iteration, count, for good
    double delta2, rmax2;       // residual replacement: pause when rr < delta2 * rmax2
    int pause;
};

// sum of a per-thread double over a 256-thread block, valid in thread 0
__device__ __forceinline__ double block_sum(double v, double* s_red) {
    v = sem::wave_sum(v);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += s_red[q];
    __syncthreads();
    return t;
}

// fixed-order sum of n partials (stride `stride`) by one 1024-thread block
__device__ double final_sum(const double* __restrict__ part, int n, int stride, double* s_red) {
    double v = 0.0;
    for (int q = threadIdx.x; q < n; q += blockDim.x) v += part[(int64_t)q * stride];
    v = sem::wave_sum(v);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += s_red[q];
    __syncthreads();
    return t;
}

#define GRID_LOOP(i, n) \
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)
// The same grid-stride loop with the workgroups in XCD order (sem::xcd_order):
// in every sweep each XCD takes one contiguous eighth, so the copies that
// neighbouring unique nodes gather from the same element lines meet in one L2.
#define GRID_LOOP_XCD(i, n)                                                                       \
    for (int64_t i = sem::xcd_order(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x; i < (n); \
         i += (int64_t)gridDim.x * blockDim.x)

// assembled value of unique node u: sum of its local copies, stored
// contiguously at wc[uoff[u] .. uoff[u+1]) (CSR order: the network's output).  The
// first eight copies (every node of a conforming hexahedral mesh) are loaded
// by independent predicated loads, issued together, and summed in CSR order;
// a longer segment continues in a loop.  The count of copies goes to *m.
template <typename T>
__device__ __forceinline__ T assemble(const T* __restrict__ wc, const int32_t* __restrict__ uoff,
                                      int64_t u, int32_t* m = nullptr) {
    const int32_t b = uoff[u], e = uoff[u + 1];
    T v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = b + q < e ? wc[b + q] : T(0);
    T s = v[0];
#pragma unroll
    for (int q = 1; q < 8; ++q)
        if (b + q < e) s += v[q];
    for (int32_t q = b + 8; q < e; ++q) s += wc[q];
    if (m) *m = e - b;
    return s;
}

using sem::assemble_local;

// out_u = (T) in_L at the first local copy of u (a continuous local field)
template <typename T>
__global__ void to_unique_kernel(T* __restrict__ out, const double* __restrict__ in,
                                 const int32_t* __restrict__ uoff, const int32_t* __restrict__ uidx,
                                 int64_t nu) {
    GRID_LOOP(u, nu) out[u] = (T)in[uidx[uoff[u]]];
}

// out_L = in_u[lid[L]] (0 on Dirichlet nodes, lid = -1)
__global__ void to_local_kernel(double* __restrict__ out, const double* __restrict__ in,
                                const int32_t* __restrict__ lid, int64_t n) {
    GRID_LOOP(L, n) {
        const int32_t u = lid[L];
        out[L] = u >= 0 ? in[u] : 0.0;
    }
}

// out_u = 1 / (sum of the copies of the element diagonal d_L)
template <typename T>
__global__ void assembled_recip_kernel(T* __restrict__ out, const double* __restrict__ d,
                                       const int32_t* __restrict__ uoff,
                                       const int32_t* __restrict__ uidx, int64_t nu) {
    GRID_LOOP(u, nu) {
        const int32_t b = uoff[u], e = uoff[u + 1];
        double s = 0.0;
        for (int32_t q = b; q < e; ++q) s += d[uidx[q]];
        out[u] = (T)(1.0 / s);
    }
}

// r = rhs, x = 0, p = Minv r; partials (r.Minv.r, r.r)
template <typename T>
__global__ void pcg_init_kernel(T* __restrict__ x, T* __restrict__ r, T* __restrict__ p,
                                const T* __restrict__ rhs, const T* __restrict__ minv, int64_t n,
                                double* __restrict__ part) {
    __shared__ double s_red[kBlock / 64];
    double a = 0.0, b = 0.0;
    GRID_LOOP(u, n) {
        const T rv = rhs[u];
        const T z = minv[u] * rv;
        x[u] = T(0);
        r[u] = rv;
        p[u] = z;
        a += (double)rv * (double)z;
        b += (double)rv * (double)rv;
    }
    a = block_sum(a, s_red);
    b = block_sum(b, s_red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

__global__ void pcg_init_final(Scal* __restrict__ S, const double* __restrict__ part, int n,
                               double tol, int maxit) {
    __shared__ double s_red[kFinal / 64];
    const double rz = final_sum(part, n, 2, s_red);
    const double bb = final_sum(part + 1, n, 2, s_red);
    if (threadIdx.x == 0) {
        S->rz = rz;
        S->bb = bb;
        S->tol2 = tol * tol * bb;
        S->it = 0;
        S->breakdown = 0;
        S->maxit = maxit;
        S->njac = 0;
        S->usej = 0;
        S->fallback = 0;
        S->delta2 = 0.0;
        S->rmax2 = bb;
        S->pause = 0;
        S->done = (bb == 0.0 || maxit <= 0) ? 1 : 0;
    }
}

__global__ void pcg_alpha_final(Scal* __restrict__ S, const double* __restrict__ part, int n) {
    if (S->done) return;
    __shared__ double s_red[kFinal / 64];
    const double pAp = final_sum(part, n, 1, s_red);
    if (threadIdx.x == 0) {
        S->pAp = pAp;
        if (!(pAp > 0.0) || !isfinite(pAp)) {
            S->breakdown = 1;
            S->done = 1;
        } else {
            S->alpha = S->rz / pAp;
        }
    }
}

// w_u = assembled w_L; x += alpha p, r -= alpha w; partials (r.Minv.r, r.r)
template <typename T>
__global__ void pcg_update_kernel(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p,
                                  const T* __restrict__ wl, const T* __restrict__ minv,
                                  const int32_t* __restrict__ uoff, const int32_t* __restrict__ uidx,
                                  int64_t n, const Scal* __restrict__ S, double* __restrict__ part) {
    if (S->done) return;
    __shared__ double s_red[kBlock / 64];
    const T alpha = (T)S->alpha;
    double a = 0.0, b = 0.0;
    GRID_LOOP_XCD(u, n) {
        const T wv = assemble_local(wl, uoff, uidx, u);
        x[u] += alpha * p[u];
        const T rv = r[u] - alpha * wv;
        r[u] = rv;
        a += (double)rv * (double)(minv[u] * rv);
        b += (double)rv * (double)rv;
    }
    a = block_sum(a, s_red);
    b = block_sum(b, s_red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

__global__ void pcg_beta_final(Scal* __restrict__ S, const double* __restrict__ part, int n) {
    if (S->done) return;
    __shared__ double s_red[kFinal / 64];
    const double rz = final_sum(part, n, 2, s_red);
    const double rr = final_sum(part + 1, n, 2, s_red);
    if (threadIdx.x == 0) {
        S->it += 1;
        S->rr = rr;
        S->beta = rz / S->rz;
        S->rz = rz;
        if (!isfinite(rr) || !isfinite(rz)) {
            S->breakdown = 1;
            S->done = 1;
        } else if (S->delta2 > 0.0 && (rr <= S->tol2 || rr < S->delta2 * S->rmax2)) {
            S->pause = 1;            // residual replacement due (or convergence to verify)
            S->done = 1;
        } else if (rr <= S->tol2 || S->it >= S->maxit) {
            S->done = 1;
        }
    }
}

// p = Minv r + beta p
template <typename T>
__global__ void pcg_p_kernel(T* __restrict__ p, const T* __restrict__ r, const T* __restrict__ minv,
                             int64_t n, const Scal* __restrict__ S) {
    if (S->done) return;
    const T beta = (T)S->beta;
    GRID_LOOP(u, n) p[u] = minv[u] * r[u] + beta * p[u];
}

// partials of (sum a, sum a*a)
template <typename T>
__global__ void sums_kernel(const T* __restrict__ a, int64_t n, double* __restrict__ part) {
    __shared__ double s_red[kBlock / 64];
    double s = 0.0, q = 0.0;
    GRID_LOOP(u, n) {
        const double v = (double)a[u];
        s += v;
        q += v * v;
    }
    s = block_sum(s, s_red);
    q = block_sum(q, s_red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s;
        part[2 * blockIdx.x + 1] = q;
    }
}

__global__ void sums_final(double* __restrict__ out, const double* __restrict__ part, int n) {
    __shared__ double s_red[kFinal / 64];
    const double s = final_sum(part, n, 2, s_red);
    const double q = final_sum(part + 1, n, 2, s_red);
    if (threadIdx.x == 0) {
        out[0] = s;
        out[1] = q;
    }
}

// x -= sums[0] / count
__global__ void sub_mean_kernel(double* __restrict__ x, const double* __restrict__ sums, double count,
                                int64_t n) {
    const double c = sums[0] / count;
    GRID_LOOP(u, n) x[u] -= c;
}

// r_u = b_u - assembled w_L
__global__ void residual_kernel(double* __restrict__ r, const double* __restrict__ b,
                                const double* __restrict__ wl, const int32_t* __restrict__ uoff,
                                const int32_t* __restrict__ uidx, int64_t nu) {
    GRID_LOOP_XCD(u, nu) r[u] = b[u] - assemble_local(wl, uoff, uidx, u);
}

// IR: rhat = (float)((r - mean) / norm), mean = s0 * inv_nu (inv_nu = 1 / nu on
// the singular periodic operator, 0 where no mean is projected),
// norm^2 = q - mean s0
__global__ void ir_scale_kernel(float* __restrict__ rhat, const double* __restrict__ r,
                                const double* __restrict__ sums, double inv_nu, int64_t n) {
    const double c = sums[0] * inv_nu;
    const double nrm2 = sums[1] - c * sums[0];
    const double inv = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
    GRID_LOOP(u, n) rhat[u] = (float)((r[u] - c) * inv);
}

// IR: x += norm * d (float64 update)
__global__ void ir_update_kernel(double* __restrict__ x, const float* __restrict__ d,
                                 const double* __restrict__ sums, double inv_nu, int64_t n) {
    const double c = sums[0] * inv_nu;
    const double nrm2 = sums[1] - c * sums[0];
    const double nrm = nrm2 > 0.0 ? sqrt(nrm2) : 0.0;
    GRID_LOOP(u, n) x[u] += nrm * (double)d[u];
}

// partials of sum_L owner_L x_L (float64 owner weights), for sem_remove_mean
__global__ void wsum_kernel(const double* __restrict__ x, const double* __restrict__ owner,
                            int64_t n, double* __restrict__ part) {
    __shared__ double s_red[kBlock / 64];
    double s = 0.0;
    GRID_LOOP(L, n) s += owner[L] * x[L];
    s = block_sum(s, s_red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void wsum_final(double* __restrict__ out, const double* __restrict__ part, int n) {
    __shared__ double s_red[kFinal / 64];
    const double s = final_sum(part, n, 1, s_red);
    if (threadIdx.x == 0) out[0] = s;
}

__global__ void add_kernel(double* __restrict__ x, const double* __restrict__ d, int64_t n) {
    GRID_LOOP(u, n) x[u] += d[u];
}

__global__ void zero_kernel(double* __restrict__ x, int64_t n) {
    GRID_LOOP(u, n) x[u] = 0.0;
}

template <typename T>
__global__ void to_type_kernel(T* __restrict__ out, const double* __restrict__ in, int64_t n) {
    GRID_LOOP(L, n) out[L] = (T)in[L];
}

__device__ inline uint16_t bf16_rne(float f) {
    uint32_t b = __float_as_uint(f);
    if ((b & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((b >> 16) | 0x40u);
    b += 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

__global__ void to_bf16_kernel(uint16_t* __restrict__ out, const double* __restrict__ in, int64_t n) {
    GRID_LOOP(L, n) out[L] = bf16_rne((float)in[L]);
}

// slice-blocked pair packing of the six factors (the layout of AxArgs::Gp):
// local node L = s + ij with s = e lx^3 + k lx^2; pair a at 2-vector 3 s + a lx^2 + ij
struct Six { const double* g[6]; int l2; };
template <typename T>
__device__ __forceinline__ T cvt(double v);
template <> __device__ __forceinline__ double cvt<double>(double v) { return v; }
template <> __device__ __forceinline__ float cvt<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ uint16_t cvt<uint16_t>(double v) { return bf16_rne((float)v); }

// the bfloat16 solver copy: per node the record (h1 g11, h1 g22, h1 g33,
// h1 g12, h1 g13, h1 g23), each product rounded float64 -> float32 -> bfloat16
// (h1 = 1 when the operator has none)
__global__ void pack_bf16_kernel(uint16_t* __restrict__ out, Six G, const double* __restrict__ h1, int64_t n) {
    GRID_LOOP(L, n) {
        const double h = h1 ? h1[L] : 1.0;
#pragma unroll
        for (int a = 0; a < 6; ++a) out[6 * L + a] = bf16_rne((float)(h * G.g[a][L]));
    }
}

template <typename T>
__global__ void pack_kernel(T* __restrict__ out, Six G, int64_t n) {
    GRID_LOOP(L, n) {
        const int64_t ij = L % G.l2, s = L - ij;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int64_t v = 3 * s + (int64_t)a * G.l2 + ij;
            out[2 * v] = cvt<T>(G.g[2 * a][L]);
            out[2 * v + 1] = cvt<T>(G.g[2 * a + 1][L]);
        }
    }
}

// ---- flexible CG (Notay's FCG(1)) with a variable preconditioner ----------
// partials: r.z, non-finite count of z, z.w_prev, (Minv r).w_prev
template <typename T>
__global__ void fcg_dots_kernel(const T* __restrict__ r, const T* __restrict__ z,
                                const T* __restrict__ wprev, const T* __restrict__ minv, int64_t n,
                                const Scal* __restrict__ S, double* __restrict__ part) {
    if (S->done) return;
    __shared__ double s_red[kBlock / 64];
    const bool first = S->it == 0;
    double rz = 0.0, bad = 0.0, zw = 0.0, jw = 0.0;
    GRID_LOOP(u, n) {
        const double zv = (double)z[u];
        const double rv = (double)r[u];
        if (!isfinite(zv)) bad += 1.0;
        rz += rv * zv;
        if (!first) {
            const double wv = (double)wprev[u];
            zw += zv * wv;
            jw += (double)(minv[u] * r[u]) * wv;
        }
    }
    rz = block_sum(rz, s_red);
    bad = block_sum(bad, s_red);
    zw = block_sum(zw, s_red);
    jw = block_sum(jw, s_red);
    if (threadIdx.x == 0) {
        part[4 * blockIdx.x] = rz;
        part[4 * blockIdx.x + 1] = bad;
        part[4 * blockIdx.x + 2] = zw;
        part[4 * blockIdx.x + 3] = jw;
    }
}

// the same partials, with z assembled here from the network's CSR-ordered
// element contributions: z_u = mult_u^-1/2 sum_segment zl (+ Minv_u r_u), written out
template <typename T>
__global__ void fcg_dots_asm_kernel(T* __restrict__ z, const float* __restrict__ zl,
                                    const int32_t* __restrict__ uoff, const T* __restrict__ r,
                                    const T* __restrict__ wprev, const T* __restrict__ minv, bool jbase,
                                    int64_t n, const Scal* __restrict__ S, double* __restrict__ part) {
    if (S->done) return;
    __shared__ double s_red[kBlock / 64];
    const bool first = S->it == 0;
    double rz = 0.0, bad = 0.0, zw = 0.0, jw = 0.0;
    GRID_LOOP(u, n) {
        int32_t m;
        const float s = assemble(zl, uoff, u, &m);
        const T rt = r[u], mv = minv[u];
        double zd = (double)s * rsqrt((double)m);
        if (jbase) zd += (double)mv * (double)rt;
        const T zt = (T)zd;
        z[u] = zt;
        const double zv = (double)zt, rv = (double)rt;
        if (!isfinite(zv)) bad += 1.0;
        rz += rv * zv;
        if (!first) {
            const double wv = (double)wprev[u];
            zw += zv * wv;
            jw += (double)(mv * rt) * wv;
        }
    }
    rz = block_sum(rz, s_red);
    bad = block_sum(bad, s_red);
    zw = block_sum(zw, s_red);
    jw = block_sum(jw, s_red);
    if (threadIdx.x == 0) {
        part[4 * blockIdx.x] = rz;
        part[4 * blockIdx.x + 1] = bad;
        part[4 * blockIdx.x + 2] = zw;
        part[4 * blockIdx.x + 3] = jw;
    }
}

__global__ void fcg_gamma_final(Scal* __restrict__ S, const double* __restrict__ part, int n) {
    if (S->done) return;
    __shared__ double s_red[kFinal / 64];
    const double rz = final_sum(part, n, 4, s_red);
    const double bad = final_sum(part + 1, n, 4, s_red);
    const double zw = final_sum(part + 2, n, 4, s_red);
    const double jw = final_sum(part + 3, n, 4, s_red);
    if (threadIdx.x == 0) {
        const int usej = (S->fallback || bad > 0.0 || !(rz > 0.0) || !isfinite(zw)) ? 1 : 0;
        S->usej = usej;
        S->njac += usej;
        S->beta = S->it == 0 ? 0.0 : (usej ? jw : zw) / S->pw_prev;   // gamma of FCG(1)
    }
}

// p = z_eff - gamma p (z_eff = Minv r when the network output is rejected); partials p.r
template <typename T>
__global__ void fcg_p_kernel(T* __restrict__ p, const T* __restrict__ z, const T* __restrict__ r,
                             const T* __restrict__ minv, int64_t n, const Scal* __restrict__ S,
                             double* __restrict__ part) {
    if (S->done) return;
    __shared__ double s_red[kBlock / 64];
    const bool usej = S->usej != 0;
    const bool first = S->it == 0;
    const T gamma = (T)S->beta;
    double pr = 0.0;
    GRID_LOOP(u, n) {
        const T rv = r[u];
        const T ze = usej ? minv[u] * rv : z[u];
        const T pv = first ? ze : ze - gamma * p[u];
        p[u] = pv;
        pr += (double)pv * (double)rv;
    }
    pr = block_sum(pr, s_red);
    if (threadIdx.x == 0) part[blockIdx.x] = pr;
}

// alpha = p.r / p.A.p; keep p.A.p for the next gamma
__global__ void fcg_alpha_final(Scal* __restrict__ S, const double* __restrict__ part_ax, int nax,
                                const double* __restrict__ part_pr, int npr) {
    if (S->done) return;
    __shared__ double s_red[kFinal / 64];
    const double pAp = final_sum(part_ax, nax, 1, s_red);
    const double pr = final_sum(part_pr, npr, 1, s_red);
    if (threadIdx.x == 0) {
        S->pAp = pAp;
        if (!(pAp > 0.0) || !isfinite(pAp) || !isfinite(pr)) {
            S->breakdown = 1;
            S->done = 1;
        } else {
            S->alpha = pr / pAp;
            S->pw_prev = pAp;
        }
    }
}

// FCG keeps the assembled w of the previous iteration: w_u = assembled w_L,
// then x += alpha p, r -= alpha w_u; partials (r.Minv.r, r.r)
template <typename T>
__global__ void fcg_update_kernel(T* __restrict__ x, T* __restrict__ r, T* __restrict__ wu,
                                  const T* __restrict__ p, const T* __restrict__ wl,
                                  const T* __restrict__ minv, const int32_t* __restrict__ uoff,
                                  const int32_t* __restrict__ uidx, int64_t n,
                                  const Scal* __restrict__ S, double* __restrict__ part) {
    if (S->done) return;
    __shared__ double s_red[kBlock / 64];
    const T alpha = (T)S->alpha;
    double a = 0.0, b = 0.0;
    GRID_LOOP_XCD(u, n) {
        const T wv = assemble_local(wl, uoff, uidx, u);
        wu[u] = wv;
        x[u] += alpha * p[u];
        const T rv = r[u] - alpha * wv;
        r[u] = rv;
        a += (double)rv * (double)(minv[u] * rv);
        b += (double)rv * (double)rv;
    }
    a = block_sum(a, s_red);
    b = block_sum(b, s_red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

// residual replacement: x64 += xl, xl = 0 (float64 accumulation of the
// low-precision update)
__global__ void rr_accumulate_kernel(double* __restrict__ x64, float* __restrict__ xl, int64_t n) {
    GRID_LOOP(u, n) {
        x64[u] += (double)xl[u];
        xl[u] = 0.f;
    }
}

// r = (float) r64; partials (r.Minv.r, r.r) in float64 from the float values
__global__ void rr_replace_kernel(float* __restrict__ r, const double* __restrict__ r64,
                                  const float* __restrict__ minv, int64_t n, double* __restrict__ part) {
    __shared__ double s_red[kBlock / 64];
    double a = 0.0, b = 0.0;
    GRID_LOOP(u, n) {
        const float rv = (float)r64[u];
        r[u] = rv;
        a += (double)rv * (double)(minv[u] * rv);
        b += (double)rv * (double)rv;
    }
    a = block_sum(a, s_red);
    b = block_sum(b, s_red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

// resume after a replacement: rz from the new residual, rmax = its norm
__global__ void rr_resume_final(Scal* __restrict__ S, const double* __restrict__ part, int n) {
    __shared__ double s_red[kFinal / 64];
    const double rz = final_sum(part, n, 2, s_red);
    const double rr = final_sum(part + 1, n, 2, s_red);
    if (threadIdx.x == 0) {
        S->rz = rz;
        S->rr = rr;
        S->rmax2 = rr;
        S->pause = 0;
        S->done = (S->it >= S->maxit) ? 1 : 0;
    }
}

__global__ void set_delta(Scal* __restrict__ S, double delta2) {
    if (threadIdx.x == 0 && blockIdx.x == 0) S->delta2 = delta2;
}

__global__ void set_fallback(Scal* __restrict__ S) {
    if (threadIdx.x == 0 && blockIdx.x == 0) S->fallback = 1;
}

}  // namespace

// One precision level of the solver: unique-node vectors of type T (x, r, p,
// Minv, and for flexible CG z and the assembled w), the element-local operator
// output wl (n_local), and the operator form that acts on them.
struct Level {
    sem::AxKind kind;
    sem::AxArgs A;
    void *x = nullptr, *r = nullptr, *p = nullptr, *wl = nullptr, *minv = nullptr;
    void *z = nullptr, *wu = nullptr;
};

struct sem_cg_s {
    sem_ctx_t ctx = nullptr;
    sem_gs_t gs = nullptr;
    int precision = SEM_SOLVE_F64;
    int64_t n = 0;                 // local nodes
    int64_t nu = 0;                // unique nodes
    sem::AxArgs A64{};
    Scal* S = nullptr;
    double* part = nullptr;        // max(4*kGrid, ax_blocks) doubles
    double* part2 = nullptr;       // kGrid doubles (flexible CG: p.r partials)
    double* sums = nullptr;        // 2 doubles
    Scal* S_host = nullptr;        // pinned
    double* sums_host = nullptr;   // pinned
    Level lv64{}, lv32{};
    double *b64 = nullptr, *x64 = nullptr, *r64 = nullptr;   // unique float64
    double* d64 = nullptr;         // float64 solves: correction after a true-residual check
    double* wl64 = nullptr;                                    // local float64
    float* rhs32 = nullptr;        // IR: normalised inner right-hand side (unique)
    sem_lp_t lp = nullptr;
    sem_mg_t mg = nullptr;         // multigrid V-cycle (flexible CG), or null
    std::vector<void*> allocs;
};

namespace {

// The periodic Poisson operator is singular (null space: the constants), so
// its solves project out the mean; with Dirichlet nodes or a Helmholtz mass
// term the operator is positive definite.
inline bool projects(sem_cg_t cg) { return cg->gs->n_masked == 0 && !cg->A64.hb; }

// flexible CG runs whenever a preconditioner other than Jacobi is bound
inline bool flexible(sem_cg_t cg) { return cg->lp || cg->mg; }

int cg_alloc(sem_cg_t cg, void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return sem::check_hip(cg->ctx, e, "sem_cg_setup: hipMalloc");
    cg->allocs.push_back(*p);
    return SEM_OK;
}

unsigned vec_grid(int64_t n, int cap = kGrid) {
    int64_t b = (n + kBlock - 1) / kBlock;
    return (unsigned)(b < cap ? (b < 1 ? 1 : b) : cap);
}

template <typename T>
unsigned vec_grid_t(int64_t n) { return vec_grid(n, sizeof(T) == 8 ? kGrid : kGrid32); }

// PCG on level lv from x = 0 with right-hand side rhs (unique, type T);
// leaves the iterate in lv.x.
template <typename T>
int pcg_run(sem_cg_t cg, Level& lv, const T* rhs, double tol, int maxit, int check_every,
            int* iters_out, int* breakdown_out) {
    sem_ctx_t ctx = cg->ctx;
    hipStream_t st = ctx->stream;
    const int64_t n = cg->nu;
    const unsigned g = vec_grid_t<T>(n);
    T* x = (T*)lv.x; T* r = (T*)lv.r; T* p = (T*)lv.p; T* wl = (T*)lv.wl;
    const T* minv = (const T*)lv.minv;
    const int32_t *lid = cg->gs->lid, *uoff = cg->gs->uoff, *uidx = cg->gs->uidx;
    pcg_init_kernel<T><<<g, kBlock, 0, st>>>(x, r, p, rhs, minv, n, cg->part);
    pcg_init_final<<<1, kFinal, 0, st>>>(cg->S, cg->part, (int)g, tol, maxit);
    SEM_LAUNCH_CHECK(ctx);
    const int nb = sem::ax_blocks(lv.A.lx, lv.A.nel);
    for (;;) {
        for (int q = 0; q < check_every; ++q) {
            int rc = sem::launch_ax(ctx, lv.kind, lv.A, wl, p, &cg->S->done, cg->part, lid);
            if (rc) return rc;
            pcg_alpha_final<<<1, kFinal, 0, st>>>(cg->S, cg->part, nb);
            pcg_update_kernel<T><<<g, kBlock, 0, st>>>(x, r, p, wl, minv, uoff, uidx, n, cg->S, cg->part);
            pcg_beta_final<<<1, kFinal, 0, st>>>(cg->S, cg->part, (int)g);
            pcg_p_kernel<T><<<g, kBlock, 0, st>>>(p, r, minv, n, cg->S);
        }
        SEM_LAUNCH_CHECK(ctx);
        SEM_HIP(ctx, hipMemcpyAsync(cg->S_host, cg->S, sizeof(Scal), hipMemcpyDeviceToHost, st));
        SEM_HIP(ctx, hipStreamSynchronize(st));
        if (cg->S_host->done) break;
    }
    *iters_out = cg->S_host->it;
    *breakdown_out = cg->S_host->breakdown;
    return SEM_OK;
}

int residual64(sem_cg_t cg, const double* xu);
template <typename T> int vec_sums(sem_cg_t cg, const T* a);
int read_sums(sem_cg_t cg, double* s, double* q);

// stagnation guard of the network: records (iteration, r.r) and reports
// whether r.r has failed to fall by 4x (the relative residual to halve) over
// the last 256 iterations
bool stagnated(std::vector<std::pair<int, double>>& hist, int it, double rr) {
    hist.emplace_back(it, rr);
    for (auto q = hist.rbegin(); q != hist.rend(); ++q)
        if (it - q->first >= 256) return rr > 0.25 * q->second;
    return false;
}

// z = P(r) for one flexible-CG iteration and the partials of fcg_gamma_final:
// the multigrid V-cycle, or the network (its linear form assembles z inside
// the dot kernel).  After the solve has fallen back, the kernels take the
// Jacobi z themselves (S->fallback) and no preconditioner runs.
template <typename T>
int precondition(sem_cg_t cg, T* z, const T* r, const T* wu, const T* minv, bool fallen, unsigned g) {
    hipStream_t st = cg->ctx->stream;
    const int64_t n = cg->nu;
    const int* skip = &cg->S->done;
    const bool f64 = sizeof(T) == 8;
    int rc = SEM_OK;
    if (!fallen && cg->mg) {
        rc = sem::mg_apply(cg->mg, z, r, f64, skip);
    } else if (!fallen) {
        const float* zl = nullptr;
        bool jb = false;
        rc = sem::lp_apply_partial(cg->lp, r, f64, skip, &zl, &jb);
        if (rc == SEM_OK) {
            fcg_dots_asm_kernel<T><<<g, kBlock, 0, st>>>(z, zl, cg->gs->uoff, r, wu, minv, jb, n, cg->S, cg->part);
            SEM_LAUNCH_CHECK(cg->ctx);
            return SEM_OK;
        }
        rc = sem::lp_apply(cg->lp, z, r, f64, skip, true);    // the nonlinear network
    }
    if (rc) return rc;
    fcg_dots_kernel<T><<<g, kBlock, 0, st>>>(r, z, wu, minv, n, cg->S, cg->part);
    SEM_LAUNCH_CHECK(cg->ctx);
    return SEM_OK;
}

// Mixed-precision CG with residual replacement (reliable updates; Strzodka
// and Goeddeke 2006, Clark et al. 2010): float32 vectors and the reduced
// operator drive the Krylov iteration; whenever the float32 residual has
// fallen by `delta` since the last replacement, the accumulated update is
// added to the float64 x, the residual is replaced by the float64 b - A x, and
// the iteration continues with the same search direction.  Converged when
// the replaced float64 residual meets tol.
int rr_run(sem_cg_t cg, Level& lv, double tol, double delta, int maxit, int check_every,
           double bnorm, int* iters_out, int* replacements, int* breakdown_out, double* hist, int nhist,
           int* njac_out, int* fell_back) {
    sem_ctx_t ctx = cg->ctx;
    hipStream_t st = ctx->stream;
    const int64_t n = cg->nu;
    const unsigned g = vec_grid_t<float>(n);
    float* x = (float*)lv.x; float* r = (float*)lv.r; float* p = (float*)lv.p; float* wl = (float*)lv.wl;
    const float* minv = (const float*)lv.minv;
    const int32_t *lid = cg->gs->lid, *uoff = cg->gs->uoff, *uidx = cg->gs->uidx;
    // x64 = 0, r64 = b; inner start: x = 0, r = (float) b, p = Minv r
    zero_kernel<<<g, kBlock, 0, st>>>(cg->x64, n);
    rr_replace_kernel<<<g, kBlock, 0, st>>>(cg->rhs32, cg->b64, minv, n, cg->part);
    pcg_init_kernel<float><<<g, kBlock, 0, st>>>(x, r, p, cg->rhs32, minv, n, cg->part);
    pcg_init_final<<<1, kFinal, 0, st>>>(cg->S, cg->part, (int)g, tol, maxit);
    set_delta<<<1, 1, 0, st>>>(cg->S, delta * delta);
    SEM_LAUNCH_CHECK(ctx);
    const int nb = sem::ax_blocks(lv.A.lx, lv.A.nel);
    int nrep = 0;
    float* z = (float*)lv.z;
    float* wu = (float*)lv.wu;
    bool fallen = false;
    std::vector<std::pair<int, double>> rr_hist;
    for (;;) {
        for (int q = 0; q < check_every; ++q) {
            if (flexible(cg)) {   // flexible CG step (Jacobi where the output is rejected)
                int rc = precondition<float>(cg, z, r, wu, minv, fallen, g);
                if (rc) return rc;
                fcg_gamma_final<<<1, kFinal, 0, st>>>(cg->S, cg->part, (int)g);
                fcg_p_kernel<float><<<g, kBlock, 0, st>>>(p, z, r, minv, n, cg->S, cg->part2);
                rc = sem::launch_ax(ctx, lv.kind, lv.A, wl, p, &cg->S->done, cg->part, lid);
                if (rc) return rc;
                fcg_alpha_final<<<1, kFinal, 0, st>>>(cg->S, cg->part, nb, cg->part2, (int)g);
                fcg_update_kernel<float><<<g, kBlock, 0, st>>>(x, r, wu, p, wl, minv, uoff, uidx, n, cg->S,
                                                               cg->part);
                pcg_beta_final<<<1, kFinal, 0, st>>>(cg->S, cg->part, (int)g);
                continue;
            }
            int rc = sem::launch_ax(ctx, lv.kind, lv.A, wl, p, &cg->S->done, cg->part, lid);
            if (rc) return rc;
            pcg_alpha_final<<<1, kFinal, 0, st>>>(cg->S, cg->part, nb);
            pcg_update_kernel<float><<<g, kBlock, 0, st>>>(x, r, p, wl, minv, uoff, uidx, n, cg->S, cg->part);
            pcg_beta_final<<<1, kFinal, 0, st>>>(cg->S, cg->part, (int)g);
            pcg_p_kernel<float><<<g, kBlock, 0, st>>>(p, r, minv, n, cg->S);
        }
        SEM_LAUNCH_CHECK(ctx);
        SEM_HIP(ctx, hipMemcpyAsync(cg->S_host, cg->S, sizeof(Scal), hipMemcpyDeviceToHost, st));
        SEM_HIP(ctx, hipStreamSynchronize(st));
        const Scal& H = *cg->S_host;
        if (!H.done) {
            if (flexible(cg) && !fallen && stagnated(rr_hist, H.it, H.rr)) {
                set_fallback<<<1, 1, 0, st>>>(cg->S);      // Jacobi for good
                SEM_LAUNCH_CHECK(ctx);
                fallen = true;
            }
            continue;
        }
        if (H.breakdown) break;
        // replacement: fold the update into x64, recompute the float64 residual
        rr_accumulate_kernel<<<g, kBlock, 0, st>>>(cg->x64, x, n);
        SEM_LAUNCH_CHECK(ctx);
        int rc = residual64(cg, cg->x64);
        if (rc) return rc;
        rc = vec_sums(cg, cg->r64);
        if (rc) return rc;
        double s0, q0;
        rc = read_sums(cg, &s0, &q0);
        if (rc) return rc;
        const double rel = bnorm > 0 ? std::sqrt(q0) / bnorm : 0.0;
        if (nrep < nhist) hist[nrep] = rel;
        ++nrep;
        if (rel <= tol || H.it >= maxit) break;
        // the float64 residual carries the (tiny) mean that rounding left; drop it
        if (projects(cg)) sub_mean_kernel<<<g, kBlock, 0, st>>>(cg->r64, cg->sums, (double)n, n);
        rr_replace_kernel<<<g, kBlock, 0, st>>>(r, cg->r64, minv, n, cg->part);
        rr_resume_final<<<1, kFinal, 0, st>>>(cg->S, cg->part, (int)g);
        // PCG: the paused iteration skipped its direction update, redone with
        // the replaced residual and that iteration's beta (flexible CG forms
        // its direction at the start of the next iteration instead)
        if (!flexible(cg)) pcg_p_kernel<float><<<g, kBlock, 0, st>>>(p, r, minv, n, cg->S);
        SEM_LAUNCH_CHECK(ctx);
    }
    *iters_out = cg->S_host->it;
    *replacements = nrep;
    *breakdown_out = cg->S_host->breakdown;
    *njac_out = cg->S_host->njac;
    *fell_back = fallen ? 1 : 0;
    return SEM_OK;
}

// flexible CG on level lv with the bound network; same contract as pcg_run
template <typename T>
int fcg_run(sem_cg_t cg, Level& lv, const T* rhs, double tol, int maxit, int check_every,
            int* iters_out, int* breakdown_out, int* njac_out, int* fell_back) {
    sem_ctx_t ctx = cg->ctx;
    hipStream_t st = ctx->stream;
    const int64_t n = cg->nu;
    const unsigned g = vec_grid_t<T>(n);
    T* x = (T*)lv.x; T* r = (T*)lv.r; T* p = (T*)lv.p; T* wl = (T*)lv.wl; T* z = (T*)lv.z;
    T* wu = (T*)lv.wu;
    const T* minv = (const T*)lv.minv;
    const int32_t *lid = cg->gs->lid, *uoff = cg->gs->uoff, *uidx = cg->gs->uidx;
    pcg_init_kernel<T><<<g, kBlock, 0, st>>>(x, r, p, rhs, minv, n, cg->part);
    pcg_init_final<<<1, kFinal, 0, st>>>(cg->S, cg->part, (int)g, tol, maxit);
    SEM_LAUNCH_CHECK(ctx);
    const int nb = sem::ax_blocks(lv.A.lx, lv.A.nel);
    const bool f64 = sizeof(T) == 8;
    bool fallen = false;
    std::vector<std::pair<int, double>> hist;   // (iteration, r.r) at each check
    for (;;) {
        for (int q = 0; q < check_every; ++q) {
            int rc = precondition<T>(cg, z, r, wu, minv, fallen, g);
            if (rc) return rc;
            fcg_gamma_final<<<1, kFinal, 0, st>>>(cg->S, cg->part, (int)g);
            fcg_p_kernel<T><<<g, kBlock, 0, st>>>(p, z, r, minv, n, cg->S, cg->part2);
            rc = sem::launch_ax(ctx, lv.kind, lv.A, wl, p, &cg->S->done, cg->part, lid);
            if (rc) return rc;
            fcg_alpha_final<<<1, kFinal, 0, st>>>(cg->S, cg->part, nb, cg->part2, (int)g);
            fcg_update_kernel<T><<<g, kBlock, 0, st>>>(x, r, wu, p, wl, minv, uoff, uidx, n, cg->S, cg->part);
            pcg_beta_final<<<1, kFinal, 0, st>>>(cg->S, cg->part, (int)g);
        }
        SEM_LAUNCH_CHECK(ctx);
        SEM_HIP(ctx, hipMemcpyAsync(cg->S_host, cg->S, sizeof(Scal), hipMemcpyDeviceToHost, st));
        SEM_HIP(ctx, hipStreamSynchronize(st));
        if (cg->S_host->done) break;
        if (!fallen && stagnated(hist, cg->S_host->it, cg->S_host->rr)) {
            set_fallback<<<1, 1, 0, st>>>(cg->S);
            SEM_LAUNCH_CHECK(ctx);
            fallen = true;
        }
    }
    *iters_out = cg->S_host->it;
    *breakdown_out = cg->S_host->breakdown;
    *njac_out = cg->S_host->njac;
    *fell_back = fallen ? 1 : 0;
    return SEM_OK;
}

// sums of (a, a*a) over the unique vector a into cg->sums (device)
template <typename T>
int vec_sums(sem_cg_t cg, const T* a) {
    const unsigned g = vec_grid(cg->nu);
    sums_kernel<T><<<g, kBlock, 0, cg->ctx->stream>>>(a, cg->nu, cg->part);
    sums_final<<<1, kFinal, 0, cg->ctx->stream>>>(cg->sums, cg->part, (int)g);
    SEM_LAUNCH_CHECK(cg->ctx);
    return SEM_OK;
}

int read_sums(sem_cg_t cg, double* s, double* q) {
    SEM_HIP(cg->ctx, hipMemcpyAsync(cg->sums_host, cg->sums, 2 * sizeof(double),
                                    hipMemcpyDeviceToHost, cg->ctx->stream));
    SEM_HIP(cg->ctx, hipStreamSynchronize(cg->ctx->stream));
    *s = cg->sums_host[0];
    *q = cg->sums_host[1];
    return SEM_OK;
}

// r64 = b64 - A x (unique, float64)
int residual64(sem_cg_t cg, const double* xu) {
    int rc = sem::launch_ax(cg->ctx, sem::AxKind::F64, cg->A64, cg->wl64, xu, nullptr, nullptr, cg->gs->lid);
    if (rc) return rc;
    residual_kernel<<<vec_grid(cg->nu), kBlock, 0, cg->ctx->stream>>>(cg->r64, cg->b64, cg->wl64,
                                                                      cg->gs->uoff, cg->gs->uidx, cg->nu);
    SEM_LAUNCH_CHECK(cg->ctx);
    return SEM_OK;
}

int remove_mean_u(sem_cg_t cg, double* xu) {
    if (!projects(cg)) return SEM_OK;
    int rc = vec_sums(cg, xu);
    if (rc) return rc;
    sub_mean_kernel<<<vec_grid(cg->nu), kBlock, 0, cg->ctx->stream>>>(xu, cg->sums, (double)cg->nu, cg->nu);
    SEM_LAUNCH_CHECK(cg->ctx);
    return SEM_OK;
}

}  // namespace

namespace sem {

void pack_factors_f32(hipStream_t st, float* out, const double* const* G, int64_t n, int lx) {
    Six six;
    for (int q = 0; q < 6; ++q) six.g[q] = G[q];
    six.l2 = lx * lx;
    pack_kernel<float><<<vec_grid(n), kBlock, 0, st>>>(out, six, n);
}

void pack_factors_bf16(hipStream_t st, uint16_t* out, const double* const* G, const double* h1, int64_t n,
                       int lx) {
    Six six;
    for (int q = 0; q < 6; ++q) six.g[q] = G[q];
    six.l2 = lx * lx;
    pack_bf16_kernel<<<vec_grid(n), kBlock, 0, st>>>(out, six, h1, n);
}

}  // namespace sem

extern "C" int sem_cg_setup(sem_ctx_t ctx, sem_gs_t gs, const sem_operator_t* A,
                            const sem_solve_opts_t* opts, sem_cg_t* out) {
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (!out || !gs || !A || !opts) return sem::fail(ctx, SEM_EINVAL, "sem_cg_setup: null argument");
    *out = nullptr;
    if (gs->ctx != ctx) return sem::fail(ctx, SEM_EINVAL, "sem_cg_setup: plan belongs to another context");
    if (!sem::lx_ok(A->lx)) return sem::fail(ctx, SEM_EUNSUPPORTED_LX, "sem_cg_setup: lx=%d", A->lx);
    const int64_t n = A->nel * A->lx * A->lx * A->lx;
    if (A->nel <= 0 || n != gs->n_local)
        return sem::fail(ctx, SEM_EINVAL, "sem_cg_setup: operator size %lld does not match plan %lld",
                         (long long)n, (long long)gs->n_local);
    const double* Dp[6] = {A->dx, A->dy, A->dz, A->dxt, A->dyt, A->dzt};
    const double* Gp[6] = {A->g11, A->g22, A->g33, A->g12, A->g13, A->g23};
    for (int q = 0; q < 6; ++q)
        if (!Dp[q] || !Gp[q]) return sem::fail(ctx, SEM_EINVAL, "sem_cg_setup: null operator array");
    if (opts->precision < SEM_SOLVE_F64 || opts->precision > SEM_SOLVE_BF16_IR)
        return sem::fail(ctx, SEM_EINVAL, "sem_cg_setup: bad precision %d", opts->precision);
    if (gs->n_unique == 0) return sem::fail(ctx, SEM_EINVAL, "sem_cg_setup: the plan has no unknowns");

    auto* cg = new sem_cg_s();
    cg->ctx = ctx;
    cg->gs = gs;
    cg->precision = opts->precision;
    cg->n = n;
    cg->nu = gs->n_unique;
    for (int q = 0; q < 6; ++q) { cg->A64.D[q] = Dp[q]; cg->A64.G[q] = Gp[q]; }
    cg->A64.h1 = A->h1;
    cg->A64.hb = A->h2b;
    cg->A64.nel = A->nel;
    cg->A64.lx = A->lx;
    hipStream_t st = ctx->stream;
    const int64_t nu = cg->nu;
    const unsigned gl = vec_grid(n), gu = vec_grid(nu);
    const int nb = sem::ax_blocks(A->lx, A->nel);
    const size_t npart = (size_t)std::max(4 * kGrid, nb);
    const size_t u64 = sizeof(double) * nu, u32 = sizeof(float) * nu;
    auto bail = [&](int code) { sem_cg_destroy(cg); return code; };
#define CG_ALLOC(ptr, bytes) do { int rc_ = cg_alloc(cg, (void**)&(ptr), (bytes)); if (rc_) return bail(rc_); } while (0)
    CG_ALLOC(cg->S, sizeof(Scal));
    CG_ALLOC(cg->part, sizeof(double) * npart);
    CG_ALLOC(cg->part2, sizeof(double) * kGrid);
    CG_ALLOC(cg->sums, sizeof(double) * 2);
    CG_ALLOC(cg->b64, u64);
    CG_ALLOC(cg->x64, u64);
    CG_ALLOC(cg->r64, u64);
    CG_ALLOC(cg->wl64, sizeof(double) * n);
    Six six;
    for (int q = 0; q < 6; ++q) six.g[q] = Gp[q];
    six.l2 = A->lx * A->lx;
    {
        void* gp = nullptr;
        CG_ALLOC(gp, sizeof(double) * 6 * n);
        pack_kernel<double><<<gl, kBlock, 0, st>>>((double*)gp, six, n);
        cg->A64.Gp = gp;
    }
    {
        hipError_t e = hipHostMalloc(&cg->S_host, sizeof(Scal), hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc(&cg->sums_host, 2 * sizeof(double), hipHostMallocDefault);
        if (e != hipSuccess) return bail(sem::check_hip(ctx, e, "sem_cg_setup: hipHostMalloc"));
    }
    if (opts->learned && opts->mg)
        return bail(sem::fail(ctx, SEM_EINVAL, "sem_cg_setup: learned and mg preconditioners are exclusive"));
    if (opts->mg) {
        if (sem::mg_nel(opts->mg) != A->nel || sem::mg_plan(opts->mg) != gs)
            return bail(sem::fail(ctx, SEM_EINVAL, "sem_cg_setup: the multigrid hierarchy is not built on this operator and plan"));
        cg->mg = opts->mg;
    }
    if (opts->learned) {
        if (sem::lp_rows(opts->learned) != A->nel || sem::lp_plan(opts->learned) != gs)
            return bail(sem::fail(ctx, SEM_EINVAL, "sem_cg_setup: the network is not bound to this operator and plan"));
        cg->lp = opts->learned;
    }
    // element diagonal (local, float64) in wl64; assembled and inverted per level below
    rc = sem_ax_diag(ctx, cg->wl64, A->dx, A->h1, A->g11, A->g22, A->g33, A->g12, A->g13, A->g23,
                     A->nel, A->lx);
    if (rc) return bail(rc);
    if (A->h2b) add_kernel<<<gl, kBlock, 0, st>>>(cg->wl64, A->h2b, n);   // + the diagonal mass term

    Level& L64 = cg->lv64;
    L64.kind = sem::AxKind::F64;
    L64.A = cg->A64;
    if (opts->precision == SEM_SOLVE_F64) {
        CG_ALLOC(L64.r, u64); CG_ALLOC(L64.p, u64); CG_ALLOC(L64.minv, u64);
        L64.x = cg->x64;
        L64.wl = cg->wl64;
        if (flexible(cg)) { CG_ALLOC(L64.z, u64); CG_ALLOC(L64.wu, u64); }
        CG_ALLOC(cg->d64, u64);
        assembled_recip_kernel<double><<<gu, kBlock, 0, st>>>((double*)L64.minv, cg->wl64, gs->uoff, gs->uidx, nu);
    } else {
        Level& L = cg->lv32;
        const bool bf = opts->precision == SEM_SOLVE_BF16_IR;
        L.kind = bf ? sem::AxKind::F32_BF16 : sem::AxKind::F32;
        CG_ALLOC(L.x, u32); CG_ALLOC(L.r, u32); CG_ALLOC(L.p, u32); CG_ALLOC(L.minv, u32);
        CG_ALLOC(L.wl, sizeof(float) * n);
        CG_ALLOC(cg->rhs32, u32);
        if (flexible(cg)) { CG_ALLOC(L.z, u32); CG_ALLOC(L.wu, u32); }
        assembled_recip_kernel<float><<<gu, kBlock, 0, st>>>((float*)L.minv, cg->wl64, gs->uoff, gs->uidx, nu);
        const int l2 = A->lx * A->lx;
        for (int q = 0; q < 6; ++q) {
            void* d = nullptr;
            CG_ALLOC(d, sizeof(float) * l2);
            to_type_kernel<float><<<1, kBlock, 0, st>>>((float*)d, Dp[q], l2);
            L.A.D[q] = d;
        }
        const size_t vs = bf ? sizeof(uint16_t) : sizeof(float);
        L.A.h1 = nullptr;
        for (int q = 0; q < 6; ++q) L.A.G[q] = nullptr;     // the solver form reads the packed copy
        {
            void* d = nullptr;
            CG_ALLOC(d, vs * 6 * n);
            if (bf) pack_bf16_kernel<<<gl, kBlock, 0, st>>>((uint16_t*)d, six, A->h1, n);   // h1 folded in
            else pack_kernel<float><<<gl, kBlock, 0, st>>>((float*)d, six, n);
            L.A.Gp = d;
        }
        if (A->h1 && !bf) {
            void* d = nullptr;
            CG_ALLOC(d, vs * n);
            to_type_kernel<float><<<gl, kBlock, 0, st>>>((float*)d, A->h1, n);
            L.A.h1 = d;
        }
        if (A->h2b) {          // the mass term in the storage type of h1 and G
            void* d = nullptr;
            CG_ALLOC(d, vs * n);
            if (bf) to_bf16_kernel<<<gl, kBlock, 0, st>>>((uint16_t*)d, A->h2b, n);
            else to_type_kernel<float><<<gl, kBlock, 0, st>>>((float*)d, A->h2b, n);
            L.A.hb = d;
        }
        L.A.nel = A->nel;
        L.A.lx = A->lx;
    }
#undef CG_ALLOC
    SEM_LAUNCH_CHECK(ctx);
    SEM_HIP(ctx, hipStreamSynchronize(st));
    *out = cg;
    return SEM_OK;
}

extern "C" int sem_cg_destroy(sem_cg_t cg) {
    if (!cg) return SEM_OK;
    if (cg->ctx) {
        (void)hipSetDevice(cg->ctx->device);
        (void)hipStreamSynchronize(cg->ctx->stream);
    }
    for (void* p : cg->allocs) (void)hipFree(p);
    if (cg->S_host) (void)hipHostFree(cg->S_host);
    if (cg->sums_host) (void)hipHostFree(cg->sums_host);
    delete cg;
    return SEM_OK;
}

extern "C" int sem_cg_solve(sem_cg_t cg, double* x, const double* b, const sem_solve_opts_t* opts,
                            sem_solve_stats_t* stats) {
    if (!cg) return sem::fail(nullptr, SEM_EINVAL, "sem_cg_solve: null solver");
    sem_ctx_t ctx = cg->ctx;
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (!x || !b || !opts || !stats) return sem::fail(ctx, SEM_EINVAL, "sem_cg_solve: null argument");
    if (opts->precision != cg->precision)
        return sem::fail(ctx, SEM_EINVAL, "sem_cg_solve: precision %d differs from set-up (%d)",
                         opts->precision, cg->precision);
    if (opts->learned != cg->lp || opts->mg != cg->mg)
        return sem::fail(ctx, SEM_EINVAL, "sem_cg_solve: preconditioner differs from set-up");
    if (opts->ir_mode != 0 && opts->ir_mode != 1)
        return sem::fail(ctx, SEM_EINVAL, "sem_cg_solve: bad ir_mode %d", opts->ir_mode);

    if (!(opts->tol > 0.0)) return sem::fail(ctx, SEM_EINVAL, "sem_cg_solve: tol must be > 0");
    *stats = sem_solve_stats_t{};
    // a multigrid iteration costs several operator applications: check more often
    const int check = opts->check_every > 0 ? opts->check_every : (cg->mg ? 4 : 16);
    const int maxit = opts->maxit > 0 ? opts->maxit : 100000;
    hipStream_t st = ctx->stream;
    const int64_t nu = cg->nu;
    const unsigned gu = vec_grid(nu);
    const int32_t *uoff = cg->gs->uoff, *uidx = cg->gs->uidx;

    to_unique_kernel<double><<<gu, kBlock, 0, st>>>(cg->b64, b, uoff, uidx, nu);
    SEM_LAUNCH_CHECK(ctx);
    rc = vec_sums(cg, cg->b64);
    if (rc) return rc;
    double bs, bq;
    rc = read_sums(cg, &bs, &bq);
    if (rc) return rc;
    const double bnorm = std::sqrt(bq);

    if (cg->precision == SEM_SOLVE_F64) {
        Level& L = cg->lv64;
        int its = 0, brk = 0, nj = 0, fb = 0;
        if (flexible(cg)) rc = fcg_run<double>(cg, L, cg->b64, opts->tol, maxit, check, &its, &brk, &nj, &fb);
        else rc = pcg_run<double>(cg, L, cg->b64, opts->tol, maxit, check, &its, &brk);
        if (rc) return rc;
        // The Krylov loop stops on its recursively updated residual, which can
        // drift below the true one.  Check b - A x in float64; while it misses
        // tol, solve A d = r to the relative tolerance that closes the gap and
        // add d to x (at most four times, within the same iteration budget).
        for (int pass = 0; pass < 4 && !brk && its < maxit; ++pass) {
            rc = residual64(cg, cg->x64);
            if (!rc) rc = vec_sums(cg, cg->r64);
            double rs, rq;
            if (!rc) rc = read_sums(cg, &rs, &rq);
            if (rc) return rc;
            const double rnorm = std::sqrt(rq);
            if (!(rnorm > opts->tol * bnorm)) break;
            if (projects(cg)) {
                sub_mean_kernel<<<gu, kBlock, 0, st>>>(cg->r64, cg->sums, (double)nu, nu);
                SEM_LAUNCH_CHECK(ctx);
            }
            const double tol_d = opts->tol * bnorm / rnorm;
            int its_d = 0, brk_d = 0, nj_d = 0, fb_d = 0;
            L.x = cg->d64;                       // the correction goes to d64, x64 is kept
            if (flexible(cg)) rc = fcg_run<double>(cg, L, cg->r64, tol_d, maxit - its, check, &its_d, &brk_d, &nj_d, &fb_d);
            else rc = pcg_run<double>(cg, L, cg->r64, tol_d, maxit - its, check, &its_d, &brk_d);
            L.x = cg->x64;
            if (rc) return rc;
            add_kernel<<<gu, kBlock, 0, st>>>(cg->x64, cg->d64, nu);
            SEM_LAUNCH_CHECK(ctx);
            its += its_d;
            brk |= brk_d;
            nj += nj_d;
            fb |= fb_d;
        }
        stats->jacobi_steps = nj;
        stats->fell_back = fb;
        stats->iterations = its;
        stats->breakdown = brk;
    } else {
        Level& L = cg->lv32;
        const bool bf = cg->precision == SEM_SOLVE_BF16_IR;
        if (opts->ir_mode == 1) {
            int its = 0, nrep = 0, brk = 0, nj = 0, fb = 0;
            // the V-cycle cuts the residual by about 2x per iteration: replace less often
            const double delta = opts->delta > 0 ? opts->delta : (cg->mg ? 1e-3 : 0.1);
            rc = rr_run(cg, L, opts->tol, delta, maxit, check, bnorm, &its,
                        &nrep, &brk, stats->relres_hist, 64, &nj, &fb);
            if (rc) return rc;
            stats->jacobi_steps = nj;
            stats->fell_back = fb;
            stats->iterations = its + nrep;
            stats->outer = nrep;
            stats->breakdown = brk;
            goto finish;
        }
        {
        const double inv_nu = projects(cg) && nu > 0 ? 1.0 / (double)nu : 0.0;
        const double itol = opts->inner_tol > 0 ? opts->inner_tol : (bf ? 1e-2 : 1e-6);
        const int imax = opts->inner_maxit > 0 ? opts->inner_maxit : 500;
        const int omax = std::min(opts->max_outer > 0 ? opts->max_outer : 60, 64);
        zero_kernel<<<gu, kBlock, 0, st>>>(cg->x64, nu);
        SEM_HIP(ctx, hipMemcpyAsync(cg->r64, cg->b64, sizeof(double) * nu, hipMemcpyDeviceToDevice, st));
        int total = 0;
        for (int outer = 0; outer < omax; ++outer) {
            // r64 holds b - A x; project out its mean and normalise into the inner rhs
            rc = vec_sums(cg, cg->r64);
            if (rc) return rc;
            double s, q;
            rc = read_sums(cg, &s, &q);
            if (rc) return rc;
            const double c = s * inv_nu;
            const double rn = std::sqrt(std::max(q - c * s, 0.0));
            const double rel = bnorm > 0 ? rn / bnorm : 0.0;
            if (outer > 0) stats->relres_hist[outer - 1] = rel;
            if (rel <= opts->tol || total >= maxit) break;
            ir_scale_kernel<<<gu, kBlock, 0, st>>>(cg->rhs32, cg->r64, cg->sums, inv_nu, nu);
            int its = 0, brk = 0, nj = 0, fb = 0;
            if (flexible(cg))
                rc = fcg_run<float>(cg, L, cg->rhs32, itol, std::min(imax, maxit - total), check,
                                    &its, &brk, &nj, &fb);
            else
                rc = pcg_run<float>(cg, L, cg->rhs32, itol, std::min(imax, maxit - total), check,
                                    &its, &brk);
            if (rc) return rc;
            stats->jacobi_steps += nj;
            stats->fell_back |= fb;
            total += its;
            stats->outer = outer + 1;
            if (brk) stats->breakdown = 1;
            ir_update_kernel<<<gu, kBlock, 0, st>>>(cg->x64, (const float*)L.x, cg->sums, inv_nu, nu);
            rc = remove_mean_u(cg, cg->x64);
            if (rc) return rc;
            rc = residual64(cg, cg->x64);
            if (rc) return rc;
            total += 1;
        }
        stats->iterations = total;
        }
    }
finish:
    // x: mean-free (periodic), back to the local layout; final float64 residual
    rc = remove_mean_u(cg, cg->x64);
    if (rc) return rc;
    rc = residual64(cg, cg->x64);
    if (rc) return rc;
    rc = vec_sums(cg, cg->r64);
    if (rc) return rc;
    double rs, rq;
    rc = read_sums(cg, &rs, &rq);
    if (rc) return rc;
    to_local_kernel<<<vec_grid(cg->n), kBlock, 0, st>>>(x, cg->x64, cg->gs->lid, cg->n);
    SEM_LAUNCH_CHECK(ctx);
    SEM_HIP(ctx, hipStreamSynchronize(st));
    stats->relres = bnorm > 0 ? std::sqrt(rq) / bnorm : 0.0;
    stats->converged = stats->relres <= opts->tol;
    if (stats->breakdown && !stats->converged) return sem::fail(ctx, SEM_EBREAKDOWN, "sem_cg_solve: breakdown");
    if (!stats->converged) return SEM_NOT_CONVERGED;
    return stats->fell_back ? SEM_FELL_BACK : SEM_OK;
}

extern "C" int sem_remove_mean(sem_gs_t gs, double* x) {
    if (!gs) return sem::fail(nullptr, SEM_EINVAL, "sem_remove_mean: null plan");
    sem_ctx_t ctx = gs->ctx;
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (gs->n_masked > 0)
        return sem::fail(ctx, SEM_EINVAL, "sem_remove_mean: the plan has Dirichlet nodes (no null space)");
    if (gs->n_local == 0) return SEM_OK;
    if (!x) return sem::fail(ctx, SEM_EINVAL, "sem_remove_mean: null field");
    const int64_t n = gs->n_local;
    const unsigned g = vec_grid(n);
    hipStream_t st = ctx->stream;
    wsum_kernel<<<g, kBlock, 0, st>>>(x, gs->owner, n, ctx->red + 2);
    wsum_final<<<1, kFinal, 0, st>>>(ctx->red, ctx->red + 2, (int)g);
    sub_mean_kernel<<<g, kBlock, 0, st>>>(x, ctx->red, (double)gs->n_unique, n);
    SEM_LAUNCH_CHECK(ctx);
    return SEM_OK;
}

// ----------------------------------------------------------------------------
// sem_remove_mean_static: sem_remove_mean with its reduction partials in a
// fixed device array instead of the context's workspace, for callers that
// cannot allocate.  Each GPU holds its own copy of `scratch` at its own
// address; host code never passes the array's name to a kernel, only the
// address that hipGetSymbolAddress returned for the current device.
namespace {

constexpr int kScratchSlots = 2 + kGrid;   // the mean, a spare slot, one partial per workgroup
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kScratchSlots];

std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on device dev (made current by the caller)
int scratch_address(sem_ctx_t ctx, int dev, double** out) {
    if (dev < 0 || dev >= kMaxDevices)
        return sem::fail(ctx, SEM_EINVAL, "sem_remove_mean_static: device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return sem::check_hip(ctx, e, "sem_remove_mean_static: hipGetSymbolAddress");
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return SEM_OK;
}

}  // namespace

extern "C" int sem_remove_mean_static(sem_gs_t gs, double* x) {
    if (!gs) return sem::fail(nullptr, SEM_EINVAL, "sem_remove_mean_static: null plan");
    sem_ctx_t ctx = gs->ctx;
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (gs->n_masked > 0)
        return sem::fail(ctx, SEM_EINVAL, "sem_remove_mean_static: the plan has Dirichlet nodes (no null space)");
    if (gs->n_local == 0) return SEM_OK;
    if (!x) return sem::fail(ctx, SEM_EINVAL, "sem_remove_mean_static: null field");
    const int64_t n = gs->n_local;
    const unsigned g = vec_grid(n);
    if (2 + (int64_t)g > kScratchSlots)
        return sem::fail(ctx, SEM_EINVAL, "sem_remove_mean_static: %u partials exceed the %d-slot scratch array",
                         g, kScratchSlots);
    double* sp = nullptr;
    rc = scratch_address(ctx, ctx->device, &sp);
    if (rc) return rc;
    hipStream_t st = ctx->stream;
    // every partial and the mean are written before they are read: nothing to clear
    wsum_kernel<<<g, kBlock, 0, st>>>(x, gs->owner, n, sp + 2);
    wsum_final<<<1, kFinal, 0, st>>>(sp, sp + 2, (int)g);
    sub_mean_kernel<<<g, kBlock, 0, st>>>(x, sp, (double)gs->n_unique, n);
    SEM_LAUNCH_CHECK(ctx);
    return SEM_OK;
}
