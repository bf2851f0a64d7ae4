// Krylov solves around the assembled operator y = gs(Ax(x)).
//
//  * Jacobi-preconditioned CG (Hestenes-Stiefel; Saad, Alg. 9.1), M = diag(A_G),
//    x_0 = 0, stopped on the recursively updated residual.
//  * Float64 iterative refinement (Wilkinson; Carson and Higham 2018) around
//    inner PCG solves whose vectors are float32 and whose operator is the
//    float32 or the bfloat16-factor form of the element operator; dot products
//    are always accumulated in float64.
//
// Everything stays on the device: scalars (alpha, beta, r.z, ...) live in a
// small device struct, a `done` flag turns every later kernel of a converged
// solve into an early return, and the host reads the flag once every
// `check_every` iterations.  Dots of continuous fields count one owner copy of
// each global node (a bit mask), so they equal the dots of the unique vectors.
// Reductions are two-stage with a fixed number of partials and a fixed
// summation order: results are bitwise reproducible.
#include <cmath>
#include <vector>

#include "sem_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr int kGrid = 1024;           // vector kernels: fixed grid -> fixed partial count
constexpr int kFinal = 1024;          // threads of the single-block finalisers

struct Scal {
    double rz, pAp, alpha, beta, rr, bb, tol2, mean, pw_prev;
    int done, it, breakdown, maxit;
    int usej, njac, fallback;   // flexible CG: Jacobi this iteration, count, for good
};

__device__ __forceinline__ bool owner_bit(const uint32_t* __restrict__ m, int64_t L) {
    return (m[L >> 5] >> (L & 31)) & 1u;
}

// sum of a per-thread double over a 256-thread block, written by thread 0
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

__global__ void owner_bits_kernel(uint32_t* __restrict__ bits, const double* __restrict__ owner,
                                  int64_t n) {
    const int64_t wd = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t nw = (n + 31) >> 5;
    if (wd >= nw) return;
    uint32_t b = 0;
    for (int q = 0; q < 32; ++q) {
        const int64_t L = (wd << 5) + q;
        if (L < n && owner[L] != 0.0) b |= 1u << q;
    }
    bits[wd] = b;
}

template <typename T>
__global__ void recip_kernel(T* __restrict__ out, const double* __restrict__ d, int64_t n) {
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n;
         L += (int64_t)gridDim.x * blockDim.x)
        out[L] = (T)(1.0 / d[L]);
}

// r = rhs, x = 0, p = Minv r; partials (r.Minv.r, r.r) over owners
template <typename T>
__global__ void pcg_init_kernel(T* __restrict__ x, T* __restrict__ r, T* __restrict__ p,
                                const T* __restrict__ rhs, const T* __restrict__ minv,
                                const uint32_t* __restrict__ own, int64_t n,
                                double* __restrict__ part) {
    __shared__ double s_red[kBlock / 64];
    double a = 0.0, b = 0.0;
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n;
         L += (int64_t)gridDim.x * blockDim.x) {
        const T rv = rhs[L];
        const T z = minv[L] * rv;
        x[L] = T(0);
        r[L] = rv;
        p[L] = z;
        if (owner_bit(own, L)) {
            a += (double)rv * (double)z;
            b += (double)rv * (double)rv;
        }
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

// x += alpha p, r -= alpha w; partials (r.Minv.r, r.r) over owners
template <typename T>
__global__ void pcg_update_kernel(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p,
                                  const T* __restrict__ w, const T* __restrict__ minv,
                                  const uint32_t* __restrict__ own, int64_t n,
                                  const Scal* __restrict__ S, double* __restrict__ part) {
    if (S->done) return;
    __shared__ double s_red[kBlock / 64];
    const T alpha = (T)S->alpha;
    double a = 0.0, b = 0.0;
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n;
         L += (int64_t)gridDim.x * blockDim.x) {
        x[L] += alpha * p[L];
        const T rv = r[L] - alpha * w[L];
        r[L] = rv;
        if (owner_bit(own, L)) {
            a += (double)rv * (double)(minv[L] * rv);
            b += (double)rv * (double)rv;
        }
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
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n;
         L += (int64_t)gridDim.x * blockDim.x)
        p[L] = minv[L] * r[L] + beta * p[L];
}

// partials of (sum_own a, sum_own a*a) for a float64 or float32 vector
template <typename T>
__global__ void owner_sums_kernel(const T* __restrict__ a, const uint32_t* __restrict__ own,
                                  int64_t n, double* __restrict__ part) {
    __shared__ double s_red[kBlock / 64];
    double s = 0.0, q = 0.0;
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n;
         L += (int64_t)gridDim.x * blockDim.x) {
        if (owner_bit(own, L)) {
            const double v = (double)a[L];
            s += v;
            q += v * v;
        }
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

// x -= c, with c = sums[0] / n_unique (the mean over unique nodes)
__global__ void sub_mean_kernel(double* __restrict__ x, const double* __restrict__ sums,
                                double n_unique, int64_t n) {
    const double c = sums[0] / n_unique;
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n;
         L += (int64_t)gridDim.x * blockDim.x)
        x[L] -= c;
}

// r = b - w (float64)
__global__ void residual_kernel(double* __restrict__ r, const double* __restrict__ b,
                                const double* __restrict__ w, int64_t n) {
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n;
         L += (int64_t)gridDim.x * blockDim.x)
        r[L] = b[L] - w[L];
}

// IR: rhat = (float)((r - mean) / norm) with mean = s0/nu, norm = sqrt(q - nu mean^2)
__global__ void ir_scale_kernel(float* __restrict__ rhat, const double* __restrict__ r,
                                const double* __restrict__ sums, double n_unique, int64_t n) {
    const double c = sums[0] / n_unique;
    const double nrm2 = sums[1] - n_unique * c * c;
    const double inv = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n;
         L += (int64_t)gridDim.x * blockDim.x)
        rhat[L] = (float)((r[L] - c) * inv);
}

// IR: x += norm * d (float64 update)
__global__ void ir_update_kernel(double* __restrict__ x, const float* __restrict__ d,
                                 const double* __restrict__ sums, double n_unique, int64_t n) {
    const double c = sums[0] / n_unique;
    const double nrm2 = sums[1] - n_unique * c * c;
    const double nrm = nrm2 > 0.0 ? sqrt(nrm2) : 0.0;
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n;
         L += (int64_t)gridDim.x * blockDim.x)
        x[L] += nrm * (double)d[L];
}

// partials of sum_L owner_L x_L (float64 owner weights)
__global__ void wsum_kernel(const double* __restrict__ x, const double* __restrict__ owner,
                            int64_t n, double* __restrict__ part) {
    __shared__ double s_red[kBlock / 64];
    double s = 0.0;
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n;
         L += (int64_t)gridDim.x * blockDim.x)
        s += owner[L] * x[L];
    s = block_sum(s, s_red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void wsum_final(double* __restrict__ out, const double* __restrict__ part, int n) {
    __shared__ double s_red[kFinal / 64];
    const double s = final_sum(part, n, 1, s_red);
    if (threadIdx.x == 0) out[0] = s;
}

__global__ void zero_kernel(double* __restrict__ x, int64_t n) {
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n;
         L += (int64_t)gridDim.x * blockDim.x)
        x[L] = 0.0;
}

template <typename T>
__global__ void to_type_kernel(T* __restrict__ out, const double* __restrict__ in, int64_t n) {
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n;
         L += (int64_t)gridDim.x * blockDim.x)
        out[L] = (T)in[L];
}

__device__ inline uint16_t bf16_rne(float f) {
    uint32_t b = __float_as_uint(f);
    if ((b & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((b >> 16) | 0x40u);
    b += 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

__global__ void to_bf16_kernel(uint16_t* __restrict__ out, const double* __restrict__ in, int64_t n) {
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n;
         L += (int64_t)gridDim.x * blockDim.x)
        out[L] = bf16_rne((float)in[L]);
}


// ---- flexible CG (Notay's FCG(1)) with a variable preconditioner ----------
// partials over owners: r.z, non-finite count of z, z.w_prev, (Minv r).w_prev
template <typename T>
__global__ void fcg_dots_kernel(const T* __restrict__ r, const T* __restrict__ z,
                                const T* __restrict__ wprev, const T* __restrict__ minv,
                                const uint32_t* __restrict__ own, int64_t n,
                                const Scal* __restrict__ S, double* __restrict__ part) {
    if (S->done) return;
    __shared__ double s_red[kBlock / 64];
    const bool first = S->it == 0;
    double rz = 0.0, bad = 0.0, zw = 0.0, jw = 0.0;
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n;
         L += (int64_t)gridDim.x * blockDim.x) {
        const double zv = (double)z[L];
        if (!isfinite(zv)) bad += 1.0;
        if (owner_bit(own, L)) {
            const double rv = (double)r[L];
            rz += rv * zv;
            if (!first) {
                const double wv = (double)wprev[L];
                zw += zv * wv;
                jw += (double)(minv[L] * r[L]) * wv;
            }
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

// p = z_eff - gamma p (z_eff = Minv r when the network output is rejected);
// partials over owners of p.r
template <typename T>
__global__ void fcg_p_kernel(T* __restrict__ p, const T* __restrict__ z, const T* __restrict__ r,
                             const T* __restrict__ minv, const uint32_t* __restrict__ own, int64_t n,
                             const Scal* __restrict__ S, double* __restrict__ part) {
    if (S->done) return;
    __shared__ double s_red[kBlock / 64];
    const bool usej = S->usej != 0;
    const bool first = S->it == 0;
    const T gamma = (T)S->beta;
    double pr = 0.0;
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n;
         L += (int64_t)gridDim.x * blockDim.x) {
        const T rv = r[L];
        const T ze = usej ? minv[L] * rv : z[L];
        const T pv = first ? ze : ze - gamma * p[L];
        p[L] = pv;
        if (owner_bit(own, L)) pr += (double)pv * (double)rv;
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

__global__ void set_fallback(Scal* __restrict__ S) {
    if (threadIdx.x == 0 && blockIdx.x == 0) S->fallback = 1;
}

}  // namespace

// One precision level of the solver: vectors of type T and the operator form
// that acts on them.
struct Level {
    sem::AxKind kind;
    sem::AxArgs A;
    void *x = nullptr, *r = nullptr, *p = nullptr, *w = nullptr, *minv = nullptr;
    void* z = nullptr;   // flexible CG: the preconditioner's output
};

struct sem_cg_s {
    sem_ctx_t ctx = nullptr;
    sem_gs_t gs = nullptr;
    int precision = SEM_SOLVE_F64;
    int64_t n = 0;
    double n_unique = 0;
    sem::AxArgs A64{};
    uint32_t* own = nullptr;
    Scal* S = nullptr;
    double* part = nullptr;        // max(4*kGrid, ax_blocks) doubles
    double* part2 = nullptr;       // kGrid doubles (flexible CG: p.r partials)
    sem_lp_t lp = nullptr;
    double* sums = nullptr;        // 2 doubles
    Scal* S_host = nullptr;        // pinned
    double* sums_host = nullptr;   // pinned
    Level lv64{}, lv32{};
    double *r64 = nullptr, *w64 = nullptr;
    float* rhs32 = nullptr;        // IR: normalised inner right-hand side
    std::vector<void*> allocs;
};

namespace {

int cg_alloc(sem_cg_t cg, void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return sem::check_hip(cg->ctx, e, "sem_cg_setup: hipMalloc");
    cg->allocs.push_back(*p);
    return SEM_OK;
}

unsigned vec_grid(int64_t n) {
    int64_t b = (n + kBlock - 1) / kBlock;
    return (unsigned)(b < kGrid ? (b < 1 ? 1 : b) : kGrid);
}

// PCG on level lv from x = 0 with right-hand side rhs (type T, continuous);
// leaves the iterate in lv.x.  Returns SEM_OK and fills S_host on exit.
template <typename T>
int pcg_run(sem_cg_t cg, Level& lv, const T* rhs, double tol, int maxit, int check_every,
            int* iters_out, int* breakdown_out) {
    sem_ctx_t ctx = cg->ctx;
    hipStream_t st = ctx->stream;
    const int64_t n = cg->n;
    const unsigned g = vec_grid(n);
    T* x = (T*)lv.x; T* r = (T*)lv.r; T* p = (T*)lv.p; T* w = (T*)lv.w;
    const T* minv = (const T*)lv.minv;
    pcg_init_kernel<T><<<g, kBlock, 0, st>>>(x, r, p, rhs, minv, cg->own, n, cg->part);
    pcg_init_final<<<1, kFinal, 0, st>>>(cg->S, cg->part, (int)g, tol, maxit);
    SEM_LAUNCH_CHECK(ctx);
    const int nb = sem::ax_blocks(lv.A.lx, lv.A.nel);
    int done_it = 0;
    for (;;) {
        for (int q = 0; q < check_every; ++q) {
            int rc = sem::launch_ax(ctx, lv.kind, lv.A, w, p, &cg->S->done, cg->part);
            if (rc) return rc;
            rc = sem_gs(cg->gs, w, sizeof(T) == 8 ? SEM_F64 : SEM_F32);
            if (rc) return rc;
            pcg_alpha_final<<<1, kFinal, 0, st>>>(cg->S, cg->part, nb);
            pcg_update_kernel<T><<<g, kBlock, 0, st>>>(x, r, p, w, minv, cg->own, n, cg->S, cg->part);
            pcg_beta_final<<<1, kFinal, 0, st>>>(cg->S, cg->part, (int)g);
            pcg_p_kernel<T><<<g, kBlock, 0, st>>>(p, r, minv, n, cg->S);
        }
        SEM_LAUNCH_CHECK(ctx);
        SEM_HIP(ctx, hipMemcpyAsync(cg->S_host, cg->S, sizeof(Scal), hipMemcpyDeviceToHost, st));
        SEM_HIP(ctx, hipStreamSynchronize(st));
        done_it = cg->S_host->it;
        if (cg->S_host->done) break;
    }
    *iters_out = done_it;
    *breakdown_out = cg->S_host->breakdown;
    return SEM_OK;
}

// flexible CG on level lv with the bound network; same contract as pcg_run
template <typename T>
int fcg_run(sem_cg_t cg, Level& lv, const T* rhs, double tol, int maxit, int check_every,
            int* iters_out, int* breakdown_out, int* njac_out, int* fell_back) {
    sem_ctx_t ctx = cg->ctx;
    hipStream_t st = ctx->stream;
    const int64_t n = cg->n;
    const unsigned g = vec_grid(n);
    T* x = (T*)lv.x; T* r = (T*)lv.r; T* p = (T*)lv.p; T* w = (T*)lv.w; T* z = (T*)lv.z;
    const T* minv = (const T*)lv.minv;
    pcg_init_kernel<T><<<g, kBlock, 0, st>>>(x, r, p, rhs, minv, cg->own, n, cg->part);
    pcg_init_final<<<1, kFinal, 0, st>>>(cg->S, cg->part, (int)g, tol, maxit);
    SEM_LAUNCH_CHECK(ctx);
    const int nb = sem::ax_blocks(lv.A.lx, lv.A.nel);
    const bool f64 = sizeof(T) == 8;
    bool fallen = false;
    // the fallback flag starts cleared for every solve
    SEM_HIP(ctx, hipMemcpyAsync(cg->S_host, cg->S, sizeof(Scal), hipMemcpyDeviceToHost, st));
    SEM_HIP(ctx, hipStreamSynchronize(st));
    cg->S_host->fallback = 0;
    SEM_HIP(ctx, hipMemcpyAsync(cg->S, cg->S_host, sizeof(Scal), hipMemcpyHostToDevice, st));
    std::vector<std::pair<int, double>> hist;   // (iteration, rr) at each check
    for (;;) {
        for (int q = 0; q < check_every; ++q) {
            int rc = SEM_OK;
            if (!fallen) rc = sem::lp_apply(cg->lp, z, r, f64, &cg->S->done);
            if (rc) return rc;
            fcg_dots_kernel<T><<<g, kBlock, 0, st>>>(r, z, w, minv, cg->own, n, cg->S, cg->part);
            fcg_gamma_final<<<1, kFinal, 0, st>>>(cg->S, cg->part, (int)g);
            fcg_p_kernel<T><<<g, kBlock, 0, st>>>(p, z, r, minv, cg->own, n, cg->S, cg->part2);
            rc = sem::launch_ax(ctx, lv.kind, lv.A, w, p, &cg->S->done, cg->part);
            if (rc) return rc;
            rc = sem::gs_launch(cg->gs, w, f64 ? SEM_F64 : SEM_F32, &cg->S->done);
            if (rc) return rc;
            fcg_alpha_final<<<1, kFinal, 0, st>>>(cg->S, cg->part, nb, cg->part2, (int)g);
            pcg_update_kernel<T><<<g, kBlock, 0, st>>>(x, r, p, w, minv, cg->own, n, cg->S, cg->part);
            pcg_beta_final<<<1, kFinal, 0, st>>>(cg->S, cg->part, (int)g);
        }
        SEM_LAUNCH_CHECK(ctx);
        SEM_HIP(ctx, hipMemcpyAsync(cg->S_host, cg->S, sizeof(Scal), hipMemcpyDeviceToHost, st));
        SEM_HIP(ctx, hipStreamSynchronize(st));
        if (cg->S_host->done) break;
        // stagnation guard: relative residual not halved over 256 iterations
        hist.emplace_back(cg->S_host->it, cg->S_host->rr);
        if (!fallen) {
            for (auto it = hist.rbegin(); it != hist.rend(); ++it) {
                if (cg->S_host->it - it->first >= 256) {
                    if (cg->S_host->rr > 0.25 * it->second) {   // rr is squared: halving = 1/4
                        set_fallback<<<1, 1, 0, st>>>(cg->S);
                        SEM_LAUNCH_CHECK(ctx);
                        fallen = true;
                    }
                    break;
                }
            }
        }
    }
    *iters_out = cg->S_host->it;
    *breakdown_out = cg->S_host->breakdown;
    *njac_out = cg->S_host->njac;
    *fell_back = fallen ? 1 : 0;
    return SEM_OK;
}

// sums over owners of (a, a*a) into cg->sums (device) -- asynchronous
template <typename T>
int owner_sums(sem_cg_t cg, const T* a) {
    const unsigned g = vec_grid(cg->n);
    owner_sums_kernel<T><<<g, kBlock, 0, cg->ctx->stream>>>(a, cg->own, cg->n, cg->part);
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

// relres of x against b in float64: w = A x, r = b - w
int true_relres(sem_cg_t cg, const double* x, const double* b, double bnorm, double* relres) {
    int rc = sem::launch_ax(cg->ctx, sem::AxKind::F64, cg->A64, cg->w64, x, nullptr, nullptr);
    if (rc) return rc;
    rc = sem_gs(cg->gs, cg->w64, SEM_F64);
    if (rc) return rc;
    residual_kernel<<<vec_grid(cg->n), kBlock, 0, cg->ctx->stream>>>(cg->r64, b, cg->w64, cg->n);
    rc = owner_sums(cg, cg->r64);
    if (rc) return rc;
    double s, q;
    rc = read_sums(cg, &s, &q);
    if (rc) return rc;
    *relres = bnorm > 0 ? std::sqrt(q) / bnorm : 0.0;
    return SEM_OK;
}

int remove_mean(sem_cg_t cg, double* x) {
    int rc = owner_sums(cg, x);
    if (rc) return rc;
    sub_mean_kernel<<<vec_grid(cg->n), kBlock, 0, cg->ctx->stream>>>(x, cg->sums, cg->n_unique, cg->n);
    SEM_LAUNCH_CHECK(cg->ctx);
    return SEM_OK;
}

}  // namespace

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

    auto* cg = new sem_cg_s();
    cg->ctx = ctx;
    cg->gs = gs;
    cg->precision = opts->precision;
    cg->n = n;
    cg->n_unique = (double)gs->n_unique;
    for (int q = 0; q < 6; ++q) { cg->A64.D[q] = Dp[q]; cg->A64.G[q] = Gp[q]; }
    cg->A64.h1 = A->h1;
    cg->A64.nel = A->nel;
    cg->A64.lx = A->lx;
    hipStream_t st = ctx->stream;
    const unsigned g = vec_grid(n);
    const int nb = sem::ax_blocks(A->lx, A->nel);
    const size_t npart = (size_t)std::max(4 * kGrid, nb);
    const int64_t nw = (n + 31) / 32;
    const size_t v64 = sizeof(double) * n, v32 = sizeof(float) * n;
    auto bail = [&](int code) { sem_cg_destroy(cg); return code; };
#define CG_ALLOC(ptr, bytes) do { int rc_ = cg_alloc(cg, (void**)&(ptr), (bytes)); if (rc_) return bail(rc_); } while (0)
    CG_ALLOC(cg->own, sizeof(uint32_t) * nw);
    CG_ALLOC(cg->S, sizeof(Scal));
    CG_ALLOC(cg->part, sizeof(double) * npart);
    CG_ALLOC(cg->sums, sizeof(double) * 2);
    CG_ALLOC(cg->part2, sizeof(double) * kGrid);
    if (opts->learned) {
        if (sem::lp_rows(opts->learned) != A->nel || sem::lp_plan(opts->learned) != gs)
            return bail(sem::fail(ctx, SEM_EINVAL, "sem_cg_setup: the network is not bound to this operator and plan"));
        cg->lp = opts->learned;
    }
    CG_ALLOC(cg->r64, v64);
    CG_ALLOC(cg->w64, v64);
    {
        hipError_t e = hipHostMalloc(&cg->S_host, sizeof(Scal), hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc(&cg->sums_host, 2 * sizeof(double), hipHostMallocDefault);
        if (e != hipSuccess) return bail(sem::check_hip(ctx, e, "sem_cg_setup: hipHostMalloc"));
    }
    owner_bits_kernel<<<(unsigned)((nw + kBlock - 1) / kBlock), kBlock, 0, st>>>(cg->own, gs->owner, n);
    // assembled Jacobi diagonal (float64) in r64
    rc = sem_ax_diag(ctx, cg->r64, A->dx, A->h1, A->g11, A->g22, A->g33, A->g12, A->g13, A->g23,
                     A->nel, A->lx);
    if (rc) return bail(rc);
    rc = sem_gs(gs, cg->r64, SEM_F64);
    if (rc) return bail(rc);

    Level& L64 = cg->lv64;
    L64.kind = sem::AxKind::F64;
    L64.A = cg->A64;
    if (opts->precision == SEM_SOLVE_F64) {
        CG_ALLOC(L64.x, v64); CG_ALLOC(L64.r, v64); CG_ALLOC(L64.p, v64); CG_ALLOC(L64.minv, v64);
        if (cg->lp) CG_ALLOC(L64.z, v64);
        L64.w = cg->w64;
        recip_kernel<double><<<g, kBlock, 0, st>>>((double*)L64.minv, cg->r64, n);
    } else {
        Level& L = cg->lv32;
        const bool bf = opts->precision == SEM_SOLVE_BF16_IR;
        L.kind = bf ? sem::AxKind::F32_BF16 : sem::AxKind::F32;
        CG_ALLOC(L.x, v32); CG_ALLOC(L.r, v32); CG_ALLOC(L.p, v32); CG_ALLOC(L.w, v32); CG_ALLOC(L.minv, v32);
        CG_ALLOC(cg->rhs32, v32);
        if (cg->lp) CG_ALLOC(L.z, v32);
        recip_kernel<float><<<g, kBlock, 0, st>>>((float*)L.minv, cg->r64, n);
        // derivative matrices in float32
        const int l2 = A->lx * A->lx;
        for (int q = 0; q < 6; ++q) {
            void* d = nullptr;
            CG_ALLOC(d, sizeof(float) * l2);
            to_type_kernel<float><<<1, kBlock, 0, st>>>((float*)d, Dp[q], l2);
            L.A.D[q] = d;
        }
        const size_t vs = bf ? sizeof(uint16_t) * n : v32;
        const double* src[7] = {Gp[0], Gp[1], Gp[2], Gp[3], Gp[4], Gp[5], A->h1};
        for (int q = 0; q < 7; ++q) {
            if (!src[q]) { L.A.h1 = nullptr; continue; }
            void* d = nullptr;
            CG_ALLOC(d, vs);
            if (bf) to_bf16_kernel<<<g, kBlock, 0, st>>>((uint16_t*)d, src[q], n);
            else to_type_kernel<float><<<g, kBlock, 0, st>>>((float*)d, src[q], n);
            if (q < 6) L.A.G[q] = d; else L.A.h1 = d;
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
    if (opts->learned != cg->lp)
        return sem::fail(ctx, SEM_EINVAL, "sem_cg_solve: preconditioner differs from set-up");
    if (!(opts->tol > 0.0)) return sem::fail(ctx, SEM_EINVAL, "sem_cg_solve: tol must be > 0");
    *stats = sem_solve_stats_t{};
    const int check = opts->check_every > 0 ? opts->check_every : 16;
    const int maxit = opts->maxit > 0 ? opts->maxit : 100000;
    hipStream_t st = ctx->stream;
    const int64_t n = cg->n;

    rc = owner_sums(cg, b);
    if (rc) return rc;
    double bs, bq;
    rc = read_sums(cg, &bs, &bq);
    if (rc) return rc;
    const double bnorm = std::sqrt(bq);

    if (cg->precision == SEM_SOLVE_F64) {
        Level& L = cg->lv64;
        int its = 0, brk = 0, nj = 0, fb = 0;
        if (cg->lp) rc = fcg_run<double>(cg, L, b, opts->tol, maxit, check, &its, &brk, &nj, &fb);
        else rc = pcg_run<double>(cg, L, b, opts->tol, maxit, check, &its, &brk);
        if (rc) return rc;
        stats->jacobi_steps = nj;
        stats->fell_back = fb;
        SEM_HIP(ctx, hipMemcpyAsync(x, L.x, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
        rc = remove_mean(cg, x);
        if (rc) return rc;
        stats->iterations = its;
        stats->breakdown = brk;
    } else {
        Level& L = cg->lv32;
        const bool bf = cg->precision == SEM_SOLVE_BF16_IR;
        const double itol = opts->inner_tol > 0 ? opts->inner_tol : (bf ? 1e-2 : 1e-6);
        const int imax = opts->inner_maxit > 0 ? opts->inner_maxit : 500;
        const int omax = std::min(opts->max_outer > 0 ? opts->max_outer : 60, 64);
        zero_kernel<<<vec_grid(n), kBlock, 0, st>>>(x, n);
        SEM_HIP(ctx, hipMemcpyAsync(cg->r64, b, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
        int total = 0;
        for (int outer = 0; outer < omax; ++outer) {
            // r64 holds b - A x; project out its mean and normalise into the inner rhs
            rc = owner_sums(cg, cg->r64);
            if (rc) return rc;
            double s, q;
            rc = read_sums(cg, &s, &q);
            if (rc) return rc;
            const double c = s / cg->n_unique;
            const double rn = std::sqrt(std::max(q - cg->n_unique * c * c, 0.0));
            const double rel = bnorm > 0 ? rn / bnorm : 0.0;
            if (outer > 0) stats->relres_hist[outer - 1] = rel;
            if (rel <= opts->tol || total >= maxit) break;
            ir_scale_kernel<<<vec_grid(n), kBlock, 0, st>>>(cg->rhs32, cg->r64, cg->sums,
                                                             cg->n_unique, n);
            int its = 0, brk = 0, nj = 0, fb = 0;
            if (cg->lp)
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
            ir_update_kernel<<<vec_grid(n), kBlock, 0, st>>>(x, (const float*)L.x, cg->sums,
                                                              cg->n_unique, n);
            rc = remove_mean(cg, x);
            if (rc) return rc;
            // float64 residual r64 = b - A x
            rc = sem::launch_ax(ctx, sem::AxKind::F64, cg->A64, cg->w64, x, nullptr, nullptr);
            if (rc) return rc;
            rc = sem_gs(cg->gs, cg->w64, SEM_F64);
            if (rc) return rc;
            residual_kernel<<<vec_grid(n), kBlock, 0, st>>>(cg->r64, b, cg->w64, n);
            SEM_LAUNCH_CHECK(ctx);
            total += 1;
        }
        stats->iterations = total;
    }
    double rel = 0.0;
    rc = true_relres(cg, x, b, bnorm, &rel);
    if (rc) return rc;
    stats->relres = rel;
    stats->converged = rel <= opts->tol;
    if (stats->breakdown && !stats->converged) return sem::fail(ctx, SEM_EBREAKDOWN, "sem_cg_solve: breakdown");
    if (!stats->converged) return SEM_NOT_CONVERGED;
    return stats->fell_back ? SEM_FELL_BACK : SEM_OK;
}

extern "C" int sem_remove_mean(sem_gs_t gs, double* x) {
    if (!gs) return sem::fail(nullptr, SEM_EINVAL, "sem_remove_mean: null plan");
    sem_ctx_t ctx = gs->ctx;
    int rc = sem::enter(ctx);
    if (rc) return rc;
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
