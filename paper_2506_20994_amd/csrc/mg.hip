// Multigrid preconditioner for the box solves: one symmetric V-cycle over a
// hierarchy of re-discretised box operators with Chebyshev-Jacobi smoothing.
//
// The operator's Poisson solve (Sec. 3) with Jacobi needs an iteration count
// that grows with the mesh; the classical remedy for spectral elements
// coarsens the polynomial degree on the same elements (p-multigrid; Ronquist
// and Patera 1987) and then the trilinear (lx = 2) mesh (h-coarsening).
//  * Levels: the caller's operator (n^3 elements, lx); lx -> max(2, lx / 2) on
//    the same elements down to lx = 2; then the lx = 2 box n^3 -> (n/2)^3 while
//    n is even and n / 2 >= n_coarse.  The last level is solved exactly with
//    a dense inverse, of A + c 1 1^T on the singular periodic box
//    (c = mean diagonal / unknowns: the pseudo-inverse on mean-free vectors).
//  * Every level below the first is re-discretised by the library's own set-up
//    calls (box mesh, isoparametric geometry, gather-scatter plan) on the same
//    deformed box, with h1 = 1 and, for Helmholtz operators, h2 B of that level.
//    With the Galerkin option every lx = 2 level below the first is instead
//    P^T A P of the level above (no geometry of its own).  P acts element by
//    element, so that product is the sum over elements of J^T A_e J: one dense
//    8 x 8 matrix per lx = 2 element -- for a p-transfer from the same element's
//    operator applied to the 8 interpolated coarse basis functions, for an
//    h-transfer summed over the 8 children (Trottenberg, Oosterlee and
//    Schueller 2001 for Galerkin coarse operators).
//  * Transfer P: the coarse level's continuous field evaluated at the fine
//    level's nodes -- p: the coarse Lagrange basis at the fine GLL points of
//    the same element; h: the parent element's trilinear basis at the child's
//    nodes (reference coordinate -1 + parity + i).  Restriction P^T.
//  * Smoother: k steps of the Chebyshev semi-iteration (Saad 2003, Alg. 12.1;
//    Adams, Brezina, Hu and Tuminaro 2003) in D^-1 A, D the assembled
//    diagonal, for the interval [lo lmax, hi lmax]; lmax is estimated by
//    Lanczos on D^-1/2 A D^-1/2 (largest Ritz value).
//  * V(b): x = S(b, 0); x += P V(P^T (b - A x)); x = S(b, x).
//
// Vectors are float32 on the unique nodes of each level (the layout the solver
// iterates in).  The operators run in the solver form of ax_kernel (unique
// input through lid, element-local output) and the smoothing kernels assemble
// that output through the plan's CSR lists.  P and P^T act element by element
// with the 1-D transfer matrices in LDS (sum factorisation).  Each fine unique
// node is taken from its first local copy (its owner); that is exact because a
// coarse basis function that is non-zero at a fine node belongs to every
// element containing that node.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "sem_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr int kVecGrid = 2048;
constexpr int kMaxF3 = SEM_LX_MAX * SEM_LX_MAX * SEM_LX_MAX;   // fine element nodes
constexpr int kMaxC = SEM_LX_MAX / 2;                          // coarse lx of any transfer
constexpr int64_t kCoarseMax = 2048;                           // unknowns of the dense coarsest solve

#define MG_LOOP(i, n) \
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

unsigned vgrid(int64_t n) {
    const int64_t b = (n + kBlock - 1) / kBlock;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, kVecGrid));
}

using sem::assemble_local;

// ---------------------------------------------------------------- smoothing
// First Chebyshev step from x = 0: b is the caller's vector (bin) or the
// assembled restricted field (bl, then also stored to bout); r = b,
// d = c0 Minv b, x = d.
__global__ void cheb_first_kernel(float* __restrict__ x, float* __restrict__ r, float* __restrict__ d,
                                  float* __restrict__ bout, const float* __restrict__ bin,
                                  const float* __restrict__ bl, const float* __restrict__ minv, float c0,
                                  const int32_t* __restrict__ uoff, const int32_t* __restrict__ uidx, int64_t nu,
                                  const int* __restrict__ skip) {
    if (skip && *skip) return;
    MG_LOOP(u, nu) {
        const float bv = bl ? assemble_local(bl, uoff, uidx, u) : bin[u];
        if (bout) bout[u] = bv;
        r[u] = bv;
        const float dv = c0 * minv[u] * bv;
        d[u] = dv;
        x[u] = dv;
    }
}

// Later steps: r -= A d (assembled from wl), d = c1 d + c2 Minv r, x += d.
__global__ void cheb_step_kernel(float* __restrict__ x, float* __restrict__ r, float* __restrict__ d,
                                 const float* __restrict__ wl, const float* __restrict__ minv, float c1, float c2,
                                 const int32_t* __restrict__ uoff, const int32_t* __restrict__ uidx, int64_t nu,
                                 const int* __restrict__ skip) {
    if (skip && *skip) return;
    MG_LOOP(u, nu) {
        const float rv = r[u] - assemble_local(wl, uoff, uidx, u);
        r[u] = rv;
        const float dv = c1 * d[u] + c2 * minv[u] * rv;
        d[u] = dv;
        x[u] += dv;
    }
}

// r -= A d: the residual b - A x after the pre-smoothing's last step
__global__ void cheb_resid_kernel(float* __restrict__ r, const float* __restrict__ wl,
                                  const int32_t* __restrict__ uoff, const int32_t* __restrict__ uidx, int64_t nu,
                                  const int* __restrict__ skip) {
    if (skip && *skip) return;
    MG_LOOP(u, nu) r[u] -= assemble_local(wl, uoff, uidx, u);
}

// First step from a given x (post-smoothing): r = b - A x, d = c0 Minv r, x += d.
__global__ void cheb_post_kernel(float* __restrict__ x, float* __restrict__ r, float* __restrict__ d,
                                 const float* __restrict__ b, const float* __restrict__ wl,
                                 const float* __restrict__ minv, float c0, const int32_t* __restrict__ uoff,
                                 const int32_t* __restrict__ uidx, int64_t nu, const int* __restrict__ skip) {
    if (skip && *skip) return;
    MG_LOOP(u, nu) {
        const float rv = b[u] - assemble_local(wl, uoff, uidx, u);
        r[u] = rv;
        const float dv = c0 * minv[u] * rv;
        d[u] = dv;
        x[u] += dv;
    }
}

// ---------------------------------------------------------------- transfers
// J holds the 1-D matrices [parity][i][a] = coarse basis a at fine point i
// (lxf x lxc each; the p-transfer uses parity 0 only).

// P^T: one workgroup per coarse element E.  For each of its children (the
// element itself for p, the eight elements of the finer box for h) the
// owner-masked fine residual is loaded, contracted with J^T along i, j, k and
// summed into the coarse element's nodes; the result is written in the coarse
// level's local layout (assembled by the coarse level's first smoothing step).
__global__ void __launch_bounds__(kBlock)
restrict_kernel(float* __restrict__ blc, const float* __restrict__ rf, const int32_t* __restrict__ lidf,
                const uint8_t* __restrict__ ownf, const float* __restrict__ J, int lxf, int lxc, int h,
                int nf, int nc, int64_t nelc, const int* __restrict__ skip) {
    if (skip && *skip) return;
    __shared__ float sv[kMaxF3];
    __shared__ float t1[SEM_LX_MAX * SEM_LX_MAX * kMaxC];
    __shared__ float t2[SEM_LX_MAX * kMaxC * kMaxC];
    __shared__ float sJ[2 * SEM_LX_MAX * kMaxC];
    const int tid = threadIdx.x;
    const int64_t E = blockIdx.x;
    const int f3 = lxf * lxf * lxf, c3 = lxc * lxc * lxc, fc = lxf * lxc;
    for (int q = tid; q < 2 * fc; q += blockDim.x) sJ[q] = J[q];
    const int64_t ecx = E % nc, ecy = (E / nc) % nc, ecz = E / ((int64_t)nc * nc);
    float acc = 0.f;
    const int nch = h ? 8 : 1;
    for (int ch = 0; ch < nch; ++ch) {
        const int px = ch & 1, py = (ch >> 1) & 1, pz = ch >> 2;
        const int64_t ef = h ? (2 * ecx + px) + nf * ((2 * ecy + py) + (int64_t)nf * (2 * ecz + pz)) : E;
        const float* Jx = sJ + (h ? px : 0) * fc;
        const float* Jy = sJ + (h ? py : 0) * fc;
        const float* Jz = sJ + (h ? pz : 0) * fc;
        __syncthreads();                       // sJ loaded; the previous child's t2 consumed
        for (int q = tid; q < f3; q += blockDim.x) {
            const int64_t L = ef * f3 + q;
            sv[q] = ownf[L] ? rf[lidf[L]] : 0.f;
        }
        __syncthreads();
        for (int q = tid; q < lxf * fc; q += blockDim.x) {      // t1[k][j][a] = sum_i J[i][a] v[k][j][i]
            const int a = q % lxc, kj = q / lxc;
            float s = 0.f;
            for (int i = 0; i < lxf; ++i) s += Jx[i * lxc + a] * sv[kj * lxf + i];
            t1[q] = s;
        }
        __syncthreads();
        for (int q = tid; q < fc * lxc; q += blockDim.x) {      // t2[k][b][a] = sum_j J[j][b] t1[k][j][a]
            const int a = q % lxc, b = (q / lxc) % lxc, k = q / (lxc * lxc);
            float s = 0.f;
            for (int j = 0; j < lxf; ++j) s += Jy[j * lxc + b] * t1[(k * lxf + j) * lxc + a];
            t2[q] = s;
        }
        __syncthreads();
        if (tid < c3) {                                         // acc[c][b][a] += sum_k J[k][c] t2[k][b][a]
            const int a = tid % lxc, b = (tid / lxc) % lxc, c = tid / (lxc * lxc);
            float s = 0.f;
            for (int k = 0; k < lxf; ++k) s += Jz[k * lxc + c] * t2[(k * lxc + b) * lxc + a];
            acc += s;
        }
    }
    if (tid < c3) blc[E * c3 + tid] = acc;
}

// x_f += P x_c: one workgroup per fine element; the coarse element's values
// (0 on Dirichlet nodes) are interpolated along i, j, k and added at the fine
// element's owner nodes.
__global__ void __launch_bounds__(kBlock)
prolong_kernel(float* __restrict__ xf, const float* __restrict__ xc, const int32_t* __restrict__ lidf,
               const uint8_t* __restrict__ ownf, const int32_t* __restrict__ lidc, const float* __restrict__ J,
               int lxf, int lxc, int h, int nf, int nc, int64_t nelf, const int* __restrict__ skip) {
    if (skip && *skip) return;
    __shared__ float sc[kMaxC * kMaxC * kMaxC];
    __shared__ float t1[kMaxC * kMaxC * SEM_LX_MAX];
    __shared__ float t2[kMaxC * SEM_LX_MAX * SEM_LX_MAX];
    __shared__ float sJ[2 * SEM_LX_MAX * kMaxC];
    const int tid = threadIdx.x;
    const int64_t e = blockIdx.x;
    const int f3 = lxf * lxf * lxf, c3 = lxc * lxc * lxc, fc = lxf * lxc;
    for (int q = tid; q < 2 * fc; q += blockDim.x) sJ[q] = J[q];
    const int64_t ex = e % nf, ey = (e / nf) % nf, ez = e / ((int64_t)nf * nf);
    const int64_t E = h ? (ex >> 1) + nc * ((ey >> 1) + (int64_t)nc * (ez >> 1)) : e;
    const float* Jx = sJ + (h ? (int)(ex & 1) : 0) * fc;
    const float* Jy = sJ + (h ? (int)(ey & 1) : 0) * fc;
    const float* Jz = sJ + (h ? (int)(ez & 1) : 0) * fc;
    for (int q = tid; q < c3; q += blockDim.x) {
        const int32_t id = lidc[E * c3 + q];
        sc[q] = id >= 0 ? xc[id] : 0.f;
    }
    __syncthreads();
    for (int q = tid; q < lxc * fc; q += blockDim.x) {          // t1[c][b][i] = sum_a J[i][a] sc[c][b][a]
        const int i = q % lxf, cb = q / lxf;
        float s = 0.f;
        for (int a = 0; a < lxc; ++a) s += Jx[i * lxc + a] * sc[cb * lxc + a];
        t1[q] = s;
    }
    __syncthreads();
    for (int q = tid; q < fc * lxf; q += blockDim.x) {          // t2[c][j][i] = sum_b J[j][b] t1[c][b][i]
        const int i = q % lxf, j = (q / lxf) % lxf, c = q / (lxf * lxf);
        float s = 0.f;
        for (int b = 0; b < lxc; ++b) s += Jy[j * lxc + b] * t1[(c * lxc + b) * lxf + i];
        t2[q] = s;
    }
    __syncthreads();
    for (int q = tid; q < f3; q += blockDim.x) {                // out[k][j][i] = sum_c J[k][c] t2[c][j][i]
        const int ji = q % (lxf * lxf), k = q / (lxf * lxf);
        float s = 0.f;
        for (int c = 0; c < lxc; ++c) s += Jz[k * lxc + c] * t2[c * lxf * lxf + ji];
        const int64_t L = e * f3 + q;
        if (ownf[L]) xf[lidf[L]] += s;
    }
}

// The p-transfers (same elements, lxf -> lxc) with one wave per element and
// four elements per workgroup, so that no workgroup barrier is needed between
// the three contractions (the wave orders its own LDS traffic).  A lane takes
// whole fine rows (k, j) -- a row's lid, owner flags and values are contiguous
// -- and the coarse side is spread over the lanes.
constexpr int kWaveElems = 4;

// a fine row's unique indices and owner flags (LF consecutive local nodes from
// L0): vector loads when LF is a multiple of 4 (L0 is then 16-byte aligned for
// the indices and 4-byte aligned for the flags)
template <int LF>
__device__ __forceinline__ void load_row(int32_t (&id)[LF], bool (&own)[LF], const int32_t* __restrict__ lidf,
                                         const uint8_t* __restrict__ ownf, int64_t L0) {
    if constexpr (LF % 4 == 0) {
#pragma unroll
        for (int q = 0; q < LF / 4; ++q) {
            const int4 v = *reinterpret_cast<const int4*>(lidf + L0 + 4 * q);
            const uint32_t f = *reinterpret_cast<const uint32_t*>(ownf + L0 + 4 * q);
            id[4 * q] = v.x; id[4 * q + 1] = v.y; id[4 * q + 2] = v.z; id[4 * q + 3] = v.w;
#pragma unroll
            for (int b = 0; b < 4; ++b) own[4 * q + b] = ((f >> (8 * b)) & 0xffu) != 0u;
        }
    } else {
#pragma unroll
        for (int i = 0; i < LF; ++i) {
            id[i] = lidf[L0 + i];
            own[i] = ownf[L0 + i] != 0;
        }
    }
}

// P^T: blc[E][c][b][a] = sum_{k,j,i} J[k][c] J[j][b] J[i][a] (owner-masked r_f)[E][k][j][i]
template <int LF, int LC>
__global__ void __launch_bounds__(64 * kWaveElems)
restrict_p_wave_kernel(float* __restrict__ blc, const float* __restrict__ rf, const int32_t* __restrict__ lidf,
                       const uint8_t* __restrict__ ownf, const float* __restrict__ J, int64_t nel,
                       const int* __restrict__ skip) {
    if (skip && *skip) return;
    constexpr int F2 = LF * LF, F3 = F2 * LF, C3 = LC * LC * LC;
    __shared__ float sJ[LF * LC];
    __shared__ float s1[kWaveElems][LF * LF * LC];   // [k][j][a]
    __shared__ float s2[kWaveElems][LF * LC * LC];   // [k][b][a]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int q = tid; q < LF * LC; q += blockDim.x) sJ[q] = J[q];
    __syncthreads();
    const int64_t E = (int64_t)blockIdx.x * kWaveElems + w;
    const bool live = E < nel;
    for (int row = lane; row < F2; row += 64) {            // row = k LF + j
        float v[LF];
        int32_t id[LF];
        bool own[LF];
        const int64_t L0 = E * F3 + (int64_t)row * LF;
        if (live) load_row<LF>(id, own, lidf, ownf, L0);
#pragma unroll
        for (int i = 0; i < LF; ++i) v[i] = (live && own[i]) ? rf[id[i]] : 0.f;
#pragma unroll
        for (int a = 0; a < LC; ++a) {
            float s = 0.f;
#pragma unroll
            for (int i = 0; i < LF; ++i) s += sJ[i * LC + a] * v[i];
            s1[w][row * LC + a] = s;
        }
    }
    sem::wave_fence_barrier();
    for (int o = lane; o < LF * LC * LC; o += 64) {
        const int a = o % LC, b = (o / LC) % LC, k = o / (LC * LC);
        float s = 0.f;
#pragma unroll
        for (int j = 0; j < LF; ++j) s += sJ[j * LC + b] * s1[w][(k * LF + j) * LC + a];
        s2[w][o] = s;
    }
    sem::wave_fence_barrier();
    for (int o = lane; o < C3; o += 64) {
        const int a = o % LC, b = (o / LC) % LC, c = o / (LC * LC);
        float s = 0.f;
#pragma unroll
        for (int k = 0; k < LF; ++k) s += sJ[k * LC + c] * s2[w][(k * LC + b) * LC + a];
        if (live) blc[E * C3 + o] = s;
    }
}

// x_f += P x_c at the owner nodes of each fine element
template <int LF, int LC>
__global__ void __launch_bounds__(64 * kWaveElems)
prolong_p_wave_kernel(float* __restrict__ xf, const float* __restrict__ xc, const int32_t* __restrict__ lidf,
                      const uint8_t* __restrict__ ownf, const int32_t* __restrict__ lidc, const float* __restrict__ J,
                      int64_t nel, const int* __restrict__ skip) {
    if (skip && *skip) return;
    constexpr int F2 = LF * LF, F3 = F2 * LF, C3 = LC * LC * LC;
    __shared__ float sJ[LF * LC];
    __shared__ float sc[kWaveElems][C3];              // [c][b][a]
    __shared__ float t1[kWaveElems][LC * LC * LF];    // [c][b][i]
    __shared__ float t2[kWaveElems][LC * LF * LF];    // [c][j][i]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int q = tid; q < LF * LC; q += blockDim.x) sJ[q] = J[q];
    __syncthreads();
    const int64_t E = (int64_t)blockIdx.x * kWaveElems + w;
    const bool live = E < nel;
    for (int o = lane; o < C3; o += 64) {
        const int32_t id = live ? lidc[E * C3 + o] : -1;
        sc[w][o] = id >= 0 ? xc[id] : 0.f;
    }
    sem::wave_fence_barrier();
    for (int o = lane; o < LC * LC * LF; o += 64) {
        const int i = o % LF, cb = o / LF;
        float s = 0.f;
#pragma unroll
        for (int a = 0; a < LC; ++a) s += sJ[i * LC + a] * sc[w][cb * LC + a];
        t1[w][o] = s;
    }
    sem::wave_fence_barrier();
    for (int o = lane; o < LC * LF * LF; o += 64) {
        const int i = o % LF, j = (o / LF) % LF, c = o / (LF * LF);
        float s = 0.f;
#pragma unroll
        for (int b = 0; b < LC; ++b) s += sJ[j * LC + b] * t1[w][(c * LC + b) * LF + i];
        t2[w][o] = s;
    }
    sem::wave_fence_barrier();
    if (!live) return;
    for (int row = lane; row < F2; row += 64) {            // row = k LF + j
        const int k = row / LF, j = row % LF;
        const int64_t L0 = E * F3 + (int64_t)row * LF;
        int32_t id[LF];
        bool own[LF];
        load_row<LF>(id, own, lidf, ownf, L0);
        // the row's owner nodes are distinct unique nodes: all loads first, then the stores
        float old[LF];
#pragma unroll
        for (int i = 0; i < LF; ++i) old[i] = own[i] ? xf[id[i]] : 0.f;
#pragma unroll
        for (int i = 0; i < LF; ++i) {
            float s = 0.f;
#pragma unroll
            for (int c = 0; c < LC; ++c) s += sJ[k * LC + c] * t2[w][(c * LF + j) * LF + i];
            if (own[i]) xf[id[i]] = old[i] + s;
        }
    }
}

// x_f += P x_c of an h-transfer (lx = 2 boxes): one thread per fine local node,
// adding at its owner copy the parent's trilinear interpolant at its vertex
__global__ void prolong_h_kernel(float* __restrict__ xf, const float* __restrict__ xc, const int32_t* __restrict__ lidf,
                                 const uint8_t* __restrict__ ownf, const int32_t* __restrict__ lidc, int nf, int nc,
                                 int64_t nelf, const int* __restrict__ skip) {
    if (skip && *skip) return;
    MG_LOOP(L, nelf * 8) {
        if (!ownf[L]) continue;
        const int64_t e = L >> 3;
        const int i = (int)(L & 7), ix = i & 1, iy = (i >> 1) & 1, iz = i >> 2;
        const int64_t ex = e % nf, ey = (e / nf) % nf, ez = e / ((int64_t)nf * nf);
        const int px = (int)(ex & 1), py = (int)(ey & 1), pz = (int)(ez & 1);
        const int64_t E = (ex >> 1) + nc * ((ey >> 1) + (int64_t)nc * (ez >> 1));
        float s = 0.f;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int ax = c & 1, ay = (c >> 1) & 1, az = c >> 2;
            const float wgt = (float)(ax ? px + ix : 2 - px - ix) * (float)(ay ? py + iy : 2 - py - iy) *
                              (float)(az ? pz + iz : 2 - pz - iz) * 0.125f;
            if (wgt == 0.f) continue;
            const int32_t id = lidc[E * 8 + c];
            if (id >= 0) s += wgt * xc[id];
        }
        xf[lidf[L]] += s;
    }
}

// P^T of an h-transfer (lx = 2 boxes): one thread per coarse element node c,
// summing over the 8 children and their 8 nodes with the parent's trilinear
// basis at the child's vertices
__global__ void restrict_h_kernel(float* __restrict__ blc, const float* __restrict__ rf, const int32_t* __restrict__ lidf,
                                  const uint8_t* __restrict__ ownf, int nf, int nc, int64_t nelc,
                                  const int* __restrict__ skip) {
    if (skip && *skip) return;
    MG_LOOP(t, nelc * 8) {
        const int64_t E = t >> 3;
        const int c = (int)(t & 7), ax = c & 1, ay = (c >> 1) & 1, az = c >> 2;
        const int64_t ecx = E % nc, ecy = (E / nc) % nc, ecz = E / ((int64_t)nc * nc);
        float acc = 0.f;
        for (int ch = 0; ch < 8; ++ch) {
            const int px = ch & 1, py = (ch >> 1) & 1, pz = ch >> 2;
            const int64_t ef = (2 * ecx + px) + nf * ((2 * ecy + py) + (int64_t)nf * (2 * ecz + pz));
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int ix = i & 1, iy = (i >> 1) & 1, iz = i >> 2;
                // phi_a(eta), eta = -1 + p + i in {-1, 0, 1}: 1, 1/2 or 0
                const float wx = (float)(ax ? px + ix : 2 - px - ix) * 0.5f;
                const float wy = (float)(ay ? py + iy : 2 - py - iy) * 0.5f;
                const float wz = (float)(az ? pz + iz : 2 - pz - iz) * 0.5f;
                const float wgt = wx * wy * wz;
                const int64_t L = ef * 8 + i;
                if (wgt != 0.f && ownf[L]) acc += wgt * rf[lidf[L]];
            }
        }
        blc[t] = acc;
    }
}

// dispatch of the p-transfer wave kernels for the (lxf, lxc) pairs the level
// shapes produce; false if there is none (the workgroup-per-element kernels run)
#define MG_PAIRS(X) X(3, 2) X(4, 2) X(5, 2) X(6, 3) X(7, 3) X(8, 4) X(9, 4) X(10, 5) X(11, 5) X(12, 6)
bool restrict_p_wave(hipStream_t st, int lf, int lc, float* blc, const float* rf, const int32_t* lidf,
                     const uint8_t* ownf, const float* J, int64_t nel, const int* skip) {
    const unsigned g = (unsigned)((nel + kWaveElems - 1) / kWaveElems);
#define MG_R(F, C) if (lf == F && lc == C) { \
        restrict_p_wave_kernel<F, C><<<g, 64 * kWaveElems, 0, st>>>(blc, rf, lidf, ownf, J, nel, skip); return true; }
    MG_PAIRS(MG_R)
#undef MG_R
    return false;
}
bool prolong_p_wave(hipStream_t st, int lf, int lc, float* xf, const float* xc, const int32_t* lidf,
                    const uint8_t* ownf, const int32_t* lidc, const float* J, int64_t nel, const int* skip) {
    const unsigned g = (unsigned)((nel + kWaveElems - 1) / kWaveElems);
#define MG_P(F, C) if (lf == F && lc == C) { \
        prolong_p_wave_kernel<F, C><<<g, 64 * kWaveElems, 0, st>>>(xf, xc, lidf, ownf, lidc, J, nel, skip); return true; }
    MG_PAIRS(MG_P)
#undef MG_P
    return false;
}
#undef MG_PAIRS

// Coarsest level: x = Ainv b with b assembled from the restricted local field
// (bl) or given (bin).  Every workgroup assembles all of b into LDS, then each
// of its waves forms kCoarseRows rows of Ainv b, the lanes striding along the
// row (coalesced) and a wave sum closing it.
constexpr int kCoarseRows = 4;
__global__ void __launch_bounds__(kBlock)
coarse_kernel(float* __restrict__ x, const float* __restrict__ bin, const float* __restrict__ bl,
              const float* __restrict__ ainv, const int32_t* __restrict__ uoff, const int32_t* __restrict__ uidx,
              int nu, const int* __restrict__ skip) {
    if (skip && *skip) return;
    __shared__ float sb[kCoarseMax];
    for (int u = threadIdx.x; u < nu; u += blockDim.x) sb[u] = bl ? assemble_local(bl, uoff, uidx, u) : bin[u];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int row0 = (blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)) * kCoarseRows;
    for (int q = 0; q < kCoarseRows; ++q) {
        const int i = row0 + q;
        if (i >= nu) break;                       // uniform across the wave
        const float* row = ainv + (int64_t)i * nu;
        float s = 0.f;
        for (int j = lane; j < nu; j += 64) s += row[j] * sb[j];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) x[i] = s;
    }
}

unsigned coarse_grid(int64_t nu) {
    const int64_t rows_per_block = (kBlock / 64) * kCoarseRows;
    return (unsigned)std::max<int64_t>(1, (nu + rows_per_block - 1) / rows_per_block);
}

// Galerkin level operator: w_l = M_e u_e, one thread per local node of the
// lx = 2 elements (M row-major per element, 8 x 8; Dirichlet nodes read 0)
__global__ void dense_ax_kernel(float* __restrict__ wl, const float* __restrict__ u, const float* __restrict__ M,
                                const int32_t* __restrict__ lid, int64_t nloc, const int* __restrict__ skip) {
    if (skip && *skip) return;
    MG_LOOP(L, nloc) {
        const int64_t e8 = L & ~(int64_t)7;
        const float* row = M + 8 * L;
        float s = 0.f;
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const int32_t id = lid[e8 + a];
            s += row[a] * (id >= 0 ? u[id] : 0.f);
        }
        wl[L] = s;
    }
}

// The coarse basis function bc (0..7, lexicographic over the 2 x 2 x 2 coarse
// element) interpolated to the lf^3 nodes of every element: J[i][a] (lf x 2).
__global__ void basis_field_kernel(double* __restrict__ ul, const double* __restrict__ J, int lf, int bc,
                                   int64_t n) {
    const int f3 = lf * lf * lf;
    const int ax = bc & 1, ay = (bc >> 1) & 1, az = bc >> 2;
    MG_LOOP(L, n) {
        const int q = (int)(L % f3);
        const int i = q % lf, j = (q / lf) % lf, k = q / (lf * lf);
        ul[L] = J[k * 2 + az] * J[j * 2 + ay] * J[i * 2 + ax];
    }
}

// Column bc of the Galerkin element matrices: M_e[a][bc] = sum_i J3[i][a] (A_e J3[:, bc])[i]
// from wl = A (basis field bc), one thread per (element, a).
__global__ void project_basis_kernel(double* __restrict__ M, const double* __restrict__ wl,
                                     const double* __restrict__ J, int lf, int bc, int64_t nel) {
    const int f3 = lf * lf * lf;
    MG_LOOP(t, nel * 8) {
        const int64_t e = t >> 3;
        const int a = (int)(t & 7);
        const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
        const double* w = wl + e * f3;
        double s = 0.0;
        for (int q = 0; q < f3; ++q) {
            const int i = q % lf, j = (q / lf) % lf, k = q / (lf * lf);
            s += J[k * 2 + az] * J[j * 2 + ay] * J[i * 2 + ax] * w[q];
        }
        M[e * 64 + a * 8 + bc] = s;
    }
}

// h-Galerkin: M_E = sum over the 8 children c of J_c^T M_c J_c, J_c the
// parent's trilinear basis at the child's vertices (reference coordinate
// -1 + parity + i); one thread per (coarse element, a, b).
__global__ void galerkin_h_kernel(double* __restrict__ Mc, const double* __restrict__ Mf, int nf, int nc,
                                  int64_t nelc) {
    MG_LOOP(t, nelc * 64) {
        const int64_t E = t >> 6;
        const int a = (int)((t >> 3) & 7), b = (int)(t & 7);
        const int64_t ecx = E % nc, ecy = (E / nc) % nc, ecz = E / ((int64_t)nc * nc);
        double s = 0.0;
        for (int ch = 0; ch < 8; ++ch) {
            const int px = ch & 1, py = (ch >> 1) & 1, pz = ch >> 2;
            const int64_t ef = (2 * ecx + px) + nf * ((2 * ecy + py) + (int64_t)nf * (2 * ecz + pz));
            const double* m = Mf + ef * 64;
            double ja[8], jb[8];
            for (int i = 0; i < 8; ++i) {    // J_c[i][a]: product over x, y, z of phi_{a_d}(-1 + p_d + i_d)
                const int ix = i & 1, iy = (i >> 1) & 1, iz = i >> 2;
                auto phi = [](int p, int ii, int aa) {
                    const double eta = -1.0 + p + ii;
                    return aa ? 0.5 * (1.0 + eta) : 0.5 * (1.0 - eta);
                };
                ja[i] = phi(px, ix, a & 1) * phi(py, iy, (a >> 1) & 1) * phi(pz, iz, a >> 2);
                jb[i] = phi(px, ix, b & 1) * phi(py, iy, (b >> 1) & 1) * phi(pz, iz, b >> 2);
            }
            for (int i = 0; i < 8; ++i) {
                if (ja[i] == 0.0) continue;
                double r = 0.0;
                for (int j = 0; j < 8; ++j) r += m[i * 8 + j] * jb[j];
                s += ja[i] * r;
            }
        }
        Mc[t] = s;
    }
}

// the diagonals of the element matrices in the local layout
__global__ void mat_diag_kernel(double* __restrict__ dl, const double* __restrict__ M, int64_t nloc) {
    MG_LOOP(L, nloc) dl[L] = M[8 * L + (L & 7)];
}

// ----------------------------------------------------------------- set-up
__global__ void to_f32_kernel(float* __restrict__ out, const double* __restrict__ in, double scale, int64_t n) {
    MG_LOOP(L, n) out[L] = (float)(scale * in[L]);
}

__global__ void to_f64_kernel(double* __restrict__ out, const float* __restrict__ in, int64_t n,
                              const int* __restrict__ skip) {
    if (skip && *skip) return;
    MG_LOOP(L, n) out[L] = (double)in[L];
}

__global__ void from_f64_kernel(float* __restrict__ out, const double* __restrict__ in, int64_t n,
                                const int* __restrict__ skip) {
    if (skip && *skip) return;
    MG_LOOP(L, n) out[L] = (float)in[L];
}

__global__ void add_scaled_kernel(double* __restrict__ d, const double* __restrict__ b, double s, int64_t n) {
    MG_LOOP(L, n) d[L] += s * b[L];
}

__global__ void scale_f64_kernel(double* __restrict__ d, double s, int64_t n) {
    MG_LOOP(L, n) d[L] *= s;
}

__global__ void scale_f32_kernel(float* __restrict__ v, float s, int64_t n) {
    MG_LOOP(L, n) v[L] *= s;
}

__global__ void zero_f32_kernel(float* __restrict__ v, int64_t n) {
    MG_LOOP(L, n) v[L] = 0.f;
}

// Minv_u = 1 / (assembled diagonal) from the element-local diagonal dl
__global__ void diag_recip_kernel(float* __restrict__ minv, const double* __restrict__ dl,
                                  const int32_t* __restrict__ uoff, const int32_t* __restrict__ uidx, int64_t nu) {
    MG_LOOP(u, nu) minv[u] = (float)(1.0 / assemble_local(dl, uoff, uidx, u));
}

// own[L] = 1 for the first local copy of a unique node, 0 otherwise (and on
// Dirichlet nodes)
__global__ void owner_kernel(uint8_t* __restrict__ own, const int32_t* __restrict__ lid,
                             const int32_t* __restrict__ uoff, const int32_t* __restrict__ uidx, int64_t n) {
    MG_LOOP(L, n) {
        const int32_t u = lid[L];
        own[L] = (u >= 0 && uidx[uoff[u]] == (int32_t)L) ? 1 : 0;
    }
}

// unit vector e_j in the local layout (every copy of unique node j)
__global__ void unit_local_kernel(double* __restrict__ ul, const int32_t* __restrict__ lid, int64_t j, int64_t n) {
    MG_LOOP(L, n) ul[L] = lid[L] == (int32_t)j ? 1.0 : 0.0;
}

__global__ void column_kernel(double* __restrict__ col, const double* __restrict__ wl,
                              const int32_t* __restrict__ uoff, const int32_t* __restrict__ uidx, int64_t nu) {
    MG_LOOP(u, nu) col[u] = assemble_local(wl, uoff, uidx, u);
}

// ---- Lanczos on M = D^-1/2 A D^-1/2 (float32 vectors, float64 partial sums)
__device__ __forceinline__ double block_sum(double v, double* s_red) {
    v = sem::wave_sum(v);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += s_red[q];
    return t;
}

// deterministic start vector: a hash of the index mapped to [-1, 1)
__global__ void start_kernel(float* __restrict__ v, int64_t nu, uint32_t seed, double* __restrict__ part) {
    __shared__ double s_red[kBlock / 64];
    double s = 0.0;
    MG_LOOP(u, nu) {
        uint32_t h = (uint32_t)u * 2654435761u ^ seed;
        h ^= h >> 16; h *= 0x7feb352du; h ^= h >> 15; h *= 0x846ca68bu; h ^= h >> 16;
        const float val = (float)((double)h * (2.0 / 4294967296.0) - 1.0);
        v[u] = val;
        s += (double)val * val;
    }
    s = block_sum(s, s_red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out = D^-1/2 v
__global__ void half_jacobi_kernel(float* __restrict__ out, const float* __restrict__ v,
                                   const float* __restrict__ minv, int64_t nu) {
    MG_LOOP(u, nu) out[u] = sqrtf(minv[u]) * v[u];
}

// w = D^-1/2 (A p) - beta vprev and partials of w . v
__global__ void lanczos_w_kernel(float* __restrict__ w, const float* __restrict__ wl, const float* __restrict__ v,
                                 const float* __restrict__ vprev, const float* __restrict__ minv, float beta,
                                 const int32_t* __restrict__ uoff, const int32_t* __restrict__ uidx, int64_t nu,
                                 double* __restrict__ part) {
    __shared__ double s_red[kBlock / 64];
    double s = 0.0;
    MG_LOOP(u, nu) {
        const float wv = sqrtf(minv[u]) * assemble_local(wl, uoff, uidx, u) - beta * vprev[u];
        w[u] = wv;
        s += (double)wv * v[u];
    }
    s = block_sum(s, s_red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// w -= alpha v and partials of w . w
__global__ void lanczos_orth_kernel(float* __restrict__ w, const float* __restrict__ v, float alpha, int64_t nu,
                                    double* __restrict__ part) {
    __shared__ double s_red[kBlock / 64];
    double s = 0.0;
    MG_LOOP(u, nu) {
        const float wv = w[u] - alpha * v[u];
        w[u] = wv;
        s += (double)wv * wv;
    }
    s = block_sum(s, s_red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// vprev = v, v = w / beta
__global__ void lanczos_next_kernel(float* __restrict__ vprev, float* __restrict__ v, const float* __restrict__ w,
                                    float inv_beta, int64_t nu) {
    MG_LOOP(u, nu) {
        vprev[u] = v[u];
        v[u] = w[u] * inv_beta;
    }
}

// number of eigenvalues below x of the symmetric tridiagonal (a, b) (Sturm count)
int sturm_count(const std::vector<double>& a, const std::vector<double>& b, double x) {
    int cnt = 0;
    double q = 1.0;
    for (size_t i = 0; i < a.size(); ++i) {
        const double bb = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
        q = a[i] - x - (i > 0 ? bb / q : 0.0);
        if (q == 0.0) q = -1e-300;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

// largest eigenvalue of the symmetric tridiagonal matrix by bisection
double tridiag_max(const std::vector<double>& a, const std::vector<double>& b) {
    double lo = 1e300, hi = -1e300;
    for (size_t i = 0; i < a.size(); ++i) {      // Gershgorin
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < a.size() ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    const int m = (int)a.size();
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(hi)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (sturm_count(a, b, mid) >= m) hi = mid; else lo = mid;
    }
    return hi;
}

// 1-D matrix of the coarse Lagrange basis (nodes xc) at the fine points xf:
// J[i][a] = prod_{b != a} (xf_i - xc_b) / (xc_a - xc_b)
void lagrange_matrix(const std::vector<double>& xf, const std::vector<double>& xc, float* J) {
    const int nf = (int)xf.size(), ncn = (int)xc.size();
    for (int i = 0; i < nf; ++i)
        for (int a = 0; a < ncn; ++a) {
            double v = 1.0;
            for (int b = 0; b < ncn; ++b)
                if (b != a) v *= (xf[i] - xc[b]) / (xc[a] - xc[b]);
            J[i * ncn + a] = (float)v;
        }
}

}  // namespace

struct MgLevel {
    int n = 0, lx = 0;
    double amp = 0.0;                 // deformation amplitude of this level's box
    int64_t nel = 0, nloc = 0, nu = 0;
    sem_gs_t gs = nullptr;
    bool own_gs = false;
    sem::AxArgs A{};                  // float32 solver form (factors float32 or bfloat16)
    sem::AxKind axkind = sem::AxKind::F32;
    float* minv = nullptr;
    float *x = nullptr, *r = nullptr, *d = nullptr, *b = nullptr;   // unique
    float *wl = nullptr, *bl = nullptr;                             // local
    uint8_t* own = nullptr;
    double lmax = 0.0;
    float c0 = 0.f;
    std::vector<float> c1, c2;        // Chebyshev steps 1 .. degree-1
    int kind = -1;                    // transfer to the next level: 0 p, 1 h
    float* J = nullptr;               // [2][lx][lx of the next level]
    float* M = nullptr;               // Galerkin level: 8 x 8 element matrices (else null)
};

struct sem_mg_s {
    sem_ctx_t ctx = nullptr;
    std::vector<MgLevel> L;
    int degree = 2;
    double lo = 0.3, hi = 1.1;
    bool singular = false;
    float* ainv = nullptr;            // dense coarsest inverse
    float *b0 = nullptr, *x0 = nullptr;   // float32 copies for float64 callers
    double* part = nullptr;           // kVecGrid partial sums
    std::vector<void*> allocs;
    // The V-cycle is a fixed sequence of about 12 launches per level; it can be
    // replayed as a captured HIP graph (one per set of vector and flag
    // pointers).  Measured at 32^3 / lx = 8 the graph is no faster than the
    // launches one by one, so it is off unless asked for.
    bool graphs = false;
    hipStream_t cap_stream = nullptr;     // private capture stream (default priority)
    struct Cached { const void* z; const void* r; const int* skip; bool f64; hipGraphExec_t exec; };
    std::vector<Cached> cache;
};

namespace {

int mg_alloc(sem_mg_t mg, void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return sem::check_hip(mg->ctx, e, "sem_mg_create: hipMalloc");
    mg->allocs.push_back(*p);
    return SEM_OK;
}

// host sum of the first n partials, in index order
int sum_parts(sem_mg_t mg, int n, double* out) {
    std::vector<double> h(n);
    SEM_HIP(mg->ctx, hipMemcpyAsync(h.data(), mg->part, sizeof(double) * n, hipMemcpyDeviceToHost,
                                    mg->ctx->stream));
    SEM_HIP(mg->ctx, hipStreamSynchronize(mg->ctx->stream));
    double s = 0.0;
    for (int q = 0; q < n; ++q) s += h[q];
    *out = s;
    return SEM_OK;
}

int level_ax(sem_mg_t mg, MgLevel& lv, float* wl, const float* u, const int* skip) {
    if (lv.M) {
        dense_ax_kernel<<<vgrid(lv.nloc), kBlock, 0, mg->ctx->stream>>>(wl, u, lv.M, lv.gs->lid, lv.nloc, skip);
        SEM_LAUNCH_CHECK(mg->ctx);
        return SEM_OK;
    }
    return sem::launch_ax(mg->ctx, lv.axkind, lv.A, wl, u, skip, nullptr, lv.gs->lid);
}

// lmax of D^-1 A on level lv: the largest Ritz value of `steps` Lanczos steps
int estimate_lmax(sem_mg_t mg, MgLevel& lv, int steps, uint32_t seed) {
    hipStream_t st = mg->ctx->stream;
    const int64_t nu = lv.nu;
    const unsigned g = vgrid(nu);
    float *v = lv.r, *vprev = lv.b, *w = lv.x, *p = lv.d;
    const int32_t *uoff = lv.gs->uoff, *uidx = lv.gs->uidx;
    start_kernel<<<g, kBlock, 0, st>>>(v, nu, seed, mg->part);
    SEM_LAUNCH_CHECK(mg->ctx);
    double nn;
    int rc = sum_parts(mg, (int)g, &nn);
    if (rc) return rc;
    scale_f32_kernel<<<g, kBlock, 0, st>>>(v, (float)(1.0 / std::sqrt(nn)), nu);
    zero_f32_kernel<<<g, kBlock, 0, st>>>(vprev, nu);
    SEM_LAUNCH_CHECK(mg->ctx);
    std::vector<double> a, b;
    float beta = 0.f;
    for (int j = 0; j < steps; ++j) {
        half_jacobi_kernel<<<g, kBlock, 0, st>>>(p, v, lv.minv, nu);
        rc = level_ax(mg, lv, lv.wl, p, nullptr);
        if (rc) return rc;
        lanczos_w_kernel<<<g, kBlock, 0, st>>>(w, lv.wl, v, vprev, lv.minv, j ? beta : 0.f, uoff, uidx, nu,
                                               mg->part);
        SEM_LAUNCH_CHECK(mg->ctx);
        double alpha;
        rc = sum_parts(mg, (int)g, &alpha);
        if (rc) return rc;
        lanczos_orth_kernel<<<g, kBlock, 0, st>>>(w, v, (float)alpha, nu, mg->part);
        SEM_LAUNCH_CHECK(mg->ctx);
        double ww;
        rc = sum_parts(mg, (int)g, &ww);
        if (rc) return rc;
        a.push_back(alpha);
        const double bj = std::sqrt(std::max(ww, 0.0));
        if (j + 1 == steps || bj <= 1e-7 * std::fabs(alpha)) break;
        b.push_back(bj);
        beta = (float)bj;
        lanczos_next_kernel<<<g, kBlock, 0, st>>>(vprev, v, w, (float)(1.0 / bj), nu);
        SEM_LAUNCH_CHECK(mg->ctx);
    }
    b.resize(a.size() > 0 ? a.size() - 1 : 0);
    lv.lmax = tridiag_max(a, b);
    return SEM_OK;
}

void set_chebyshev(sem_mg_t mg, MgLevel& lv) {
    const double theta = 0.5 * (mg->hi + mg->lo) * lv.lmax, delta = 0.5 * (mg->hi - mg->lo) * lv.lmax;
    const double sigma = theta / delta;
    lv.c0 = (float)(1.0 / theta);
    lv.c1.assign(mg->degree, 0.f);
    lv.c2.assign(mg->degree, 0.f);
    double rho = 1.0 / sigma;
    for (int m = 1; m < mg->degree; ++m) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        lv.c1[m] = (float)(rn * rho);
        lv.c2[m] = (float)(2.0 * rn / delta);
        rho = rn;
    }
}

// the V-cycle on float32 unique vectors of level 0: x = V(b)
int vcycle(sem_mg_t mg, float* xout, const float* bin, const int* skip) {
    hipStream_t st = mg->ctx->stream;
    const int nl = (int)mg->L.size();
    auto& Ls = mg->L;
    if (nl == 1) {
        MgLevel& c = Ls[0];
        coarse_kernel<<<coarse_grid(c.nu), kBlock, 0, st>>>(xout, bin, nullptr, mg->ainv, c.gs->uoff, c.gs->uidx,
                                                    (int)c.nu, skip);
        SEM_LAUNCH_CHECK(mg->ctx);
        return SEM_OK;
    }
    int rc;
    for (int q = 0; q + 1 < nl; ++q) {
        MgLevel& lv = Ls[q];
        MgLevel& nx = Ls[q + 1];
        const unsigned g = vgrid(lv.nu);
        const int32_t *uoff = lv.gs->uoff, *uidx = lv.gs->uidx;
        float* x = q == 0 ? xout : lv.x;
        cheb_first_kernel<<<g, kBlock, 0, st>>>(x, lv.r, lv.d, q == 0 ? nullptr : lv.b, q == 0 ? bin : nullptr,
                                                q == 0 ? nullptr : lv.bl, lv.minv, lv.c0, uoff, uidx, lv.nu, skip);
        for (int m = 1; m < mg->degree; ++m) {
            if ((rc = level_ax(mg, lv, lv.wl, lv.d, skip))) return rc;
            cheb_step_kernel<<<g, kBlock, 0, st>>>(x, lv.r, lv.d, lv.wl, lv.minv, lv.c1[m], lv.c2[m], uoff, uidx,
                                                   lv.nu, skip);
        }
        if ((rc = level_ax(mg, lv, lv.wl, lv.d, skip))) return rc;
        cheb_resid_kernel<<<g, kBlock, 0, st>>>(lv.r, lv.wl, uoff, uidx, lv.nu, skip);
        if (lv.kind == 1 && lv.lx == 2)
            restrict_h_kernel<<<vgrid(8 * nx.nel), kBlock, 0, st>>>(nx.bl, lv.r, lv.gs->lid, lv.own, lv.n, nx.n,
                                                                    nx.nel, skip);
        else if (lv.kind != 0 || !restrict_p_wave(st, lv.lx, nx.lx, nx.bl, lv.r, lv.gs->lid, lv.own, lv.J, nx.nel,
                                                  skip))
            restrict_kernel<<<(unsigned)nx.nel, kBlock, 0, st>>>(nx.bl, lv.r, lv.gs->lid, lv.own, lv.J, lv.lx,
                                                                  nx.lx, lv.kind, lv.n, nx.n, nx.nel, skip);
        SEM_LAUNCH_CHECK(mg->ctx);
    }
    {
        MgLevel& c = Ls[nl - 1];
        coarse_kernel<<<coarse_grid(c.nu), kBlock, 0, st>>>(c.x, nullptr, c.bl, mg->ainv, c.gs->uoff, c.gs->uidx,
                                                    (int)c.nu, skip);
        SEM_LAUNCH_CHECK(mg->ctx);
    }
    for (int q = nl - 2; q >= 0; --q) {
        MgLevel& lv = Ls[q];
        MgLevel& nx = Ls[q + 1];
        const unsigned g = vgrid(lv.nu);
        const int32_t *uoff = lv.gs->uoff, *uidx = lv.gs->uidx;
        float* x = q == 0 ? xout : lv.x;
        const float* b = q == 0 ? bin : lv.b;
        const int f3 = lv.lx * lv.lx * lv.lx;
        if (lv.kind == 1 && lv.lx == 2)
            prolong_h_kernel<<<vgrid(8 * lv.nel), kBlock, 0, st>>>(x, nx.x, lv.gs->lid, lv.own, nx.gs->lid, lv.n,
                                                                   nx.n, lv.nel, skip);
        else if (lv.kind != 0 || !prolong_p_wave(st, lv.lx, nx.lx, x, nx.x, lv.gs->lid, lv.own, nx.gs->lid, lv.J,
                                                 lv.nel, skip))
            prolong_kernel<<<(unsigned)lv.nel, f3 <= 64 ? 64 : kBlock, 0, st>>>(x, nx.x, lv.gs->lid, lv.own,
                                                                                nx.gs->lid, lv.J, lv.lx, nx.lx,
                                                                                lv.kind, lv.n, nx.n, lv.nel, skip);
        if ((rc = level_ax(mg, lv, lv.wl, x, skip))) return rc;
        cheb_post_kernel<<<g, kBlock, 0, st>>>(x, lv.r, lv.d, b, lv.wl, lv.minv, lv.c0, uoff, uidx, lv.nu, skip);
        for (int m = 1; m < mg->degree; ++m) {
            if ((rc = level_ax(mg, lv, lv.wl, lv.d, skip))) return rc;
            cheb_step_kernel<<<g, kBlock, 0, st>>>(x, lv.r, lv.d, lv.wl, lv.minv, lv.c1[m], lv.c2[m], uoff, uidx,
                                                   lv.nu, skip);
        }
        SEM_LAUNCH_CHECK(mg->ctx);
    }
    return SEM_OK;
}

// level shapes (n, lx), finest first, and the kind of transfer to the next
void level_shapes(int n, int lx, int n_coarse, std::vector<int>& ns, std::vector<int>& lxs,
                  std::vector<int>& kinds) {
    while (lx > 2) {
        ns.push_back(n); lxs.push_back(lx); kinds.push_back(0);
        lx = std::max(2, lx / 2);
    }
    while (n % 2 == 0 && n / 2 >= n_coarse) {
        ns.push_back(n); lxs.push_back(2); kinds.push_back(1);
        n /= 2;
    }
    ns.push_back(n); lxs.push_back(lx); kinds.push_back(-1);
}

}  // namespace

namespace sem {

// Cholesky factorisation and inverse of an SPD matrix (row-major, n x n), in place
bool spd_inverse(std::vector<double>& A, int n) {
    std::vector<double> Lf(A);
    for (int j = 0; j < n; ++j) {
        double d = Lf[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) d -= Lf[(size_t)j * n + k] * Lf[(size_t)j * n + k];
        if (!(d > 0.0)) return false;
        d = std::sqrt(d);
        Lf[(size_t)j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double s = Lf[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) s -= Lf[(size_t)i * n + k] * Lf[(size_t)j * n + k];
            Lf[(size_t)i * n + j] = s / d;
        }
    }
    // columns of the inverse: L L^T x = e_c
    std::vector<double> y(n);
    for (int c = 0; c < n; ++c) {
        for (int i = 0; i < n; ++i) {
            double s = i == c ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) s -= Lf[(size_t)i * n + k] * y[k];
            y[i] = s / Lf[(size_t)i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = y[i];
            for (int k = i + 1; k < n; ++k) s -= Lf[(size_t)k * n + i] * y[k];
            y[i] = s / Lf[(size_t)i * n + i];
        }
        for (int i = 0; i < n; ++i) A[(size_t)i * n + c] = y[i];
    }
    return true;
}


sem_gs_t mg_plan(sem_mg_t mg) { return mg && !mg->L.empty() ? mg->L[0].gs : nullptr; }
int64_t mg_nel(sem_mg_t mg) { return mg && !mg->L.empty() ? mg->L[0].nel : 0; }

// the launches of one V-cycle on the context's stream (converting in and out
// for float64 callers)
int mg_launch(sem_mg_t mg, void* z, const void* r, bool f64, const int* skip) {
    hipStream_t st = mg->ctx->stream;
    const int64_t nu = mg->L[0].nu;
    const unsigned g = vgrid(nu);
    if (!f64) return vcycle(mg, (float*)z, (const float*)r, skip);
    from_f64_kernel<<<g, kBlock, 0, st>>>(mg->b0, (const double*)r, nu, skip);
    int rc = vcycle(mg, mg->x0, mg->b0, skip);
    if (rc) return rc;
    to_f64_kernel<<<g, kBlock, 0, st>>>((double*)z, mg->x0, nu, skip);
    SEM_LAUNCH_CHECK(mg->ctx);
    return SEM_OK;
}

// the captured graph of the V-cycle for these pointers (captured on first use)
int mg_graph(sem_mg_t mg, void* z, const void* r, bool f64, const int* skip, hipGraphExec_t* out) {
    for (const auto& c : mg->cache)
        if (c.z == z && c.r == r && c.skip == skip && c.f64 == f64) { *out = c.exec; return SEM_OK; }
    sem_ctx_t ctx = mg->ctx;
    if (!mg->cap_stream) SEM_HIP(ctx, hipStreamCreateWithFlags(&mg->cap_stream, hipStreamNonBlocking));
    hipStream_t saved = ctx->stream;
    ctx->stream = mg->cap_stream;
    hipError_t e = hipStreamBeginCapture(mg->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) { ctx->stream = saved; return sem::check_hip(ctx, e, "hipStreamBeginCapture"); }
    int rc = mg_launch(mg, z, r, f64, skip);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(mg->cap_stream, &graph);
    ctx->stream = saved;
    if (rc) { if (graph) (void)hipGraphDestroy(graph); return rc; }
    if (e != hipSuccess) return sem::check_hip(ctx, e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return sem::check_hip(ctx, e, "hipGraphInstantiate");
    mg->cache.push_back({z, r, skip, f64, exec});
    *out = exec;
    return SEM_OK;
}

int mg_apply(sem_mg_t mg, void* z, const void* r, bool f64, const int* skip) {
    if (!mg->graphs) return mg_launch(mg, z, r, f64, skip);
    hipGraphExec_t exec = nullptr;
    int rc = mg_graph(mg, z, r, f64, skip, &exec);
    if (rc) return rc;
    SEM_HIP(mg->ctx, hipGraphLaunch(exec, mg->ctx->stream));
    return SEM_OK;
}

}  // namespace sem

extern "C" int sem_mg_destroy(sem_mg_t mg) {
    if (!mg) return SEM_OK;
    if (mg->ctx) {
        (void)hipSetDevice(mg->ctx->device);
        (void)hipStreamSynchronize(mg->ctx->stream);
    }
    for (auto& c : mg->cache) (void)hipGraphExecDestroy(c.exec);
    if (mg->cap_stream) (void)hipStreamDestroy(mg->cap_stream);
    for (auto& lv : mg->L)
        if (lv.own_gs) sem_gs_destroy(lv.gs);
    for (void* p : mg->allocs) (void)hipFree(p);
    delete mg;
    return SEM_OK;
}

extern "C" int sem_mg_create(sem_ctx_t ctx, sem_gs_t gs, const sem_operator_t* A, const sem_mg_opts_t* opts,
                             sem_mg_t* out) {
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (!out || !gs || !A || !opts) return sem::fail(ctx, SEM_EINVAL, "sem_mg_create: null argument");
    *out = nullptr;
    if (gs->ctx != ctx) return sem::fail(ctx, SEM_EINVAL, "sem_mg_create: plan belongs to another context");
    if (!sem::lx_ok(A->lx)) return sem::fail(ctx, SEM_EUNSUPPORTED_LX, "sem_mg_create: lx=%d", A->lx);
    const int n = opts->n;
    if (n < 1 || (int64_t)n * n * n != A->nel)
        return sem::fail(ctx, SEM_EINVAL, "sem_mg_create: nel=%lld is not n^3 for n=%d", (long long)A->nel, n);
    if (A->nel * A->lx * A->lx * A->lx != gs->n_local)
        return sem::fail(ctx, SEM_EINVAL, "sem_mg_create: operator size does not match the plan");
    if (A->h1) return sem::fail(ctx, SEM_EINVAL, "sem_mg_create: the levels are built with h1 = 1 (pass h1 = NULL)");
    if ((A->h2b != nullptr) != (opts->h2 > 0.0))
        return sem::fail(ctx, SEM_EINVAL, "sem_mg_create: h2 > 0 exactly when the operator has a mass term");
    if (gs->n_unique == 0) return sem::fail(ctx, SEM_EINVAL, "sem_mg_create: the plan has no unknowns");
    if ((gs->n_masked > 0) != (opts->dirichlet != 0))
        return sem::fail(ctx, SEM_EINVAL, "sem_mg_create: the plan's Dirichlet nodes do not match opts->dirichlet");
    const double* Dp[6] = {A->dx, A->dy, A->dz, A->dxt, A->dyt, A->dzt};
    const double* Gp[6] = {A->g11, A->g22, A->g33, A->g12, A->g13, A->g23};
    for (int q = 0; q < 6; ++q)
        if (!Dp[q] || !Gp[q]) return sem::fail(ctx, SEM_EINVAL, "sem_mg_create: null operator array");
    const int degree = opts->degree > 0 ? opts->degree : 2;
    const double lo = opts->lo > 0 ? opts->lo : 0.15, hi = opts->hi > 0 ? opts->hi : 1.1;
    const int n_coarse = opts->n_coarse > 0 ? opts->n_coarse : 2;
    const int steps = opts->lanczos_steps > 0 ? opts->lanczos_steps : 20;
    if (degree > 16 || !(hi > lo)) return sem::fail(ctx, SEM_EINVAL, "sem_mg_create: bad degree or interval");

    std::vector<int> ns, lxs, kinds;
    level_shapes(n, A->lx, n_coarse, ns, lxs, kinds);
    const int nl = (int)ns.size();
    {   // the coarsest level's unknowns (dense inverse)
        const int nc = ns.back(), lc = lxs.back();
        const int64_t m = (int64_t)nc * (lc - 1);
        const int64_t nuc = opts->dirichlet ? (m - 1) * (m - 1) * (m - 1) : m * m * m;
        if (nuc > kCoarseMax || nuc < 1)
            return sem::fail(ctx, SEM_EINVAL, "sem_mg_create: coarsest level (n=%d, lx=%d) has %lld unknowns, "
                             "outside [1, %lld]", nc, lc, (long long)nuc, (long long)kCoarseMax);
    }

    auto* mg = new sem_mg_s();
    mg->ctx = ctx;
    mg->degree = degree;
    mg->lo = lo;
    mg->hi = hi;
    mg->singular = !opts->dirichlet && !(opts->h2 > 0.0);
    hipStream_t st = ctx->stream;
    auto bail = [&](int code) { sem_mg_destroy(mg); return code; };
#define MG_ALLOC(ptr, bytes) do { int rc_ = mg_alloc(mg, (void**)&(ptr), (bytes)); if (rc_) return bail(rc_); } while (0)
#define MG_TRY(call) do { int rc_ = (call); if (rc_) return bail(rc_); } while (0)
    MG_ALLOC(mg->part, sizeof(double) * kVecGrid);
    mg->L.resize(nl);
    // float64 arrays of the coarsest level, kept until its matrix is built
    std::vector<void*> tmp;
    auto tmp_alloc = [&](void** p, size_t bytes) -> int {
        hipError_t e = hipMalloc(p, bytes);
        if (e != hipSuccess) return sem::check_hip(ctx, e, "sem_mg_create: hipMalloc");
        tmp.push_back(*p);
        return SEM_OK;
    };
    auto free_tmp = [&]() {
        (void)hipStreamSynchronize(st);
        for (void* p : tmp) (void)hipFree(p);
        tmp.clear();
    };
#define MG_TMP(ptr, bytes) do { int rc_ = tmp_alloc((void**)&(ptr), (bytes)); if (rc_) { free_tmp(); return bail(rc_); } } while (0)
#define MG_TTRY(call) do { int rc_ = (call); if (rc_) { free_tmp(); return bail(rc_); } } while (0)

    // Galerkin element matrices (float64, 64 per element) of the current and the
    // next level; freed when set-up ends
    struct Carry {
        std::vector<void*> v;
        ~Carry() { for (void* p : v) (void)hipFree(p); }
    } carry;
    const bool galerkin = opts->galerkin != 0;
    double* cur64 = nullptr;
    for (int q = 0; q < nl; ++q) {
        MgLevel& lv = mg->L[q];
        lv.n = ns[q];
        lv.lx = lxs[q];
        lv.kind = kinds[q];
        lv.nel = (int64_t)lv.n * lv.n * lv.n;
        const int lx = lv.lx, l2 = lx * lx;
        lv.nloc = lv.nel * l2 * lx;
        const int64_t nloc = lv.nloc;
        const unsigned gl = vgrid(nloc);
        const bool gal = galerkin && q > 0 && lx == 2;     // this level is P^T A P of the one above
        const double* D64[6] = {};
        const double* G64[6] = {};
        const double* hb64 = nullptr;
        double* dl = nullptr;               // element diagonal (float64, local)
        MG_TMP(dl, sizeof(double) * nloc);
        if (q == 0) {
            lv.gs = gs;
            lv.amp = opts->amp;
            for (int a = 0; a < 6; ++a) { D64[a] = Dp[a]; G64[a] = Gp[a]; }
            hb64 = A->h2b;
        } else {
            double *x = nullptr, *y = nullptr, *z = nullptr;
            int64_t* ids = nullptr;
            MG_TMP(x, sizeof(double) * nloc);
            MG_TMP(y, sizeof(double) * nloc);
            MG_TMP(z, sizeof(double) * nloc);
            MG_TMP(ids, sizeof(int64_t) * nloc);
            if (gal) {      // the node numbering only
                MG_TTRY(opts->dirichlet ? sem_box_mesh_dirichlet(ctx, lv.n, lx, 0.0, x, y, z, ids)
                                        : sem_box_mesh(ctx, lv.n, lx, 0.0, x, y, z, ids));
                lv.amp = 0.0;
            } else {
                double *bm = nullptr, *Dd = nullptr;
                double* G[6];
                MG_TMP(bm, sizeof(double) * nloc);
                for (int a = 0; a < 6; ++a) MG_TMP(G[a], sizeof(double) * nloc);
                MG_TMP(Dd, sizeof(double) * 2 * l2);
                // a level whose geometry folds (coarse trilinear elements of a strongly
                // deformed box) takes the amplitude halved until det J > 0 everywhere
                double amp = opts->amp, mindet = 0.0;
                for (int halvings = 0;; ++halvings) {
                    MG_TTRY(opts->dirichlet ? sem_box_mesh_dirichlet(ctx, lv.n, lx, amp, x, y, z, ids)
                                            : sem_box_mesh(ctx, lv.n, lx, amp, x, y, z, ids));
                    const int grc = sem_geometry(ctx, x, y, z, lv.nel, lx, G[0], G[1], G[2], G[3], G[4], G[5], bm,
                                                 &mindet);
                    if (grc == SEM_EGEOMETRY && halvings < 20) { amp = halvings == 19 ? 0.0 : 0.5 * amp; continue; }
                    MG_TTRY(grc);
                    break;
                }
                lv.amp = amp;
                std::vector<double> dx(l2), dxt(l2);
                MG_TTRY(sem_gll(lx, nullptr, nullptr, dx.data(), dxt.data()));
                MG_TTRY(sem::check_hip(ctx, hipMemcpy(Dd, dx.data(), sizeof(double) * l2, hipMemcpyHostToDevice),
                                       "sem_mg_create: hipMemcpy"));
                MG_TTRY(sem::check_hip(ctx, hipMemcpy(Dd + l2, dxt.data(), sizeof(double) * l2,
                                                      hipMemcpyHostToDevice), "sem_mg_create: hipMemcpy"));
                for (int a = 0; a < 3; ++a) { D64[a] = Dd; D64[3 + a] = Dd + l2; }
                for (int a = 0; a < 6; ++a) G64[a] = G[a];
                if (opts->h2 > 0.0) {
                    scale_f64_kernel<<<gl, kBlock, 0, st>>>(bm, opts->h2, nloc);   // bm <- h2 bm
                    hb64 = bm;
                }
            }
            std::vector<int64_t> hids(nloc);
            MG_TTRY(sem::check_hip(ctx, hipStreamSynchronize(st), "sem_mg_create: hipStreamSynchronize"));
            MG_TTRY(sem::check_hip(ctx, hipMemcpy(hids.data(), ids, sizeof(int64_t) * nloc, hipMemcpyDeviceToHost),
                                   "sem_mg_create: hipMemcpy"));
            MG_TTRY(sem_gs_setup(ctx, hids.data(), nloc, &lv.gs));
            lv.own_gs = true;
        }
        lv.nu = lv.gs->n_unique;
        // the float64 operator of a re-discretised level (and of the first)
        sem::AxArgs a64{};
        for (int a = 0; a < 6; ++a) { a64.D[a] = D64[a]; a64.G[a] = G64[a]; }
        a64.h1 = nullptr;
        a64.hb = hb64;
        a64.nel = lv.nel;
        a64.lx = lx;
        if (gal) {
            // float32 element matrices for the V-cycle; Jacobi from their diagonals
            MG_ALLOC(lv.M, sizeof(float) * 64 * lv.nel);
            to_f32_kernel<<<vgrid(64 * lv.nel), kBlock, 0, st>>>(lv.M, cur64, 1.0, 64 * lv.nel);
            mat_diag_kernel<<<gl, kBlock, 0, st>>>(dl, cur64, nloc);
        } else {
            // float32 solver form
            for (int a = 0; a < 6; ++a) {
                float* d = nullptr;
                MG_ALLOC(d, sizeof(float) * l2);
                to_f32_kernel<<<1, kBlock, 0, st>>>(d, D64[a], 1.0, l2);
                lv.A.D[a] = d;
                lv.A.G[a] = nullptr;
            }
            const bool bf = q == 0 && opts->fine_bf16;   // bfloat16 factors on the finest level
            lv.axkind = bf ? sem::AxKind::F32_BF16 : sem::AxKind::F32;
            if (bf) {
                uint16_t* gp = nullptr;
                MG_ALLOC(gp, sizeof(uint16_t) * 6 * nloc);
                sem::pack_factors_bf16(st, gp, G64, nullptr, nloc, lx);
                lv.A.Gp = gp;
            } else {
                float* gp = nullptr;
                MG_ALLOC(gp, sizeof(float) * 6 * nloc);
                sem::pack_factors_f32(st, gp, G64, nloc, lx);
                lv.A.Gp = gp;
            }
            lv.A.h1 = nullptr;
            lv.A.hb = nullptr;
            if (hb64) {
                void* hb = nullptr;
                MG_ALLOC(hb, (bf ? sizeof(uint16_t) : sizeof(float)) * nloc);
                if (bf) MG_TTRY(sem_convert(ctx, hb, SEM_BF16, hb64, SEM_F64, nloc));
                else to_f32_kernel<<<gl, kBlock, 0, st>>>((float*)hb, hb64, 1.0, nloc);
                lv.A.hb = hb;
            }
            lv.A.nel = lv.nel;
            lv.A.lx = lx;
            // Jacobi: the assembled diagonal of A (+ h2 B)
            MG_TTRY(sem_ax_diag(ctx, dl, D64[0], nullptr, G64[0], G64[1], G64[2], G64[3], G64[4], G64[5], lv.nel,
                                lx));
            if (hb64) add_scaled_kernel<<<gl, kBlock, 0, st>>>(dl, hb64, 1.0, nloc);
        }
        MG_ALLOC(lv.minv, sizeof(float) * lv.nu);
        diag_recip_kernel<<<vgrid(lv.nu), kBlock, 0, st>>>(lv.minv, dl, lv.gs->uoff, lv.gs->uidx, lv.nu);
        MG_ALLOC(lv.own, nloc);
        owner_kernel<<<gl, kBlock, 0, st>>>(lv.own, lv.gs->lid, lv.gs->uoff, lv.gs->uidx, nloc);
        const size_t vu = sizeof(float) * std::max<int64_t>(lv.nu, 1);
        MG_ALLOC(lv.x, vu);
        MG_ALLOC(lv.r, vu);
        MG_ALLOC(lv.d, vu);
        MG_ALLOC(lv.b, vu);
        MG_ALLOC(lv.wl, sizeof(float) * nloc);
        if (q > 0) MG_ALLOC(lv.bl, sizeof(float) * nloc);
        SEM_LAUNCH_CHECK(ctx);
        if (q == nl - 1) {
            const int64_t m = lv.nu;
            std::vector<double> Ac((size_t)m * m, 0.0);
            if (gal) {
                // assembled from the element matrices: A[i][j] += M_e[a][b] over the
                // element's nodes a, b with plan indices i, j (Dirichlet nodes skipped)
                std::vector<double> Mh((size_t)64 * lv.nel);
                std::vector<int32_t> lidh(nloc);
                MG_TTRY(sem::check_hip(ctx, hipStreamSynchronize(st), "sem_mg_create: hipStreamSynchronize"));
                MG_TTRY(sem::check_hip(ctx, hipMemcpy(Mh.data(), cur64, sizeof(double) * Mh.size(),
                                                      hipMemcpyDeviceToHost), "sem_mg_create: hipMemcpy"));
                MG_TTRY(sem::check_hip(ctx, hipMemcpy(lidh.data(), lv.gs->lid, sizeof(int32_t) * nloc,
                                                      hipMemcpyDeviceToHost), "sem_mg_create: hipMemcpy"));
                for (int64_t e = 0; e < lv.nel; ++e)
                    for (int a = 0; a < 8; ++a) {
                        const int32_t i = lidh[e * 8 + a];
                        if (i < 0) continue;
                        for (int b = 0; b < 8; ++b) {
                            const int32_t j = lidh[e * 8 + b];
                            if (j >= 0) Ac[(size_t)i * m + j] += Mh[e * 64 + a * 8 + b];
                        }
                    }
            } else {
                // the coarsest matrix, column by column, with the float64 operator
                double *ul = nullptr, *wl = nullptr, *cols = nullptr;
                MG_TMP(ul, sizeof(double) * nloc);
                MG_TMP(wl, sizeof(double) * nloc);
                MG_TMP(cols, sizeof(double) * m * m);
                for (int64_t j = 0; j < m; ++j) {
                    unit_local_kernel<<<gl, kBlock, 0, st>>>(ul, lv.gs->lid, j, nloc);
                    MG_TTRY(sem::launch_ax(ctx, sem::AxKind::F64, a64, wl, ul, nullptr, nullptr, nullptr));
                    column_kernel<<<vgrid(m), kBlock, 0, st>>>(cols + j * m, wl, lv.gs->uoff, lv.gs->uidx, m);
                }
                SEM_LAUNCH_CHECK(ctx);
                MG_TTRY(sem::check_hip(ctx, hipStreamSynchronize(st), "sem_mg_create: hipStreamSynchronize"));
                MG_TTRY(sem::check_hip(ctx, hipMemcpy(Ac.data(), cols, sizeof(double) * m * m,
                                                      hipMemcpyDeviceToHost), "sem_mg_create: hipMemcpy"));
            }
            for (int64_t i = 0; i < m; ++i)        // symmetrise (rounding only)
                for (int64_t j = i + 1; j < m; ++j) {
                    const double s = 0.5 * (Ac[i * m + j] + Ac[j * m + i]);
                    Ac[i * m + j] = Ac[j * m + i] = s;
                }
            if (mg->singular) {
                double tr = 0.0;
                for (int64_t i = 0; i < m; ++i) tr += Ac[i * m + i];
                const double c = tr / (double)m / (double)m;
                for (auto& v : Ac) v += c;
            }
            if (!sem::spd_inverse(Ac, (int)m)) {
                free_tmp();
                return bail(sem::fail(ctx, SEM_EBREAKDOWN, "sem_mg_create: coarsest matrix is not positive definite"));
            }
            std::vector<float> Af(Ac.begin(), Ac.end());
            MG_ALLOC(mg->ainv, sizeof(float) * m * m);
            MG_TTRY(sem::check_hip(ctx, hipMemcpy(mg->ainv, Af.data(), sizeof(float) * m * m, hipMemcpyHostToDevice),
                                   "sem_mg_create: hipMemcpy"));
        } else if (galerkin && lxs[q + 1] == 2) {
            // the next level's element matrices (float64), from this level's operator
            const int64_t nel1 = (int64_t)ns[q + 1] * ns[q + 1] * ns[q + 1];
            double* next64 = nullptr;
            {
                hipError_t e = hipMalloc((void**)&next64, sizeof(double) * 64 * nel1);
                if (e != hipSuccess) { free_tmp(); return bail(sem::check_hip(ctx, e, "sem_mg_create: hipMalloc")); }
                carry.v.push_back(next64);
            }
            const double* mine = cur64;            // this level's element matrices (Galerkin level)
            if (!gal) {
                // J^T A_e J column by column: A applied to the 8 coarse basis functions
                // interpolated to this level (the identity for an lx = 2 level), then
                // projected with J^T.  For a p-transfer J is the lx = 2 basis at this
                // level's GLL points; for an h-transfer these are this level's own matrices.
                double *ul = nullptr, *wl = nullptr, *Jd = nullptr, *own64 = nullptr;
                MG_TMP(ul, sizeof(double) * nloc);
                MG_TMP(wl, sizeof(double) * nloc);
                MG_TMP(Jd, sizeof(double) * 2 * lx);
                std::vector<double> xf(lx), Jh(2 * lx);
                sem::gll_host(lx, xf.data(), nullptr, nullptr);
                for (int i = 0; i < lx; ++i) {
                    Jh[i * 2 + 0] = kinds[q] == 0 ? 0.5 * (1.0 - xf[i]) : (i == 0 ? 1.0 : 0.0);
                    Jh[i * 2 + 1] = kinds[q] == 0 ? 0.5 * (1.0 + xf[i]) : (i == 1 ? 1.0 : 0.0);
                }
                MG_TTRY(sem::check_hip(ctx, hipMemcpy(Jd, Jh.data(), sizeof(double) * 2 * lx, hipMemcpyHostToDevice),
                                       "sem_mg_create: hipMemcpy"));
                double* dst = next64;
                if (kinds[q] == 1) {
                    MG_TMP(own64, sizeof(double) * 64 * lv.nel);
                    dst = own64;
                }
                for (int bc = 0; bc < 8; ++bc) {
                    basis_field_kernel<<<gl, kBlock, 0, st>>>(ul, Jd, lx, bc, nloc);
                    MG_TTRY(sem::launch_ax(ctx, sem::AxKind::F64, a64, wl, ul, nullptr, nullptr, nullptr));
                    project_basis_kernel<<<vgrid(8 * lv.nel), kBlock, 0, st>>>(dst, wl, Jd, lx, bc, lv.nel);
                }
                mine = own64;
            }
            if (kinds[q] == 1)
                galerkin_h_kernel<<<vgrid(64 * nel1), kBlock, 0, st>>>(next64, mine, lv.n, ns[q + 1], nel1);
            SEM_LAUNCH_CHECK(ctx);
            cur64 = next64;
        }
        free_tmp();
    }
    // transfer matrices
    for (int q = 0; q + 1 < nl; ++q) {
        MgLevel& lv = mg->L[q];
        const int lf = lv.lx, lc = mg->L[q + 1].lx;
        std::vector<float> J(2 * lf * lc, 0.f);
        if (lv.kind == 0) {
            std::vector<double> xf(lf), xc(lc);
            sem::gll_host(lf, xf.data(), nullptr, nullptr);
            sem::gll_host(lc, xc.data(), nullptr, nullptr);
            lagrange_matrix(xf, xc, J.data());
        } else {
            for (int p = 0; p < 2; ++p)
                for (int i = 0; i < 2; ++i) {
                    const double eta = -1.0 + p + i;
                    J[p * 4 + i * 2 + 0] = (float)(0.5 * (1.0 - eta));
                    J[p * 4 + i * 2 + 1] = (float)(0.5 * (1.0 + eta));
                }
        }
        MG_ALLOC(lv.J, sizeof(float) * J.size());
        MG_TRY(sem::check_hip(ctx, hipMemcpy(lv.J, J.data(), sizeof(float) * J.size(), hipMemcpyHostToDevice),
                              "sem_mg_create: hipMemcpy"));
    }
    // smoothing interval of every level but the coarsest
    for (int q = 0; q + 1 < nl; ++q) {
        MG_TRY(estimate_lmax(mg, mg->L[q], steps, 0x9e3779b9u + 7919u * (uint32_t)q));
        set_chebyshev(mg, mg->L[q]);
    }
    MG_ALLOC(mg->b0, sizeof(float) * mg->L[0].nu);
    MG_ALLOC(mg->x0, sizeof(float) * mg->L[0].nu);
    SEM_LAUNCH_CHECK(ctx);
    SEM_HIP(ctx, hipStreamSynchronize(st));
#undef MG_ALLOC
#undef MG_TRY
#undef MG_TMP
#undef MG_TTRY
    *out = mg;
    return SEM_OK;
}

extern "C" int sem_mg_levels(sem_mg_t mg, int* count) {
    if (!mg || !count) return sem::fail(nullptr, SEM_EINVAL, "sem_mg_levels: null argument");
    *count = (int)mg->L.size();
    return SEM_OK;
}

extern "C" int sem_mg_level_info(sem_mg_t mg, int level, int* n, int* lx, int64_t* n_unique, double* lmax,
                                 double* amp) {
    if (!mg) return sem::fail(nullptr, SEM_EINVAL, "sem_mg_level_info: null handle");
    if (level < 0 || level >= (int)mg->L.size())
        return sem::fail(mg->ctx, SEM_EINVAL, "sem_mg_level_info: level %d outside [0, %d)", level,
                         (int)mg->L.size());
    const MgLevel& lv = mg->L[level];
    if (n) *n = lv.n;
    if (lx) *lx = lv.lx;
    if (n_unique) *n_unique = lv.nu;
    if (lmax) *lmax = lv.lmax;
    if (amp) *amp = lv.amp;
    return SEM_OK;
}

extern "C" int sem_mg_set_lmax(sem_mg_t mg, int level, double lmax) {
    if (!mg) return sem::fail(nullptr, SEM_EINVAL, "sem_mg_set_lmax: null handle");
    if (level < 0 || level + 1 >= (int)mg->L.size() || !(lmax > 0.0))
        return sem::fail(mg->ctx, SEM_EINVAL, "sem_mg_set_lmax: bad level %d or lmax", level);
    mg->L[level].lmax = lmax;
    set_chebyshev(mg, mg->L[level]);
    return SEM_OK;
}

extern "C" int sem_mg_set_graphs(sem_mg_t mg, int on) {
    if (!mg) return sem::fail(nullptr, SEM_EINVAL, "sem_mg_set_graphs: null handle");
    mg->graphs = on != 0;
    return SEM_OK;
}

extern "C" int sem_mg_apply(sem_mg_t mg, void* z, const void* r, sem_dtype_t dtype) {
    if (!mg) return sem::fail(nullptr, SEM_EINVAL, "sem_mg_apply: null handle");
    int rc = sem::enter(mg->ctx);
    if (rc) return rc;
    if (!z || !r) return sem::fail(mg->ctx, SEM_EINVAL, "sem_mg_apply: null vector");
    if (z == r) return sem::fail(mg->ctx, SEM_EINVAL, "sem_mg_apply: z must not alias r");
    if (dtype != SEM_F64 && dtype != SEM_F32) return sem::fail(mg->ctx, SEM_EINVAL, "sem_mg_apply: bad dtype");
    return sem::mg_apply(mg, z, r, dtype == SEM_F64, nullptr);
}
