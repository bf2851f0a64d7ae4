// The element-local stiffness operator w = A_e u (paper Sec. 4.2, Listing 2).
//
// Work decomposition (gfx950, wave64): a workgroup holds EPB elements; each
// element is owned by lx*lx threads (one whole wave at lx = 8), thread (i, j)
// owning the column
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
#include <type_traits>
#include <vector>

#include "sem_internal.h"

namespace {

// Streamed arrays are touched once per application, so they are read and
// written with the nontemporal hint: on gfx950 this keeps them from displacing
// reusable lines and measurably raises the achieved HBM bandwidth.
template <typename T> struct Load;
template <> struct Load<double> {
    __device__ static double get(const double* p, int64_t o) { return __builtin_nontemporal_load(p + o); }
};
template <> struct Load<float> {
    __device__ static float get(const float* p, int64_t o) { return __builtin_nontemporal_load(p + o); }
};
template <> struct Load<uint16_t> {
    __device__ static float get(const uint16_t* p, int64_t o) {
        return __uint_as_float((uint32_t)__builtin_nontemporal_load(p + o) << 16);
    }
};

template <typename T>
__device__ __forceinline__ void store_nt(T* p, int64_t o, T v) { __builtin_nontemporal_store(v, p + o); }

// The same accesses through the caches, for element slices that are not whole
// 128-byte lines: a line shared by two slices (or two elements) is then read
// from HBM once, where the nontemporal form fetched it again for its second
// user.  In float64 the nontemporal form counted 1.43, 1.22 and 1.22 times the
// algorithmic bytes at lx = 5, 6, 7 and 1.08-1.11 at lx = 9, 10, 11; through the
// caches 1.00-1.10.  That made lx = 3, 5, 6, 7 faster (5: 67 -> 51 us at
// 32768 elements) but lx = 9, 10, 11 slower by 1-3 %: there the occupancy, not
// the bytes, bounds the kernel, so they keep the nontemporal form.
template <typename T> struct LoadC;
template <> struct LoadC<double> {
    __device__ static double get(const double* p, int64_t o) { return p[o]; }
};
template <> struct LoadC<float> {
    __device__ static float get(const float* p, int64_t o) { return p[o]; }
};
template <> struct LoadC<uint16_t> {
    __device__ static float get(const uint16_t* p, int64_t o) { return __uint_as_float((uint32_t)p[o] << 16); }
};
template <bool NT, typename T>
__device__ __forceinline__ auto ld(const T* p, int64_t o) {
    if constexpr (NT) return Load<T>::get(p, o);
    else return LoadC<T>::get(p, o);
}
template <bool NT, typename T>
__device__ __forceinline__ void st(T* p, int64_t o, T v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p + o);
    else p[o] = v;
}
// nontemporal streaming when an lx^2 slice of TS is a whole number of lines, or lx >= 9
template <int LX, typename TS>
constexpr bool kStreamNT = (LX * LX * sizeof(TS)) % 128 == 0 || LX >= 9;

// Solver copies of the six factors (float64, float32), slice-blocked in
// pairs: for the slice (e, k) the pairs (g11, g22), (g33, g12), (g13, g23) of
// all lx*lx columns are stored as three consecutive runs of lx*lx two-element
// vectors, so each wave load is one contiguous block (1 KiB in float64 at
// lx = 8).  o is the node's local offset, ij its column.
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec2 __attribute__((ext_vector_type(2)));
template <typename TS> struct Packed;
template <> struct Packed<double> {
    __device__ static void get(const double* gp, int64_t o, int ij, int l2, double* g) {
        const dvec2* q = reinterpret_cast<const dvec2*>(gp) + (o - ij) * 3 + ij;
        const dvec2 a = __builtin_nontemporal_load(q), b = __builtin_nontemporal_load(q + l2),
                    c = __builtin_nontemporal_load(q + 2 * l2);
        g[0] = a.x; g[1] = a.y; g[2] = b.x; g[3] = b.y; g[4] = c.x; g[5] = c.y;
    }
};
template <> struct Packed<float> {
    __device__ static void get(const float* gp, int64_t o, int ij, int l2, float* g) {
        const fvec2* q = reinterpret_cast<const fvec2*>(gp) + (o - ij) * 3 + ij;
        const fvec2 a = __builtin_nontemporal_load(q), b = __builtin_nontemporal_load(q + l2),
                    c = __builtin_nontemporal_load(q + 2 * l2);
        g[0] = a.x; g[1] = a.y; g[2] = b.x; g[3] = b.y; g[4] = c.x; g[5] = c.y;
    }
};
// bfloat16 copies: one 12-byte record per node, (h1 g11, h1 g22, h1 g33,
// h1 g12, h1 g13, h1 g23), h1 folded in when the copy is made; a lane reads its
// node with one 12-byte load and a wave one contiguous block
template <> struct Packed<uint16_t> {
    __device__ static void get(const uint16_t* gp, int64_t o, int, int, float* g) {
        const uint32_t* q = reinterpret_cast<const uint32_t*>(gp) + 3 * o;
        const uint32_t a = __builtin_nontemporal_load(q), b = __builtin_nontemporal_load(q + 1),
                       c = __builtin_nontemporal_load(q + 2);
        g[0] = __uint_as_float(a << 16); g[1] = __uint_as_float(a & 0xffff0000u);
        g[2] = __uint_as_float(b << 16); g[3] = __uint_as_float(b & 0xffff0000u);
        g[4] = __uint_as_float(c << 16); g[5] = __uint_as_float(c & 0xffff0000u);
    }
};

#ifndef SEM_AX_PREFETCH
#define SEM_AX_PREFETCH(LX) ((LX) != 2 && (LX) != 8 && (LX) != 12)
#endif

template <int LX> struct Shape {
    static constexpr bool kWavePrivate = (64 % (LX * LX)) == 0;
    // occupancy floor (waves per SIMD) handed to the register allocator.  At
    // lx = 12 the kernel needs 169 VGPRs, two waves per SIMD; a floor of 3
    // brings it to 168 (two spilled, outside the slice loop) and, with the LDS
    // alias below, four workgroups per CU instead of two: 950 -> 774 us at
    // 32768 elements (without prefetch; with it 11 registers spill and it
    // slows down).  Floors elsewhere spilled inside the loop and lost (lx = 9,
    // 10: 4 waves per SIMD, 331 and 534 against 325 and 433 us).
    static constexpr int kWavesPerEU = LX == 12 ? 3 : 1;
    // fetch the next slice's h1 and G while the current slice is computed
    static constexpr bool kPrefetch = SEM_AX_PREFETCH(LX);
    // elements per workgroup: about four waves, LDS of float64 within ~64 KiB
    static constexpr int EPB = LX == 2 ? 64 : LX == 3 ? 28 : LX == 4 ? 16 : LX == 5 ? 10
                             : LX == 6 ? 7 : LX == 7 ? 5 : LX == 8 ? 4 : LX == 9 ? 3
                             : LX <= 11 ? 2 : 1;
};

// h1 and the six factors at offset o (node ij of a slice) of a live element;
// h = 1 and zero factors for a dead one
template <typename TS, typename TC, bool GATHER, bool NT = true>
__device__ __forceinline__ void load_factors(TC (&g)[6], TC& h, bool live, int64_t o, int ij, int l2,
                                             const TS* __restrict__ h1, const TS* __restrict__ g11,
                                             const TS* __restrict__ g22, const TS* __restrict__ g33,
                                             const TS* __restrict__ g12, const TS* __restrict__ g13,
                                             const TS* __restrict__ g23, const TS* __restrict__ gp) {
    h = 1;
    if (!live) {
#pragma unroll
        for (int a = 0; a < 6; ++a) g[a] = 0;
        return;
    }
    if constexpr (GATHER) {                    // the solver form reads the packed factors
        Packed<TS>::get(gp, o, ij, l2, g);
        if constexpr (std::is_same<TS, uint16_t>::value) return;   // h1 is folded into the record
    } else {
        g[0] = ld<NT>(g11, o); g[1] = ld<NT>(g22, o); g[2] = ld<NT>(g33, o);
        g[3] = ld<NT>(g12, o); g[4] = ld<NT>(g13, o); g[5] = ld<NT>(g23, o);
    }
    if (h1) h = ld<NT>(h1, o);
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Any form returns at once when skip is given and *skip is non-zero (a
// converged solve).  FUSE: the solver form's dot: each workgroup writes sum_L u_L w_L over its
// elements, accumulated in float64, to dot[blockIdx.x] (p^T A p before
// gather-scatter).
// GATHER: u is a unique-node vector, read as u[lid[L]] (lid streamed, u
// through the caches, since neighbouring elements share nodes; lid < 0 marks
// a Dirichlet node, read as 0).  The output stays in the local layout
// (coalesced nontemporal stores); the solver sums the copies of each unique
// node through the plan's CSR lists.
// TPE: threads per element (lx^2, or a power of two above it that divides 64,
// so that every element sits inside one wave; the extra lanes idle)
template <int LX, int EPB, typename TU, typename TS, typename TC, typename TW, bool FUSE, bool GATHER, bool HB,
          bool PF = Shape<LX>::kPrefetch, int TPE = LX * LX>
__global__ void __launch_bounds__(EPB * TPE) __attribute__((amdgpu_waves_per_eu(Shape<LX>::kWavesPerEU, 8)))
ax_kernel(TW* __restrict__ w, const TU* __restrict__ u,
          const TC* __restrict__ dx, const TC* __restrict__ dy, const TC* __restrict__ dz,
          const TC* __restrict__ dxt, const TC* __restrict__ dyt, const TC* __restrict__ dzt,
          const TS* __restrict__ h1, const TS* __restrict__ g11, const TS* __restrict__ g22,
          const TS* __restrict__ g33, const TS* __restrict__ g12, const TS* __restrict__ g13,
          const TS* __restrict__ g23, int64_t nel, const int* __restrict__ skip,
          double* __restrict__ dot, const int32_t* __restrict__ lid,
          const TS* __restrict__ gp, const TS* __restrict__ hb) {
    constexpr int L2 = LX * LX;
    constexpr int L3 = L2 * LX;
    constexpr bool WP = (64 % TPE) == 0;
    static_assert(TPE >= L2, "threads per element");
    constexpr bool NT = GATHER || kStreamNT<LX, TS>;
    if (skip && *skip) return;
    __shared__ TC s_u[EPB * L3];               // the element's u (wave-private: then the r-flux)
    __shared__ TC s_s[EPB * L3];               // s-flux
    // Elements spanning waves write the r-flux of slice k over slice k of u
    // after a workgroup barrier (every wave has read it) instead of into a third
    // array, where the LDS this frees admits one more workgroup per CU
    // (lx = 7: 3 -> 4, lx = 9 and 11: 2 -> 3, 4-5 % faster at lx 9 and 11;
    // lx = 12 with its register floor: 3 -> 4).  At the other lx the
    // registers, not the LDS, cap the workgroups, and the barrier per slice
    // would cost without a gain.
    constexpr bool ALIAS = !WP && (LX == 7 || LX == 9 || LX == 11 || LX == 12);
    __shared__ TC s_r0[(WP || ALIAS) ? 1 : EPB * L3];     // r-flux when elements span waves
    __shared__ TC s_d[6 * L2];                 // dx, dy, dz, dxt, dyt, dzt

    const int tid = threadIdx.x;
    const int el = tid / TPE;
    const int ijr = tid - el * TPE;
    const bool act = TPE == L2 || ijr < L2;    // a lane with a column
    const int ij = act ? ijr : 0;
    const int i = ij % LX;
    const int j = ij / LX;
    const int64_t e = (int64_t)blockIdx.x * EPB + el;
    const bool live = act && e < nel;
    const int64_t base = e * L3 + ij;
    TC* su = s_u + el * L3;
    TC* ss = s_s + el * L3;
    TC* sr = (WP || ALIAS) ? su : s_r0 + el * L3;
    const TC* sdz = s_d + 2 * L2;
    const TC* sdzt = s_d + 5 * L2;

    for (int q = tid; q < L2; q += EPB * TPE) {
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
        if constexpr (GATHER) {
            const int32_t q = live ? __builtin_nontemporal_load(lid + base + k * L2) : -1;
            uc[k] = q >= 0 ? (TC)u[q] : TC(0);
        }
        else
            uc[k] = live ? (TC)ld<NT>(u, base + k * L2) : TC(0);
    }
    if (act) {
#pragma unroll
        for (int k = 0; k < LX; ++k) su[k * L2 + ij] = uc[k];
    }
    __syncthreads();   // s_d is shared by every wave of the workgroup

    // The float64 solver form at lx = 8 reads the j-direction rows of D from LDS
    // instead of keeping them in registers: 138 -> 122 VGPRs, four waves per
    // SIMD instead of three, and the float64 PCG iteration 436 -> 418 us at 32^3.
    // The public form measured the same either way (188.1 us) and the float32
    // and bfloat16 forms, already at 64-78 VGPRs, slower, so they keep them.
    constexpr bool DJL = LX == 8 && GATHER && std::is_same<TC, double>::value;
    TC di[LX], dj[DJL ? 1 : LX];
    const TC* sdj = s_d + L2;
#pragma unroll
    for (int l = 0; l < LX; ++l) {
        di[l] = s_d[l * LX + i];
        if constexpr (!DJL) dj[l] = s_d[L2 + l * LX + j];
    }

    // forward passes slice by slice; the t-flux of slice k is folded straight
    // into the transposed t-sum: wt[m] += dzt[k, m] * vt_k
    TC wt[LX];
#pragma unroll
    for (int m = 0; m < LX; ++m) wt[m] = 0;
    TC ng[6], nh;                              // the next slice's factors (prefetch)
    if constexpr (PF) load_factors<TS, TC, GATHER, NT>(ng, nh, live, base, ij, L2, h1, g11, g22, g33, g12, g13, g23, gp);
#pragma unroll 1
    for (int k = 0; k < LX; ++k) {
        const int64_t o = base + k * L2;
        TC g[6], H;
        if constexpr (PF) {
#pragma unroll
            for (int a = 0; a < 6; ++a) g[a] = ng[a];
            H = nh;
            if (k + 1 < LX)
                load_factors<TS, TC, GATHER, NT>(ng, nh, live, o + L2, ij, L2, h1, g11, g22, g33, g12, g13, g23, gp);
        } else {
            load_factors<TS, TC, GATHER, NT>(g, H, live, o, ij, L2, h1, g11, g22, g33, g12, g13, g23, gp);
        }
        TC r = 0, s = 0, t = 0;
#pragma unroll
        for (int l = 0; l < LX; ++l) {
            r += di[l] * su[k * L2 + j * LX + l];
            s += (DJL ? sdj[l * LX + j] : dj[DJL ? 0 : l]) * su[k * L2 + l * LX + i];
            t += sdz[l * LX + k] * uc[l];
        }
        const TC G11 = g[0], G22 = g[1], G33 = g[2], G12 = g[3], G13 = g[4], G23 = g[5];
        const TC vr = H * (G11 * r + G12 * s + G13 * t);
        const TC vs = H * (G12 * r + G22 * s + G23 * t);
        const TC vt = H * (G13 * r + G23 * s + G33 * t);
        if (WP) wave_sync();   // every lane has read slice k before it is overwritten
        else if (ALIAS) __syncthreads();
        if (act) {
            sr[k * L2 + ij] = vr;
            ss[k * L2 + ij] = vs;
        }
#pragma unroll
        for (int m = 0; m < LX; ++m) wt[m] += sdzt[k * LX + m] * vt;
    }
    if (WP) wave_sync(); else __syncthreads();

#pragma unroll
    for (int l = 0; l < LX; ++l) {
        di[l] = s_d[3 * L2 + l * LX + i];
        if constexpr (!DJL) dj[l] = s_d[4 * L2 + l * LX + j];
    }
    double pw = 0.0;
#pragma unroll
    for (int k = 0; k < LX; ++k) {
        TC acc = wt[k];
#pragma unroll
        for (int l = 0; l < LX; ++l) {
            acc += di[l] * sr[k * L2 + j * LX + l];
            acc += (DJL ? s_d[4 * L2 + l * LX + j] : dj[DJL ? 0 : l]) * ss[k * L2 + l * LX + i];
        }
        if (live) {
            if constexpr (HB) acc += ld<NT>(hb, base + k * L2) * uc[k];   // Helmholtz: + h2 B u
            st<NT>(w, base + k * L2, (TW)acc);
        }
        if (FUSE) pw += (double)uc[k] * (double)(TW)acc;
    }
    if (FUSE) {
        constexpr int NT = EPB * TPE;
        if constexpr (NT % 64 == 0) {          // whole waves: shuffle, then one value per wave
            __shared__ double s_red[NT / 64];
            pw = sem::wave_sum(pw);
            if ((tid & 63) == 0) s_red[tid >> 6] = pw;
            __syncthreads();
            if (tid == 0) {
                double t = 0.0;
                for (int q = 0; q < NT / 64; ++q) t += s_red[q];
                dot[blockIdx.x] = t;
            }
        } else {                               // partial last wave: LDS tree
            __shared__ double s_red[NT];
            s_red[tid] = pw;
            __syncthreads();
            constexpr int P2 = NT <= 128 ? 64 : NT <= 256 ? 128 : 256;
            for (int st = P2; st > 0; st >>= 1) {
                if (tid < st && tid + st < NT) s_red[tid] += s_red[tid + st];
                __syncthreads();
            }
            if (tid == 0) dot[blockIdx.x] = s_red[0];
        }
    }
}

// Slice-pipelined column mapping: one thread per (i, j) column as in
// ax_kernel, but the element passes through LDS one k-slice at a time.  Slice
// k of u and the r- and s-fluxes of slice k - 1 sit in double buffers, so each
// slice costs one workgroup barrier, and LDS holds 6 lx^2 values per element
// instead of ax_kernel's 2-3 lx^3: large elements keep several times more
// waves in flight.  Register arrays are indexed by the run-time slice only
// through selects, so they stay in registers.  Plain (public) form only.
template <int LX> struct ShapeSlice {
    static constexpr int EPB = (512 / (LX * LX)) < 1 ? 1 : 512 / (LX * LX);
};

template <int LX, int EPB, typename TS, typename TC, typename TW, bool HB>
__global__ void __launch_bounds__(EPB * LX * LX)
ax_slice_kernel(TW* __restrict__ w, const TS* __restrict__ u,
                const TC* __restrict__ dx, const TC* __restrict__ dy, const TC* __restrict__ dz,
                const TC* __restrict__ dxt, const TC* __restrict__ dyt, const TC* __restrict__ dzt,
                const TS* __restrict__ h1, const TS* __restrict__ g11, const TS* __restrict__ g22,
                const TS* __restrict__ g33, const TS* __restrict__ g12, const TS* __restrict__ g13,
                const TS* __restrict__ g23, int64_t nel, const TS* __restrict__ hb) {
    constexpr int L2 = LX * LX;
    constexpr int L3 = L2 * LX;
    constexpr int NS = EPB * L2;
    constexpr bool NT = kStreamNT<LX, TS>;
    __shared__ TC s_d[6 * L2];
    __shared__ TC s_u[2][NS];
    __shared__ TC s_r[2][NS];
    __shared__ TC s_s[2][NS];
    const int tid = threadIdx.x;
    const int el = tid / L2;
    const int ij = tid - el * L2;
    const int i = ij % LX;
    const int j = ij / LX;
    const int64_t e = (int64_t)blockIdx.x * EPB + el;
    const bool live = e < nel;
    const int64_t base = e * L3 + ij;
    const int off = el * L2;
    for (int q = tid; q < L2; q += NS) {
        s_d[q] = dx[q];
        s_d[L2 + q] = dy[q];
        s_d[2 * L2 + q] = dz[q];
        s_d[3 * L2 + q] = dxt[q];
        s_d[4 * L2 + q] = dyt[q];
        s_d[5 * L2 + q] = dzt[q];
    }
    TC uc[LX];
#pragma unroll
    for (int k = 0; k < LX; ++k) uc[k] = live ? (TC)ld<NT>(u, base + k * L2) : TC(0);
    s_u[0][off + ij] = uc[0];
    __syncthreads();
    TC di[LX], dj[LX], ti[LX], tj[LX];
#pragma unroll
    for (int l = 0; l < LX; ++l) {
        di[l] = s_d[l * LX + i];
        dj[l] = s_d[L2 + l * LX + j];
        ti[l] = s_d[3 * L2 + l * LX + i];
        tj[l] = s_d[4 * L2 + l * LX + j];
    }
    const TC* sdz = s_d + 2 * L2;
    const TC* sdzt = s_d + 5 * L2;
    TC wt[LX];
#pragma unroll
    for (int m = 0; m < LX; ++m) wt[m] = 0;
    // iteration k: the forward passes of slice k (k < LX) and the transposed
    // r- and s-sums of slice k - 1 (k > 0)
#pragma unroll 1
    for (int k = 0; k <= LX; ++k) {
        if (k > 0) __syncthreads();
        const int b = k & 1;
        TC vr = 0, vs = 0;
        if (k < LX) {
            TC g[6], H;
            load_factors<TS, TC, false, NT>(g, H, live, base + k * L2, ij, L2, h1, g11, g22, g33, g12, g13, g23,
                                            nullptr);
            TC r = 0, s = 0, t = 0;
#pragma unroll
            for (int l = 0; l < LX; ++l) {
                r += di[l] * s_u[b][off + j * LX + l];
                s += dj[l] * s_u[b][off + l * LX + i];
                t += sdz[l * LX + k] * uc[l];
            }
            vr = H * (g[0] * r + g[3] * s + g[4] * t);
            vs = H * (g[3] * r + g[1] * s + g[5] * t);
            const TC vt = H * (g[4] * r + g[5] * s + g[2] * t);
#pragma unroll
            for (int m = 0; m < LX; ++m) wt[m] += sdzt[k * LX + m] * vt;
        }
        if (k > 0) {
            const int pb = b ^ 1;
            TC acc = 0;
#pragma unroll
            for (int l = 0; l < LX; ++l) {
                acc += ti[l] * s_r[pb][off + j * LX + l];
                acc += tj[l] * s_s[pb][off + l * LX + i];
            }
#pragma unroll
            for (int m = 0; m < LX; ++m) wt[m] += (m == k - 1) ? acc : TC(0);
        }
        if (k < LX) {
            s_r[b][off + ij] = vr;
            s_s[b][off + ij] = vs;
            TC nx = 0;
#pragma unroll
            for (int m = 1; m < LX; ++m) nx = (m == k + 1) ? uc[m] : nx;
            if (k + 1 < LX) s_u[b ^ 1][off + ij] = nx;
        }
    }
    if (live) {
#pragma unroll
        for (int k = 0; k < LX; ++k) {
            TC acc = wt[k];
            if constexpr (HB) acc += ld<NT>(hb, base + k * L2) * uc[k];   // Helmholtz: + h2 B u
            st<NT>(w, base + k * L2, (TW)acc);
        }
    }
}

// One thread per node ("3D" mapping): every load and store of the streamed
// arrays is contiguous across the workgroup.  u and the three fluxes go
// through LDS; each thread keeps the derivative-matrix rows it needs (its i,
// j, k) in registers.  One of the variants the run-time tuning times; with
// the cached streaming of the column mapping it is the slower one at every lx
// measured (lx = 3: 18.1 against 13.9 us at 32768 elements).
template <int LX> struct Shape3D {
    // whole elements per workgroup of at most 1024 threads (none above lx = 10)
    static constexpr int EPB = LX == 3 ? 16 : (1024 / (LX * LX * LX));
};

template <int LX, int EPB, typename TS, typename TC, typename TW, bool HB>
__global__ void __launch_bounds__(EPB * LX * LX * LX)
ax3d_kernel(TW* __restrict__ w, const TS* __restrict__ u,
            const TC* __restrict__ dx, const TC* __restrict__ dy, const TC* __restrict__ dz,
            const TC* __restrict__ dxt, const TC* __restrict__ dyt, const TC* __restrict__ dzt,
            const TS* __restrict__ h1, const TS* __restrict__ g11, const TS* __restrict__ g22,
            const TS* __restrict__ g33, const TS* __restrict__ g12, const TS* __restrict__ g13,
            const TS* __restrict__ g23, int64_t nel, const TS* __restrict__ hb) {
    constexpr int L2 = LX * LX;
    constexpr int L3 = L2 * LX;
    __shared__ TC s_u[EPB * L3];
    __shared__ TC s_r[EPB * L3];
    __shared__ TC s_s[EPB * L3];
    __shared__ TC s_t[EPB * L3];
    const int tid = threadIdx.x;
    const int el = tid / L3;
    const int p = tid - el * L3;
    const int i = p % LX, j = (p / LX) % LX, k = p / L2;
    const int64_t e = (int64_t)blockIdx.x * EPB + el;
    const bool live = e < nel;
    const int64_t g = e * L3 + p;               // contiguous across the workgroup
    TC* su = s_u + el * L3;
    TC* sr = s_r + el * L3;
    TC* ss = s_s + el * L3;
    TC* st = s_t + el * L3;
    TC uv = 0, G11 = 0, G22 = 0, G33 = 0, G12 = 0, G13 = 0, G23 = 0, H = 1;
    if (live) {
        uv = Load<TS>::get(u, g);
        G11 = Load<TS>::get(g11, g); G22 = Load<TS>::get(g22, g); G33 = Load<TS>::get(g33, g);
        G12 = Load<TS>::get(g12, g); G13 = Load<TS>::get(g13, g); G23 = Load<TS>::get(g23, g);
        if (h1) H = Load<TS>::get(h1, g);
    }
    su[p] = uv;
    TC di[LX], dj[LX], dk[LX];
#pragma unroll
    for (int l = 0; l < LX; ++l) {
        di[l] = dx[l * LX + i];
        dj[l] = dy[l * LX + j];
        dk[l] = dz[l * LX + k];
    }
    __syncthreads();
    TC r = 0, s = 0, t = 0;
#pragma unroll
    for (int l = 0; l < LX; ++l) {
        r += di[l] * su[k * L2 + j * LX + l];
        s += dj[l] * su[k * L2 + l * LX + i];
        t += dk[l] * su[l * L2 + j * LX + i];
    }
    sr[p] = H * (G11 * r + G12 * s + G13 * t);
    ss[p] = H * (G12 * r + G22 * s + G23 * t);
    st[p] = H * (G13 * r + G23 * s + G33 * t);
#pragma unroll
    for (int l = 0; l < LX; ++l) {
        di[l] = dxt[l * LX + i];
        dj[l] = dyt[l * LX + j];
        dk[l] = dzt[l * LX + k];
    }
    __syncthreads();
    TC acc = 0;
#pragma unroll
    for (int l = 0; l < LX; ++l) {
        acc += di[l] * sr[k * L2 + j * LX + l];
        acc += dj[l] * ss[k * L2 + l * LX + i];
        acc += dk[l] * st[l * L2 + j * LX + i];
    }
    if constexpr (HB) if (live) acc += Load<TS>::get(hb, g) * uv;   // Helmholtz: + h2 B u
    if (live) store_nt(w, g, (TW)acc);
}

// The Helmholtz term is a template flag (HB), so that the two forms are
// separate kernels (and separate rows of a kernel trace).
// the float64 public form's kernel variants (SEM_AX_* of sem.h)
constexpr bool variant_exists(int lx, int v) {
    return v == SEM_AX_COLUMN || v == SEM_AX_COLUMN_PF || v == SEM_AX_SLICE || (v == SEM_AX_3D && lx <= 10) ||
           (v == SEM_AX_WAVE && (lx == 3 || lx == 5 || lx == 6 || lx == 7));
}

template <int LX, typename TS, typename TC, typename TW, bool HB, bool PF>
void launch_column(sem_ctx_t ctx, void* w, const void* u, const void* const* D, const void* h1,
                   const void* const* G, int64_t nel, const void* hb) {
    constexpr int EPB = Shape<LX>::EPB;
    ax_kernel<LX, EPB, TS, TS, TC, TW, false, false, HB, PF><<<(unsigned)((nel + EPB - 1) / EPB), EPB * LX * LX, 0,
                                                               ctx->stream>>>(
        (TW*)w, (const TS*)u, (const TC*)D[0], (const TC*)D[1], (const TC*)D[2], (const TC*)D[3], (const TC*)D[4],
        (const TC*)D[5], (const TS*)h1, (const TS*)G[0], (const TS*)G[1], (const TS*)G[2], (const TS*)G[3],
        (const TS*)G[4], (const TS*)G[5], nel, nullptr, nullptr, nullptr, nullptr, (const TS*)hb);
}

template <int LX, typename TS, typename TC, typename TW, bool HB>
void launch_3d(sem_ctx_t ctx, void* w, const void* u, const void* const* D, const void* h1,
               const void* const* G, int64_t nel, const void* hb) {
    if constexpr (Shape3D<LX>::EPB >= 1) {
        constexpr int E3 = Shape3D<LX>::EPB;
        ax3d_kernel<LX, E3, TS, TC, TW, HB><<<(unsigned)((nel + E3 - 1) / E3), E3 * LX * LX * LX, 0, ctx->stream>>>(
            (TW*)w, (const TS*)u, (const TC*)D[0], (const TC*)D[1], (const TC*)D[2], (const TC*)D[3],
            (const TC*)D[4], (const TC*)D[5], (const TS*)h1, (const TS*)G[0], (const TS*)G[1],
            (const TS*)G[2], (const TS*)G[3], (const TS*)G[4], (const TS*)G[5], nel, (const TS*)hb);
    }
}

// a non-default variant of the float64 public form; false if it does not exist
template <int LX, typename TS, typename TC, typename TW, bool HB>
bool launch_variant(sem_ctx_t ctx, int variant, void* w, const void* u, const void* const* D, const void* h1,
                    const void* const* G, int64_t nel, const void* hb) {
    if constexpr (!std::is_same<TS, double>::value) {
        return false;
    } else {
        if (variant == SEM_AX_COLUMN_PF) {
            launch_column<LX, TS, TC, TW, HB, !Shape<LX>::kPrefetch>(ctx, w, u, D, h1, G, nel, hb);
            return true;
        }
        if (variant == SEM_AX_COLUMN) {
            launch_column<LX, TS, TC, TW, HB, Shape<LX>::kPrefetch>(ctx, w, u, D, h1, G, nel, hb);
            return true;
        }
        if (variant == SEM_AX_SLICE) {
            constexpr int ES = ShapeSlice<LX>::EPB;
            ax_slice_kernel<LX, ES, TS, TC, TW, HB><<<(unsigned)((nel + ES - 1) / ES), ES * LX * LX, 0, ctx->stream>>>(
                (TW*)w, (const TS*)u, (const TC*)D[0], (const TC*)D[1], (const TC*)D[2], (const TC*)D[3],
                (const TC*)D[4], (const TC*)D[5], (const TS*)h1, (const TS*)G[0], (const TS*)G[1],
                (const TS*)G[2], (const TS*)G[3], (const TS*)G[4], (const TS*)G[5], nel, (const TS*)hb);
            return true;
        }
        if constexpr (LX == 3 || LX == 5 || LX == 6 || LX == 7) {
            if (variant == SEM_AX_WAVE) {      // lx^2 columns padded to 16, 32 or 64 lanes
                constexpr int TPE = LX == 3 ? 16 : LX == 5 ? 32 : 64;
                constexpr int EW = 256 / TPE;
                ax_kernel<LX, EW, TS, TS, TC, TW, false, false, HB, Shape<LX>::kPrefetch, TPE>
                    <<<(unsigned)((nel + EW - 1) / EW), EW * TPE, 0, ctx->stream>>>(
                        (TW*)w, (const TS*)u, (const TC*)D[0], (const TC*)D[1], (const TC*)D[2], (const TC*)D[3],
                        (const TC*)D[4], (const TC*)D[5], (const TS*)h1, (const TS*)G[0], (const TS*)G[1],
                        (const TS*)G[2], (const TS*)G[3], (const TS*)G[4], (const TS*)G[5], nel, nullptr, nullptr,
                        nullptr, nullptr, (const TS*)hb);
                return true;
            }
        }
        if (variant == SEM_AX_3D && LX != 3 && LX <= 10) {
            launch_3d<LX, TS, TC, TW, HB>(ctx, w, u, D, h1, G, nel, hb);
            return true;
        }
        return false;
    }
}

template <int LX, typename TU, typename TS, typename TC, typename TW, bool HB>
int launch_form(sem_ctx_t ctx, void* w, const void* u, const void* const* D, const void* h1,
                const void* const* G, int64_t nel, const int* skip, double* dot, const int32_t* lid,
                const void* gp, const void* hb, int variant) {
    constexpr int EPB = Shape<LX>::EPB;
    const int64_t blocks = (nel + EPB - 1) / EPB;
    if (blocks > 0x7fffffff) return sem::fail(ctx, SEM_EINVAL, "sem_ax: nel too large");
    if (!lid && !dot && variant >= 0 &&
        launch_variant<LX, TS, TC, TW, HB>(ctx, variant, w, u, D, h1, G, nel, hb)) {
        SEM_LAUNCH_CHECK(ctx);
        return SEM_OK;
    }
#define SEM_AX_ARGS (TW*)w, (const TU*)u, (const TC*)D[0], (const TC*)D[1], (const TC*)D[2], \
        (const TC*)D[3], (const TC*)D[4], (const TC*)D[5], (const TS*)h1, (const TS*)G[0],  \
        (const TS*)G[1], (const TS*)G[2], (const TS*)G[3], (const TS*)G[4], (const TS*)G[5], \
        nel, skip, dot, lid, (const TS*)gp, (const TS*)hb
    const dim3 grid((unsigned)blocks), block(EPB * LX * LX);
    if (lid && !gp) return sem::fail(ctx, SEM_EINVAL, "launch_ax: the solver form needs packed factors");
    if (dot && lid)
        ax_kernel<LX, EPB, TU, TS, TC, TW, true, true, HB><<<grid, block, 0, ctx->stream>>>(SEM_AX_ARGS);
    else if (lid)
        ax_kernel<LX, EPB, TU, TS, TC, TW, false, true, HB><<<grid, block, 0, ctx->stream>>>(SEM_AX_ARGS);
    else if (!dot)
        ax_kernel<LX, EPB, TU, TS, TC, TW, false, false, HB><<<grid, block, 0, ctx->stream>>>(SEM_AX_ARGS);
    else
        return sem::fail(ctx, SEM_EINVAL, "launch_ax: the fused dot needs the solver form");
#undef SEM_AX_ARGS
    SEM_LAUNCH_CHECK(ctx);
    return SEM_OK;
}

template <int LX, typename TU, typename TS, typename TC, typename TW>
int launch_lx(sem_ctx_t ctx, void* w, const void* u, const void* const* D, const void* h1,
              const void* const* G, int64_t nel, const int* skip, double* dot, const int32_t* lid,
              const void* gp, const void* hb, int variant) {
    if (hb) return launch_form<LX, TU, TS, TC, TW, true>(ctx, w, u, D, h1, G, nel, skip, dot, lid, gp, hb, variant);
    return launch_form<LX, TU, TS, TC, TW, false>(ctx, w, u, D, h1, G, nel, skip, dot, lid, gp, hb, variant);
}

template <typename TU, typename TS, typename TC, typename TW>
int dispatch(sem_ctx_t ctx, int lx, void* w, const void* u, const void* const* D,
             const void* h1, const void* const* G, int64_t nel, const int* skip, double* dot,
             const int32_t* lid = nullptr, const void* gp = nullptr,
             const void* hb = nullptr, int variant = SEM_AX_DEFAULT) {
    switch (lx) {
#define SEM_AX_CASE(L) case L: return launch_lx<L, TU, TS, TC, TW>(ctx, w, u, D, h1, G, nel, skip, dot, lid, gp, hb, variant);
        SEM_AX_CASE(2) SEM_AX_CASE(3) SEM_AX_CASE(4) SEM_AX_CASE(5) SEM_AX_CASE(6) SEM_AX_CASE(7)
        SEM_AX_CASE(8) SEM_AX_CASE(9) SEM_AX_CASE(10) SEM_AX_CASE(11) SEM_AX_CASE(12)
#undef SEM_AX_CASE
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

namespace {

int ax_public(sem_ctx_t ctx, void* w, const void* u, const void* dx, const void* dy, const void* dz,
              const void* dxt, const void* dyt, const void* dzt, const void* h1, const void* g11,
              const void* g22, const void* g33, const void* g12, const void* g13, const void* g23,
              const void* hb, int64_t nel, int lx, sem_dtype_t field_dtype, sem_dtype_t out_dtype) {
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
    bool alias = overlaps(w, nw, u, nf) || overlaps(w, nw, h1, nf) || overlaps(w, nw, hb, nf);
    for (int q = 0; q < 6; ++q) alias = alias || overlaps(w, nw, G[q], nf) || overlaps(w, nw, D[q], nd);
    if (alias) return sem::fail(ctx, SEM_EINVAL, "sem_ax: output overlaps an input");
    if (f64)
        return dispatch<double, double, double, double>(ctx, lx, w, u, D, h1, G, nel, nullptr, nullptr, nullptr,
                                                        nullptr, hb, ctx->ax_variant[lx]);
    if (field_dtype == SEM_F32)
        return dispatch<float, float, float, float>(ctx, lx, w, u, D, h1, G, nel, nullptr, nullptr, nullptr,
                                                    nullptr, hb);
    return dispatch<uint16_t, uint16_t, float, float>(ctx, lx, w, u, D, h1, G, nel, nullptr, nullptr, nullptr,
                                                      nullptr, hb);
}

}  // namespace

extern "C" int sem_ax(sem_ctx_t ctx, void* w, const void* u, const void* dx, const void* dy,
                      const void* dz, const void* dxt, const void* dyt, const void* dzt,
                      const void* h1, const void* g11, const void* g22, const void* g33,
                      const void* g12, const void* g13, const void* g23, int64_t nel, int lx,
                      sem_dtype_t field_dtype, sem_dtype_t out_dtype) {
    return ax_public(ctx, w, u, dx, dy, dz, dxt, dyt, dzt, h1, g11, g22, g33, g12, g13, g23, nullptr, nel, lx,
                     field_dtype, out_dtype);
}

extern "C" int sem_ax_helmholtz(sem_ctx_t ctx, void* w, const void* u, const void* dx, const void* dy,
                                const void* dz, const void* dxt, const void* dyt, const void* dzt,
                                const void* h1, const void* g11, const void* g22, const void* g33,
                                const void* g12, const void* g13, const void* g23, const void* h2b,
                                int64_t nel, int lx, sem_dtype_t field_dtype, sem_dtype_t out_dtype) {
    if (!h2b && nel > 0) return sem::fail(ctx, SEM_EINVAL, "sem_ax_helmholtz: null h2b");
    return ax_public(ctx, w, u, dx, dy, dz, dxt, dyt, dzt, h1, g11, g22, g33, g12, g13, g23, h2b, nel, lx,
                     field_dtype, out_dtype);
}

namespace sem {

int ax_blocks(int lx, int64_t nel) {
    int epb = 1;
    switch (lx) {
#define SEM_AX_EPB(L) case L: epb = Shape<L>::EPB; break;
        SEM_AX_EPB(2) SEM_AX_EPB(3) SEM_AX_EPB(4) SEM_AX_EPB(5) SEM_AX_EPB(6) SEM_AX_EPB(7)
        SEM_AX_EPB(8) SEM_AX_EPB(9) SEM_AX_EPB(10) SEM_AX_EPB(11) SEM_AX_EPB(12)
#undef SEM_AX_EPB
        default: break;
    }
    return (int)((nel + epb - 1) / epb);
}

int launch_ax(sem_ctx_t ctx, AxKind kind, const AxArgs& a, void* w, const void* u,
              const int* skip, double* dot, const int32_t* lid) {
    const void* D[6] = {a.D[0], a.D[1], a.D[2], a.D[3], a.D[4], a.D[5]};
    const void* G[6] = {a.G[0], a.G[1], a.G[2], a.G[3], a.G[4], a.G[5]};
    switch (kind) {
        case AxKind::F64:
            return dispatch<double, double, double, double>(ctx, a.lx, w, u, D, a.h1, G, a.nel, skip, dot, lid,
                                                            a.Gp, a.hb);
        case AxKind::F32:
            return dispatch<float, float, float, float>(ctx, a.lx, w, u, D, a.h1, G, a.nel, skip, dot, lid,
                                                        a.Gp, a.hb);
        case AxKind::F32_BF16:
            return dispatch<float, uint16_t, float, float>(ctx, a.lx, w, u, D, a.h1, G, a.nel, skip, dot, lid,
                                                           a.Gp, a.hb);
    }
    return fail(ctx, SEM_EINVAL, "launch_ax: bad kind");
}

}  // namespace sem

// ------------------------------------------------------------ variant choice
namespace {

// synthetic inputs for timing: a hash of the index mapped to [-1, 1) for u,
// positive-definite factors (diagonal 1 + |.|/2, off-diagonal ./10), h1 = 1
__global__ void tune_fill_kernel(double* __restrict__ u, double* __restrict__ g11, double* __restrict__ g22,
                                 double* __restrict__ g33, double* __restrict__ g12, double* __restrict__ g13,
                                 double* __restrict__ g23, double* __restrict__ h1, int64_t n) {
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n; L += (int64_t)gridDim.x * blockDim.x) {
        uint32_t h = (uint32_t)L * 2654435761u;
        h ^= h >> 16; h *= 0x7feb352du; h ^= h >> 15;
        const double v = (double)h * (2.0 / 4294967296.0) - 1.0;
        u[L] = v;
        g11[L] = 1.0 + 0.5 * fabs(v); g22[L] = 1.0 + 0.25 * fabs(v); g33[L] = 1.0 + 0.125 * fabs(v);
        g12[L] = 0.1 * v; g13[L] = -0.1 * v; g23[L] = 0.05 * v;
        h1[L] = 1.0;
    }
}

}  // namespace

extern "C" int sem_ax_set_variant(sem_ctx_t ctx, int lx, int variant) {
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (!sem::lx_ok(lx)) return sem::fail(ctx, SEM_EUNSUPPORTED_LX, "sem_ax_set_variant: lx=%d", lx);
    if (variant != SEM_AX_DEFAULT && !variant_exists(lx, variant))
        return sem::fail(ctx, SEM_EINVAL, "sem_ax_set_variant: variant %d does not exist at lx=%d", variant, lx);
    ctx->ax_variant[lx] = variant;
    return SEM_OK;
}

extern "C" int sem_ax_get_variant(sem_ctx_t ctx, int lx, int* variant) {
    if (!ctx) return sem::fail(nullptr, SEM_EINVAL, "null context");
    if (!sem::lx_ok(lx)) return sem::fail(ctx, SEM_EUNSUPPORTED_LX, "sem_ax_get_variant: lx=%d", lx);
    if (!variant) return sem::fail(ctx, SEM_EINVAL, "sem_ax_get_variant: null output");
    *variant = ctx->ax_variant[lx];
    return SEM_OK;
}

namespace {

// every float64 variant that exists at lx timed on the given operands (`reps`
// launches after two warm-ups, HIP events on the context's stream) in two
// rounds, keeping each variant's faster round: the clocks of a GPU that was
// idle rise during the first launches, which would otherwise penalise the
// variant timed first.  The fastest is selected on the context.
int time_variants(sem_ctx_t ctx, int lx, void* w, const void* u, const void* const* D, const void* h1,
                  const void* const* G, int64_t nel, int reps, double* us, int* best) {
    hipStream_t st = ctx->stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    SEM_HIP(ctx, hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) { (void)hipEventDestroy(e0); return sem::check_hip(ctx, he, "hipEventCreate"); }
    double t_best[SEM_AX_VARIANTS];
    for (int v = 0; v < SEM_AX_VARIANTS; ++v) t_best[v] = -1.0;
    int rc = SEM_OK;
    for (int round = 0; round < 2 && rc == SEM_OK; ++round)
        for (int v = 0; v < SEM_AX_VARIANTS && rc == SEM_OK; ++v) {
            if (!variant_exists(lx, v)) continue;
            for (int q = 0; q < 2 + reps && rc == SEM_OK; ++q) {
                if (q == 2) (void)hipEventRecord(e0, st);
                rc = dispatch<double, double, double, double>(ctx, lx, w, u, D, h1, G, nel, nullptr, nullptr,
                                                              nullptr, nullptr, nullptr, v);
            }
            if (rc) break;
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            const double t = 1e3 * ms / reps;
            if (t_best[v] < 0.0 || t < t_best[v]) t_best[v] = t;
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    int best_v = SEM_AX_COLUMN;
    for (int v = 0; v < SEM_AX_VARIANTS; ++v) {
        if (us) us[v] = t_best[v];
        if (t_best[v] >= 0.0 && (t_best[best_v] < 0.0 || t_best[v] < t_best[best_v])) best_v = v;
    }
    ctx->ax_variant[lx] = best_v;
    *best = best_v;
    return SEM_OK;
}

}  // namespace

extern "C" int sem_ax_tune(sem_ctx_t ctx, int lx, int64_t nel, int reps, double* us, int* best) {
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (!sem::lx_ok(lx)) return sem::fail(ctx, SEM_EUNSUPPORTED_LX, "sem_ax_tune: lx=%d", lx);
    if (nel < 1 || reps < 1 || !best) return sem::fail(ctx, SEM_EINVAL, "sem_ax_tune: bad argument");
    const int64_t n = nel * lx * lx * lx;
    const int l2 = lx * lx;
    hipStream_t st = ctx->stream;
    std::vector<void*> tmp;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(st);
        for (void* p : tmp) (void)hipFree(p);
    };
    double* a[10] = {};
    for (int q = 0; q < 9; ++q) {
        hipError_t e = hipMalloc((void**)&a[q], sizeof(double) * n);
        if (e != hipSuccess) { cleanup(); return sem::check_hip(ctx, e, "sem_ax_tune: hipMalloc"); }
        tmp.push_back(a[q]);
    }
    {
        hipError_t e = hipMalloc((void**)&a[9], sizeof(double) * 2 * l2);
        if (e != hipSuccess) { cleanup(); return sem::check_hip(ctx, e, "sem_ax_tune: hipMalloc"); }
        tmp.push_back(a[9]);
    }
    double *u = a[0], *w = a[1], *h1 = a[8], *Dd = a[9];
    std::vector<double> dx(l2), dxt(l2);
    sem_gll(lx, nullptr, nullptr, dx.data(), dxt.data());   // the argument layout of the operator
    {
        hipError_t e = hipMemcpy(Dd, dx.data(), sizeof(double) * l2, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(Dd + l2, dxt.data(), sizeof(double) * l2, hipMemcpyHostToDevice);
        if (e != hipSuccess) { cleanup(); return sem::check_hip(ctx, e, "sem_ax_tune: hipMemcpy"); }
    }
    tune_fill_kernel<<<4096, 256, 0, st>>>(u, a[2], a[3], a[4], a[5], a[6], a[7], h1, n);
    const void* D[6] = {Dd, Dd, Dd, Dd + l2, Dd + l2, Dd + l2};
    const void* G[6] = {a[2], a[3], a[4], a[5], a[6], a[7]};
    rc = time_variants(ctx, lx, w, u, D, h1, G, nel, reps, us, best);
    cleanup();
    return rc;
}

extern "C" int sem_ax_tune_on(sem_ctx_t ctx, void* w, const void* u, const void* dx, const void* dy,
                              const void* dz, const void* dxt, const void* dyt, const void* dzt, const void* h1,
                              const void* g11, const void* g22, const void* g33, const void* g12,
                              const void* g13, const void* g23, int64_t nel, int lx, int reps, double* us,
                              int* best) {
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (!sem::lx_ok(lx)) return sem::fail(ctx, SEM_EUNSUPPORTED_LX, "sem_ax_tune_on: lx=%d", lx);
    if (nel < 1 || reps < 1 || !best || !w || !u) return sem::fail(ctx, SEM_EINVAL, "sem_ax_tune_on: bad argument");
    const void* D[6] = {dx, dy, dz, dxt, dyt, dzt};
    const void* G[6] = {g11, g22, g33, g12, g13, g23};
    for (int q = 0; q < 6; ++q)
        if (!D[q] || !G[q]) return sem::fail(ctx, SEM_EINVAL, "sem_ax_tune_on: null operator array");
    const size_t nb = (size_t)nel * lx * lx * lx * sizeof(double), nd = (size_t)lx * lx * sizeof(double);
    bool alias = overlaps(w, nb, u, nb) || overlaps(w, nb, h1, nb);
    for (int q = 0; q < 6; ++q) alias = alias || overlaps(w, nb, G[q], nb) || overlaps(w, nb, D[q], nd);
    if (alias) return sem::fail(ctx, SEM_EINVAL, "sem_ax_tune_on: output overlaps an input");
    return time_variants(ctx, lx, w, u, D, h1, G, nel, reps, us, best);
}
