// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "sem.h"

struct sem_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // small device workspace for reductions: partial sums and scalars
    double* red = nullptr;      // kRedSlots doubles
    double* host_pinned = nullptr;  // 64 doubles of pinned host memory
    // kernel variant of the float64 public operator per lx (SEM_AX_*;
    // SEM_AX_DEFAULT until sem_ax_set_variant or sem_ax_tune chooses one)
    int ax_variant[SEM_LX_MAX + 1] = {SEM_AX_DEFAULT, SEM_AX_DEFAULT, SEM_AX_DEFAULT, SEM_AX_DEFAULT, SEM_AX_DEFAULT,
                                      SEM_AX_DEFAULT, SEM_AX_DEFAULT, SEM_AX_DEFAULT, SEM_AX_DEFAULT, SEM_AX_DEFAULT,
                                      SEM_AX_DEFAULT, SEM_AX_DEFAULT, SEM_AX_DEFAULT};
};

struct sem_gs_s {
    sem_ctx_t ctx = nullptr;
    int64_t n_local = 0, n_unique = 0, n_shared = 0, n_entries = 0;
    int64_t n_masked = 0;       // Dirichlet nodes (negative ids): no unique index, zeroed by gs
    int32_t* off = nullptr;     // device, n_shared + 1
    int32_t* idx = nullptr;     // device, n_entries local indices
    double* mult = nullptr;     // device, n_local multiplicities
    double* owner = nullptr;    // device, n_local: 1 on the first copy of each id, else 0
    // dense unique numbering (ids renumbered in order of first appearance)
    int32_t* lid = nullptr;     // device, n_local: unique index of each local node (-1: Dirichlet)
    int32_t* uoff = nullptr;    // device, n_unique + 1: CSR of the local copies of every unique node
    int32_t* uidx = nullptr;    // device, n_local: local indices, ascending within a row; the
                                //   n_masked Dirichlet nodes last
    int32_t* upos = nullptr;    // device, n_local: position of each local node in uidx
};

namespace sem {

constexpr int kRedSlots = 1 << 16;

// record an error message on ctx (or the global slot when ctx is null)
int fail(sem_ctx_t ctx, int code, const char* fmt, ...);
// map a HIP error to SEM_EHIP with a message; returns SEM_OK on hipSuccess
int check_hip(sem_ctx_t ctx, hipError_t e, const char* what);
// make the context's device current
int enter(sem_ctx_t ctx);

inline bool lx_ok(int lx) { return lx >= SEM_LX_MIN && lx <= SEM_LX_MAX; }

// host-side GLL quantities (setup.hip)
void gll_host(int lx, double* xi, double* w, double* dhat /* dhat[i*lx+l] = l_l'(xi_i) */);

// operator arrays (device pointers); D in the compute precision, h1/G in the
// storage precision of the chosen AxKind
struct AxArgs {
    const void* D[6];
    const void* h1;
    const void* G[6];
    int64_t nel;
    int lx;
    // the solver form (lid != 0) reads the six factors from one packed array.
    // float64, float32: slice-blocked; for slice s = e lx^3 + k lx^2 (a
    // multiple of lx^2) and column ij, pair a of (g11,g22), (g33,g12),
    // (g13,g23) sits at 2-vector index 3 s + a lx^2 + ij.  bfloat16: one
    // record (h1 g11, h1 g22, h1 g33, h1 g12, h1 g13, h1 g23) per local node L
    // at 6 L, h1 folded in (h1 is then null)
    const void* Gp = nullptr;
    // Helmholtz: h2 B per local node in the storage type (+ h2 B u), or null
    const void* hb = nullptr;
};
enum class AxKind {
    F64,        // u, h1, G, D, w float64
    F32,        // u, h1, G, D, w float32
    F32_BF16    // u, D, w float32; h1, G bfloat16; float32 arithmetic
};
// Launch the operator.  With dot != nullptr it also skips when *skip != 0 and
// writes one float64 partial of sum u.w per workgroup (ax_blocks() of them).
// With lid != nullptr, u is a unique-node vector read as u[lid[L]] (0 where
// lid < 0); the output stays in the local layout.
int launch_ax(sem_ctx_t ctx, AxKind kind, const AxArgs& a, void* w, const void* u,
              const int* skip, double* dot, const int32_t* lid = nullptr);
int ax_blocks(int lx, int64_t nel);
// gather-scatter launch that returns at once when skip && *skip
int gs_launch(sem_gs_t gs, void* u, sem_dtype_t dtype, const int* skip);
// learned preconditioner z = P(r) on the bound operator (lp.hip); vectors
// float64 (f64) or float32; kernels return at once when skip && *skip
// unique: r and z are unique-node vectors of the bound plan, else local fields
int lp_apply(sem_lp_t lp, void* z, const void* r, bool f64, const int* skip, bool unique);
// Linear form on unique-node vectors without the final assembly: leaves the
// CSR-ordered element contributions (already weighted by 1/kappa_e, not yet by
// S = mult^-1/2) in *zl and reports whether the Jacobi base is on; the caller
// assembles z_u = S_u sum_segment zl (+ Minv_u r_u).  Returns SEM_EUNSUPPORTED_LX
// without launching anything when the network is not in its linear form.
int lp_apply_partial(sem_lp_t lp, const void* r, bool f64, const int* skip, const float** zl, bool* jacobi_base);
int64_t lp_rows(sem_lp_t lp);
sem_gs_t lp_plan(sem_lp_t lp);

// multigrid preconditioner (mg.hip): z = V(r) on unique-node vectors of its
// finest level's plan, float64 (f64) or float32; kernels return at once when
// skip && *skip
int mg_apply(sem_mg_t mg, void* z, const void* r, bool f64, const int* skip);
sem_gs_t mg_plan(sem_mg_t mg);
int64_t mg_nel(sem_mg_t mg);
// inverse of a symmetric positive definite matrix (row-major n x n, float64,
// in place) by Cholesky factorisation; false if a pivot is not positive
bool spd_inverse(std::vector<double>& A, int n);
// the six factors of an element-local operator packed for the solver form
// (the layout of AxArgs::Gp) in float32 or bfloat16 (times h1, when given);
// n local nodes, asynchronous on st
void pack_factors_f32(hipStream_t st, float* out, const double* const* G, int64_t n, int lx);
void pack_factors_bf16(hipStream_t st, uint16_t* out, const double* const* G, const double* h1, int64_t n,
                       int lx);

#ifdef __HIPCC__
// sum of the local copies of unique node u of a field in the local layout:
// wl[uidx[q]] for q in [uoff[u], uoff[u+1]), the first eight by independent
// predicated loads (issued together), summed in CSR order
template <typename T>
__device__ __forceinline__ T assemble_local(const T* __restrict__ wl, const int32_t* __restrict__ uoff,
                                            const int32_t* __restrict__ uidx, int64_t u) {
    const int32_t b = uoff[u], e = uoff[u + 1];
    int32_t L[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) L[q] = b + q < e ? uidx[b + q] : -1;
    T v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = L[q] >= 0 ? wl[L[q]] : T(0);
    T s = v[0];
#pragma unroll
    for (int q = 1; q < 8; ++q)
        if (b + q < e) s += v[q];
    for (int32_t q = b + 8; q < e; ++q) s += wl[uidx[q]];
    return s;
}

// Workgroup order for L2 locality: the hardware hands consecutive workgroups
// to the eight XCDs (each with its own L2) in turn.  With a grid of G
// workgroups, G a multiple of 8, logical block (b mod 8) G/8 + b/8 gives each
// XCD one contiguous eighth of the work; other grids keep their order.
__device__ __forceinline__ int64_t xcd_order(int64_t b, int64_t G) {
    return (G & 7) ? b : (b & 7) * (G >> 3) + (b >> 3);
}

// order LDS traffic within one wave (no workgroup barrier): a fence on each
// side of the wave barrier keeps the compiler from moving LDS accesses across it
__device__ __forceinline__ void wave_fence_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// sum over the 64 lanes of a wave
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
#endif

}  // namespace sem

#define SEM_HIP(ctx, call)                                                   \
    do {                                                                     \
        hipError_t e_ = (call);                                              \
        if (e_ != hipSuccess) return sem::check_hip((ctx), e_, #call);       \
    } while (0)

#define SEM_LAUNCH_CHECK(ctx) SEM_HIP((ctx), hipGetLastError())
