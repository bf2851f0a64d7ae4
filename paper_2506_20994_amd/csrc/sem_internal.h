// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <string>

#include "sem.h"

struct sem_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // small device workspace for reductions: partial sums and scalars
    double* red = nullptr;      // kRedSlots doubles
    unsigned int* counter = nullptr;
    double* host_pinned = nullptr;  // 64 doubles of pinned host memory
};

struct sem_gs_s {
    sem_ctx_t ctx = nullptr;
    int64_t n_local = 0, n_unique = 0, n_shared = 0, n_entries = 0;
    int32_t* off = nullptr;     // device, n_shared + 1
    int32_t* idx = nullptr;     // device, n_entries local indices
    double* mult = nullptr;     // device, n_local multiplicities
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

}  // namespace sem

#define SEM_HIP(ctx, call)                                                   \
    do {                                                                     \
        hipError_t e_ = (call);                                              \
        if (e_ != hipSuccess) return sem::check_hip((ctx), e_, #call);       \
    } while (0)

#define SEM_LAUNCH_CHECK(ctx) SEM_HIP((ctx), hipGetLastError())
