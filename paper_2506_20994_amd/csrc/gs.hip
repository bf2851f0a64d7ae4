// Gather-scatter sum u <- Q Q^T u (paper Sec. 2.1).
//
// Plan: only ids that occur more than once need work.  Those "shared" ids are
// listed in the order their first local copy appears (so neighbouring threads
// touch neighbouring memory), each with the CSR list of its local copies in
// increasing local index.  One thread per shared id sums its copies in that
// fixed order and writes the sum back to every copy: deterministic, no atomics.
//
// Negative ids mark Dirichlet nodes (homogeneous Dirichlet conditions): they
// are no unknowns.  They take no unique index (lid = -1), sit after every
// unique node's copies in the CSR order (positions n_local - n_masked ..
// n_local of uidx, in increasing local index), and gather-scatter sets them to
// zero.  Their multiplicity is 1 and their owner weight 0.
#include <algorithm>
#include <vector>

#include "sem_internal.h"

namespace {

constexpr int kBlock = 256;

// threads [0, n_shared) sum the shared ids; threads [n_shared, n_shared +
// n_masked) zero the Dirichlet nodes listed in midx
template <typename T>
__global__ void gs_kernel(T* __restrict__ u, const int32_t* __restrict__ off,
                          const int32_t* __restrict__ idx, int64_t n_shared, const int* __restrict__ skip,
                          const int32_t* __restrict__ midx, int64_t n_masked) {
    if (skip && *skip) return;
    const int64_t g = sem::xcd_order(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (g >= n_shared) {
        if (g < n_shared + n_masked) u[midx[g - n_shared]] = T(0);
        return;
    }
    // the first eight copies (a hexahedral mesh has at most eight) by independent
    // predicated loads issued together, summed in CSR order; any further copies
    // one by one
    const int32_t b = off[g], e = off[g + 1];
    int32_t L[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) L[q] = b + q < e ? idx[b + q] : -1;
    T v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = L[q] >= 0 ? u[L[q]] : T(0);
    T s = v[0];
#pragma unroll
    for (int q = 1; q < 8; ++q)
        if (L[q] >= 0) s += v[q];
    for (int32_t q = b + 8; q < e; ++q) s += u[idx[q]];
#pragma unroll
    for (int q = 0; q < 8; ++q)
        if (L[q] >= 0) u[L[q]] = s;
    for (int32_t q = b + 8; q < e; ++q) u[idx[q]] = s;
}

__global__ void mult_kernel(double* __restrict__ mult, const int32_t* __restrict__ off,
                            const int32_t* __restrict__ idx, int64_t n_shared) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= n_shared) return;
    const int32_t b = off[g], e = off[g + 1];
    for (int32_t q = b; q < e; ++q) mult[idx[q]] = (double)(e - b);
}

__global__ void owner_kernel(double* __restrict__ owner, const int32_t* __restrict__ off,
                             const int32_t* __restrict__ idx, int64_t n_shared) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= n_shared) return;
    const int32_t b = off[g], e = off[g + 1];
    for (int32_t q = b + 1; q < e; ++q) owner[idx[q]] = 0.0;   // idx is ascending: idx[b] owns
}

__global__ void zero_at_kernel(double* __restrict__ a, const int32_t* __restrict__ idx, int64_t n) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g < n) a[idx[g]] = 0.0;
}

__global__ void fill_kernel(double* __restrict__ p, double v, int64_t n) {
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n;
         L += (int64_t)gridDim.x * blockDim.x)
        p[L] = v;
}

}  // namespace

extern "C" int sem_gs_setup(sem_ctx_t ctx, const int64_t* ids, int64_t n_local, sem_gs_t* out) {
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (!out) return sem::fail(ctx, SEM_EINVAL, "sem_gs_setup: null output pointer");
    *out = nullptr;
    if (n_local < 0 || n_local >= ((int64_t)1 << 31))
        return sem::fail(ctx, SEM_EINVAL, "sem_gs_setup: n_local=%lld outside [0, 2^31)", (long long)n_local);
    if (n_local > 0 && !ids) return sem::fail(ctx, SEM_EINVAL, "sem_gs_setup: null ids");
    int64_t idmax = -1, n_masked = 0;
    for (int64_t L = 0; L < n_local; ++L) {
        if (ids[L] < 0) ++n_masked;
        else idmax = std::max(idmax, ids[L]);
    }
    // Dense relabelling when ids are sparse: map them onto 0..n_distinct-1 by
    // their sorted order, so the counting arrays stay O(n_local).
    std::vector<int64_t> relabel;
    const int64_t* key = ids;
    if (idmax > 4 * n_local + 1024) {
        std::vector<int64_t> uniq;
        uniq.reserve((size_t)(n_local - n_masked));
        for (int64_t L = 0; L < n_local; ++L)
            if (ids[L] >= 0) uniq.push_back(ids[L]);
        std::sort(uniq.begin(), uniq.end());
        uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
        relabel.resize((size_t)n_local);
        for (int64_t L = 0; L < n_local; ++L)
            relabel[(size_t)L] = ids[L] < 0 ? -1 : std::lower_bound(uniq.begin(), uniq.end(), ids[L]) - uniq.begin();
        idmax = (int64_t)uniq.size() - 1;
        key = relabel.data();
    }
    // count copies per id
    std::vector<int32_t> count((size_t)(idmax + 1), 0);
    for (int64_t L = 0; L < n_local; ++L)
        if (key[L] >= 0) ++count[(size_t)key[L]];
    int64_t n_unique = 0;
    for (int32_t c : count) n_unique += (c > 0);
    // shared ids in order of first appearance; slot[id] = shared index or -1
    std::vector<int32_t> slot((size_t)(idmax + 1), -1);
    std::vector<int32_t> off(1, 0);
    int64_t n_shared = 0;
    for (int64_t L = 0; L < n_local; ++L) {
        const int64_t g = key[L];
        if (g >= 0 && count[(size_t)g] > 1 && slot[(size_t)g] < 0) {
            slot[(size_t)g] = (int32_t)n_shared++;
            off.push_back(off.back() + count[(size_t)g]);
        }
    }
    std::vector<int32_t> idx((size_t)off.back());
    std::vector<int32_t> fillpos(off.begin(), off.end() - 1);
    for (int64_t L = 0; L < n_local; ++L) {
        if (key[L] < 0) continue;
        const int32_t s = slot[(size_t)key[L]];
        if (s >= 0) idx[(size_t)fillpos[(size_t)s]++] = (int32_t)L;
    }
    std::vector<int32_t>().swap(fillpos);
    // dense unique numbering in order of first appearance and the CSR of the
    // local copies of every unique node (reuses `slot` as id -> unique index)
    std::fill(slot.begin(), slot.end(), -1);
    std::vector<int32_t> lid((size_t)n_local);
    std::vector<int32_t> uoff(1, 0);
    uoff.reserve((size_t)n_unique + 1);
    int32_t nu = 0;
    for (int64_t L = 0; L < n_local; ++L) {
        const int64_t g = key[L];
        if (g < 0) {
            lid[(size_t)L] = -1;
            continue;
        }
        if (slot[(size_t)g] < 0) {
            slot[(size_t)g] = nu++;
            uoff.push_back(uoff.back() + count[(size_t)g]);
        }
        lid[(size_t)L] = slot[(size_t)g];
    }
    // CSR positions: the copies of every unique node, then the Dirichlet nodes
    std::vector<int32_t> uidx((size_t)n_local), upos((size_t)n_local);
    {
        std::vector<int32_t> pos(uoff.begin(), uoff.end() - 1);
        int32_t tail = uoff.back();
        for (int64_t L = 0; L < n_local; ++L) {
            const int32_t u = lid[(size_t)L];
            const int32_t q = u >= 0 ? pos[(size_t)u]++ : tail++;
            uidx[(size_t)q] = (int32_t)L;
            upos[(size_t)L] = q;
        }
    }
    std::vector<int32_t>().swap(count);
    std::vector<int32_t>().swap(slot);

    auto* gs = new sem_gs_s();
    gs->ctx = ctx;
    gs->n_local = n_local;
    gs->n_unique = n_unique;
    gs->n_shared = n_shared;
    gs->n_masked = n_masked;
    gs->n_entries = (int64_t)idx.size();
    hipError_t e = hipMalloc(&gs->off, sizeof(int32_t) * off.size());
    if (e == hipSuccess && !idx.empty()) e = hipMalloc(&gs->idx, sizeof(int32_t) * idx.size());
    if (e == hipSuccess && n_local > 0) e = hipMalloc(&gs->mult, sizeof(double) * n_local);
    if (e == hipSuccess && n_local > 0) e = hipMalloc(&gs->owner, sizeof(double) * n_local);
    if (e == hipSuccess && n_local > 0) e = hipMalloc(&gs->lid, sizeof(int32_t) * n_local);
    if (e == hipSuccess && n_local > 0) e = hipMalloc(&gs->uidx, sizeof(int32_t) * n_local);
    if (e == hipSuccess && n_local > 0) e = hipMalloc(&gs->upos, sizeof(int32_t) * n_local);
    if (e == hipSuccess && n_local > 0)
        e = hipMemcpy(gs->upos, upos.data(), sizeof(int32_t) * n_local, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&gs->uoff, sizeof(int32_t) * uoff.size());
    if (e == hipSuccess && n_local > 0)
        e = hipMemcpy(gs->lid, lid.data(), sizeof(int32_t) * n_local, hipMemcpyHostToDevice);
    if (e == hipSuccess && n_local > 0)
        e = hipMemcpy(gs->uidx, uidx.data(), sizeof(int32_t) * n_local, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(gs->uoff, uoff.data(), sizeof(int32_t) * uoff.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(gs->off, off.data(), sizeof(int32_t) * off.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !idx.empty())
        e = hipMemcpy(gs->idx, idx.data(), sizeof(int32_t) * idx.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && n_local > 0) {
        fill_kernel<<<1024, kBlock, 0, ctx->stream>>>(gs->mult, 1.0, n_local);
        fill_kernel<<<1024, kBlock, 0, ctx->stream>>>(gs->owner, 1.0, n_local);
        e = hipGetLastError();
        if (e == hipSuccess && n_shared > 0) {
            const unsigned gr = (unsigned)((n_shared + kBlock - 1) / kBlock);
            mult_kernel<<<gr, kBlock, 0, ctx->stream>>>(gs->mult, gs->off, gs->idx, n_shared);
            owner_kernel<<<gr, kBlock, 0, ctx->stream>>>(gs->owner, gs->off, gs->idx, n_shared);
            e = hipGetLastError();
        }
        if (e == hipSuccess && n_masked > 0) {
            const unsigned gr = (unsigned)((n_masked + kBlock - 1) / kBlock);
            zero_at_kernel<<<gr, kBlock, 0, ctx->stream>>>(gs->owner, gs->uidx + (n_local - n_masked), n_masked);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    }
    if (e != hipSuccess) {
        sem_gs_destroy(gs);
        return sem::check_hip(ctx, e, "sem_gs_setup");
    }
    *out = gs;
    return SEM_OK;
}

extern "C" int sem_gs_destroy(sem_gs_t gs) {
    if (!gs) return SEM_OK;
    if (gs->ctx) (void)hipSetDevice(gs->ctx->device);
    if (gs->off) (void)hipFree(gs->off);
    if (gs->idx) (void)hipFree(gs->idx);
    if (gs->mult) (void)hipFree(gs->mult);
    if (gs->owner) (void)hipFree(gs->owner);
    if (gs->lid) (void)hipFree(gs->lid);
    if (gs->uoff) (void)hipFree(gs->uoff);
    if (gs->uidx) (void)hipFree(gs->uidx);
    if (gs->upos) (void)hipFree(gs->upos);
    delete gs;
    return SEM_OK;
}

extern "C" int sem_gs_info(sem_gs_t gs, int64_t* n_unique, int64_t* n_shared) {
    if (!gs) return sem::fail(nullptr, SEM_EINVAL, "sem_gs_info: null plan");
    if (n_unique) *n_unique = gs->n_unique;
    if (n_shared) *n_shared = gs->n_shared;
    return SEM_OK;
}

extern "C" int sem_gs_dirichlet_count(sem_gs_t gs, int64_t* n_dirichlet) {
    if (!gs) return sem::fail(nullptr, SEM_EINVAL, "sem_gs_dirichlet_count: null plan");
    if (n_dirichlet) *n_dirichlet = gs->n_masked;
    return SEM_OK;
}

namespace sem {

int gs_launch(sem_gs_t gs, void* u, sem_dtype_t dtype, const int* skip) {
    sem_ctx_t ctx = gs->ctx;
    const int64_t nt = gs->n_shared + gs->n_masked;
    if (nt == 0) return SEM_OK;
    if (!u) return fail(ctx, SEM_EINVAL, "sem_gs: null field");
    constexpr int kGsBlock = 512;           // measured: 256 and 1024 threads are slower
    const unsigned grid = (unsigned)((nt + 8 * kGsBlock - 1) / (8 * kGsBlock) * 8);   // a multiple of 8
    const int32_t* midx = gs->uidx + (gs->n_local - gs->n_masked);
    if (dtype == SEM_F64)
        gs_kernel<double><<<grid, kGsBlock, 0, ctx->stream>>>((double*)u, gs->off, gs->idx, gs->n_shared, skip,
                                                              midx, gs->n_masked);
    else if (dtype == SEM_F32)
        gs_kernel<float><<<grid, kGsBlock, 0, ctx->stream>>>((float*)u, gs->off, gs->idx, gs->n_shared, skip,
                                                             midx, gs->n_masked);
    else
        return fail(ctx, SEM_EINVAL, "sem_gs: dtype %d not supported (F64 or F32)", (int)dtype);
    SEM_LAUNCH_CHECK(ctx);
    return SEM_OK;
}

}  // namespace sem

extern "C" int sem_gs(sem_gs_t gs, void* u, sem_dtype_t dtype) {
    if (!gs) return sem::fail(nullptr, SEM_EINVAL, "sem_gs: null plan");
    int rc = sem::enter(gs->ctx);
    if (rc) return rc;
    return sem::gs_launch(gs, u, dtype, nullptr);
}

extern "C" int sem_gs_mult(sem_gs_t gs, double* mult) {
    if (!gs) return sem::fail(nullptr, SEM_EINVAL, "sem_gs_mult: null plan");
    sem_ctx_t ctx = gs->ctx;
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (gs->n_local == 0) return SEM_OK;
    if (!mult) return sem::fail(ctx, SEM_EINVAL, "sem_gs_mult: null output");
    SEM_HIP(ctx, hipMemcpyAsync(mult, gs->mult, sizeof(double) * gs->n_local,
                                hipMemcpyDeviceToDevice, ctx->stream));
    return SEM_OK;
}

extern "C" int sem_gs_owner(sem_gs_t gs, double* wgt) {
    if (!gs) return sem::fail(nullptr, SEM_EINVAL, "sem_gs_owner: null plan");
    sem_ctx_t ctx = gs->ctx;
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (gs->n_local == 0) return SEM_OK;
    if (!wgt) return sem::fail(ctx, SEM_EINVAL, "sem_gs_owner: null output");
    SEM_HIP(ctx, hipMemcpyAsync(wgt, gs->owner, sizeof(double) * gs->n_local,
                                hipMemcpyDeviceToDevice, ctx->stream));
    return SEM_OK;
}
