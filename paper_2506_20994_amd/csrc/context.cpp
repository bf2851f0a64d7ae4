// Context lifetime, error reporting, scatter and precision conversion.
#include <cstdarg>
#include <cstring>

#include "sem_internal.h"

static thread_local std::string g_err;

namespace sem {

int fail(sem_ctx_t ctx, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf; else g_err = buf;
    return code;
}

int check_hip(sem_ctx_t ctx, hipError_t e, const char* what) {
    if (e == hipSuccess) return SEM_OK;
    return fail(ctx, SEM_EHIP, "%s failed: %s", what, hipGetErrorString(e));
}

int enter(sem_ctx_t ctx) {
    if (!ctx) return fail(nullptr, SEM_EINVAL, "null context");
    int cur = -1;
    SEM_HIP(ctx, hipGetDevice(&cur));
    if (cur != ctx->device) SEM_HIP(ctx, hipSetDevice(ctx->device));
    return SEM_OK;
}

}  // namespace sem

extern "C" int sem_create(sem_ctx_t* out, void* stream) {
    if (!out) return sem::fail(nullptr, SEM_EINVAL, "sem_create: null output pointer");
    *out = nullptr;
    auto* c = new sem_ctx_s();
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipMalloc(&c->red, sizeof(double) * sem::kRedSlots);
    if (e == hipSuccess) e = hipHostMalloc(&c->host_pinned, sizeof(double) * 64, hipHostMallocDefault);
    if (e != hipSuccess) {
        int rc = sem::check_hip(nullptr, e, "sem_create");
        if (c->red) (void)hipFree(c->red);
        delete c;
        return rc;
    }
    c->stream = static_cast<hipStream_t>(stream);
    *out = c;
    return SEM_OK;
}

extern "C" int sem_destroy(sem_ctx_t ctx) {
    if (!ctx) return SEM_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->red) (void)hipFree(ctx->red);
    if (ctx->host_pinned) (void)hipHostFree(ctx->host_pinned);
    delete ctx;
    return SEM_OK;
}

extern "C" int sem_set_stream(sem_ctx_t ctx, void* stream) {
    if (!ctx) return sem::fail(nullptr, SEM_EINVAL, "null context");
    ctx->stream = static_cast<hipStream_t>(stream);
    return SEM_OK;
}

extern "C" const char* sem_last_error(sem_ctx_t ctx) {
    return ctx ? ctx->err.c_str() : g_err.c_str();
}

extern "C" int sem_sync(sem_ctx_t ctx) {
    int rc = sem::enter(ctx);
    if (rc) return rc;
    SEM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return SEM_OK;
}
