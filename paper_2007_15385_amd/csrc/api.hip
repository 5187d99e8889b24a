// Host side of the C ABI declared in include/pip_voronoi.h: argument
// validation, device selection and kernel launches.  Nothing here computes
// a label; every step of the test runs in the HIP kernels.
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <string>

#include "kernels.hpp"
#include "pip_voronoi.h"

struct pip_ctx_s {
    int device = 0;
    int cu_count = 0;
    std::mutex mu;
    int stream_blocks[8][2] = {};  // cached persistent grid per (kind, dtype); 0 = unknown
};

namespace {

thread_local std::string g_err = "no error";

pip_status fail(pip_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

pip_status hip_fail(hipError_t e, const char* what) {
    return fail(PIP_EHIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

// Makes ctx's device current for the duration of a call.
struct DeviceGuard {
    int old = -1;
    bool switched = false;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev) {
        err = hipGetDevice(&old);
        if (err == hipSuccess && old != dev) {
            err = hipSetDevice(dev);
            switched = err == hipSuccess;
        }
    }
    ~DeviceGuard() {
        if (switched) (void)hipSetDevice(old);
    }
};

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

pip_status check_polygon(const double* V, int32_t n) {
    if (!V) return fail(PIP_EINVAL, "V is NULL");
    if (!aligned(V, 8)) return fail(PIP_EINVAL, "V is not 8-byte aligned");
    if (n < 3) return fail(PIP_EINVAL, "n = %d: a polygon needs at least 3 vertices", (int)n);
    if (n > PIP_MAX_EDGES)
        return fail(PIP_EUNSUPPORTED, "n = %d exceeds the compiled limit of %d edges", (int)n,
                    PIP_MAX_EDGES);
    return PIP_OK;
}

pip_status check_points(const void* Q, pip_dtype qdt, int64_t m) {
    if (qdt != PIP_F32 && qdt != PIP_F64) return fail(PIP_EINVAL, "qdt = %d is not a pip_dtype", (int)qdt);
    if (m < 0) return fail(PIP_EINVAL, "m = %lld is negative", (long long)m);
    if (m > 0 && !Q) return fail(PIP_EINVAL, "Q is NULL");
    const size_t a = qdt == PIP_F32 ? 8 : 16;
    if (m > 0 && !aligned(Q, a)) return fail(PIP_EINVAL, "Q is not %zu-byte aligned", a);
    if (m > (int64_t(1) << 46)) return fail(PIP_EUNSUPPORTED, "m = %lld is too large", (long long)m);
    return PIP_OK;
}

int persistent_blocks(pip_ctx ctx, int kind, int qdt) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    int& b = ctx->stream_blocks[kind][qdt];
    if (b == 0) {
        int per_cu = 0;
        if (pipdev::stream_max_blocks_per_cu(kind, qdt, &per_cu) != hipSuccess || per_cu < 1)
            per_cu = 1;
        b = per_cu * ctx->cu_count;
    }
    return b;
}

pip_status run_stream(pip_ctx ctx, int kind, const double* V, int32_t n, const void* Q,
                      pip_dtype qdt, int64_t m, uint32_t* labels, float* margin,
                      int32_t* status, hipStream_t stream) {
    if (!ctx) return fail(PIP_EINVAL, "ctx is NULL");
    pip_status s = check_polygon(V, n);
    if (s != PIP_OK) return s;
    s = check_points(Q, qdt, m);
    if (s != PIP_OK) return s;
    if (kind == pipdev::K_MARGIN) {
        if (m > 0 && !margin) return fail(PIP_EINVAL, "max_margin is NULL");
        if (m > 0 && !aligned(margin, 4)) return fail(PIP_EINVAL, "max_margin is not 4-byte aligned");
    } else {
        if (m > 0 && !labels) return fail(PIP_EINVAL, "labels is NULL");
        if (m > 0 && !aligned(labels, 4)) return fail(PIP_EINVAL, "labels is not 4-byte aligned");
    }
    if (status && !aligned(status, 4)) return fail(PIP_EINVAL, "status is not 4-byte aligned");
    if (m == 0 && !status) return PIP_OK;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    pipdev::StreamLaunch L;
    L.kind = kind;
    L.V = V;
    L.n = n;
    L.Q = Q;
    L.qdt = (int)qdt;
    L.m = m;
    L.labels = labels;
    L.margin = margin;
    L.status = status;
    L.max_blocks = persistent_blocks(ctx, kind, (int)qdt);
    L.stream = stream;
    hipError_t e = pipdev::launch_stream(L);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return PIP_OK;
}

}  // namespace

extern "C" {

int pip_version(void) { return 100; }

const char* pip_status_str(pip_status s) {
    switch (s) {
        case PIP_OK: return "PIP_OK";
        case PIP_EINVAL: return "PIP_EINVAL";
        case PIP_EDEGENERATE: return "PIP_EDEGENERATE";
        case PIP_ENONCONVEX: return "PIP_ENONCONVEX";
        case PIP_EHIP: return "PIP_EHIP";
        case PIP_ENOMEM: return "PIP_ENOMEM";
        case PIP_EUNSUPPORTED: return "PIP_EUNSUPPORTED";
    }
    return "PIP_UNKNOWN";
}

const char* pip_last_error(pip_ctx) { return g_err.c_str(); }

pip_status pip_create(int hip_device, pip_ctx* out) {
    if (!out) return fail(PIP_EINVAL, "out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (hip_device < 0 || hip_device >= count)
        return fail(PIP_EINVAL, "device %d does not exist (%d devices)", hip_device, count);
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, hip_device);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    pip_ctx c = new (std::nothrow) pip_ctx_s();
    if (!c) return fail(PIP_ENOMEM, "out of host memory");
    c->device = hip_device;
    c->cu_count = cus;
    *out = c;
    return PIP_OK;
}

void pip_destroy(pip_ctx ctx) { delete ctx; }

pip_status polygon_to_generators(pip_ctx ctx, const double* V, int32_t n, double* P,
                                 int32_t* status, hipStream_t stream) {
    if (!ctx) return fail(PIP_EINVAL, "ctx is NULL");
    pip_status s = check_polygon(V, n);
    if (s != PIP_OK) return s;
    if (!P) return fail(PIP_EINVAL, "P is NULL");
    if (!aligned(P, 8)) return fail(PIP_EINVAL, "P is not 8-byte aligned");
    if (status && !aligned(status, 4)) return fail(PIP_EINVAL, "status is not 4-byte aligned");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipError_t e = pipdev::launch_generators_one(V, n, P, status, stream);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return PIP_OK;
}

pip_status pip_voronoi(pip_ctx ctx, const double* V, int32_t n, const void* Q, pip_dtype qdt,
                       int64_t m, uint32_t* labels, int32_t* status, hipStream_t stream) {
    return run_stream(ctx, pipdev::K_VORONOI, V, n, Q, qdt, m, labels, nullptr, status, stream);
}

pip_status pip_sign_of_offset(pip_ctx ctx, const double* V, int32_t n, const void* Q,
                              pip_dtype qdt, int64_t m, uint32_t* labels, int32_t* status,
                              hipStream_t stream) {
    return run_stream(ctx, pipdev::K_SOO, V, n, Q, qdt, m, labels, nullptr, status, stream);
}

pip_status pip_ray_crossing(pip_ctx ctx, const double* V, int32_t n, const void* Q,
                            pip_dtype qdt, int64_t m, uint32_t* labels, int32_t* status,
                            hipStream_t stream) {
    return run_stream(ctx, pipdev::K_RAY, V, n, Q, qdt, m, labels, nullptr, status, stream);
}

pip_status pip_voronoi_fp32_plain(pip_ctx ctx, const double* V, int32_t n, const void* Q,
                                  pip_dtype qdt, int64_t m, uint32_t* labels, int32_t* status,
                                  hipStream_t stream) {
    return run_stream(ctx, pipdev::K_PLAIN, V, n, Q, qdt, m, labels, nullptr, status, stream);
}

pip_status pip_voronoi_max_margin(pip_ctx ctx, const double* V, int32_t n, const void* Q,
                                  pip_dtype qdt, int64_t m, float* max_margin, int32_t* status,
                                  hipStream_t stream) {
    return run_stream(ctx, pipdev::K_MARGIN, V, n, Q, qdt, m, nullptr, max_margin, status, stream);
}

}  // extern "C"
