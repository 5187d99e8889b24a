// Host side of the C ABI declared in include/pip_voronoi.h: argument
// validation, device selection and kernel launches.  Nothing here computes
// a label; every step of the test runs in the HIP kernels.
#include <cstdarg>
#include <cstdio>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "pip_voronoi.h"

struct pip_ctx_s {
    int device = 0;
    int cu_count = 0;
    std::mutex mu;
    int stream_blocks[8][2] = {};  // cached persistent grid per (kind, dtype); 0 = unknown
    int mfma_blocks[2][4] = {};    // same for the matrix-core screen (kind, edge bucket)
    int raster_blocks[2] = {};     // persistent grid of the raster kernel (per-edge, radial)
    int batched_blocks_per_cu = 0;
    int mfma_min_edges = 25;       // polygons with at least this many edges use the matrix cores
    int radial_min_edges = 0;      // Voronoi polygons with at least this many edges: radial pre-screen (0: off)
    int radial_blocks = 0;         // persistent grid of the radial kernel
    int allpairs_cull = 0;         // skip (polygon, wave) pairs whose bounding disk misses the points
    int cost_cull = 0;             // skip (pose, wave) pairs of the collision cost likewise
    int allpairs_pair = 0;         // antipodal edge pairs for centrally symmetric polygons
    int cost_pair = 0;             // the same for the collision cost's footprint
    int early_exit = 0;            // the raster's early break (Section 5) when every pixel is outside
    void* scratch = nullptr;       // this device's copy of the static scratch array (no-alloc calls)
    hipError_t scratch_err = hipSuccess;  // why `scratch` is null, if it is
};

// A plan: one batched request bound to its buffers, its own workspace, the
// tile shape chosen by the autotuner and the captured hipGraph.
struct pip_index_s {
    pip_ctx ctx = nullptr;
    int64_t P = 0, cells = 0, entries = 0;
    void* mem = nullptr;       // records, rows, generators, grid, counters, offsets
    void* list_mem = nullptr;  // cell lists (sized after counting)
    int sf = 1, sgx = 1, nbins = 1;  // super-cells of the binned query (sf x sf cells each)
    pipdev::LocRec* rec = nullptr;
    float4* qrec = nullptr;
    double2* gen = nullptr;
    pipdev::LocGrid* grid = nullptr;
    int32_t* cell_off = nullptr;
    pipdev::LocEntry* list = nullptr;
    int blocks = 0;
};

struct AllpairsArgs {
    int32_t P = 0, n = 0;
    const double* V = nullptr;
    const float* Q = nullptr;
    int64_t m = 0;
    uint32_t* labels = nullptr;
    int32_t* counts = nullptr;
    int32_t* status = nullptr;
};

struct CostArgs {
    const float* F = nullptr;
    int32_t n = 0;
    const float* pose = nullptr;
    int64_t K = 0;
    const float* Q = nullptr;
    int64_t m = 0;
    float* cost = nullptr;                                     // forward
    const float* grad_cost = nullptr;                          // backward
    float* grad_pose = nullptr;
    float* grad_F = nullptr;
    float* residual = nullptr;
};

struct pip_plan_s {
    pip_ctx ctx = nullptr;
    int kind = 0;  // 0: batched, 1: all pairs, 2: cost forward, 3: cost backward
    AllpairsArgs A{};
    CostArgs Cst{};
    pip_variant_config acfg{};
    uint32_t* ref_counts = nullptr;
    pipdev::BatchedDev D{};
    void* ws = nullptr;
    size_t ws_bytes = 0;
    pip_batched_config cfg{};
    float best_ms = -1.f;
    int64_t label_words = 0;
    uint32_t* ref_labels = nullptr;
    unsigned long long* d_diff = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
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

// Workspace of pip_voronoi_batched_noalloc.  Every GPU the library runs on
// holds its own copy at its own address until the process ends.  In host
// code `scratch` is only a host-side stand-in: kernels, copies and fills take
// the device address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[PIP_BATCHED_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxScratchDevices] = {};

// Device address of `scratch` on `device`, looked up once per device with
// that device current.
hipError_t scratch_address(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_addr[device] = p;
    }
    *out = g_scratch_addr[device];
    return hipSuccess;
}

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

int mfma_blocks(pip_ctx ctx, int kind, int n) {
    const int bucket = n <= 8 ? 0 : n <= 16 ? 1 : n <= 32 ? 2 : 3;
    std::lock_guard<std::mutex> lk(ctx->mu);
    int& b = ctx->mfma_blocks[kind == pipdev::K_SOO ? 1 : 0][bucket];
    if (b == 0) {
        int per_cu = 0;
        if (pipdev::stream_mfma_max_blocks_per_cu(kind, n, &per_cu) != hipSuccess || per_cu < 1)
            per_cu = 1;
        b = per_cu * ctx->cu_count;
    }
    return b;
}

int radial_blocks(pip_ctx ctx) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->radial_blocks == 0) {
        int per_cu = 0;
        if (pipdev::radial_max_blocks_per_cu(&per_cu) != hipSuccess || per_cu < 1) per_cu = 1;
        ctx->radial_blocks = per_cu * ctx->cu_count;
    }
    return ctx->radial_blocks;
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
    L.mfma = (qdt == PIP_F32 && (kind == pipdev::K_VORONOI || kind == pipdev::K_SOO) &&
              ctx->mfma_min_edges > 0 && n >= ctx->mfma_min_edges)
                 ? 1
                 : 0;
    L.radial = (qdt == PIP_F32 && kind == pipdev::K_VORONOI && ctx->radial_min_edges > 0 &&
                n >= ctx->radial_min_edges)
                   ? 1
                   : 0;
    L.max_blocks = L.radial ? radial_blocks(ctx)
                 : L.mfma   ? mfma_blocks(ctx, kind, n)
                            : persistent_blocks(ctx, kind, (int)qdt);
    L.stream = stream;
    if (qdt == PIP_F32 && kind != pipdev::K_MARGIN) {
        // the recheck queues code a point as (chunk iteration << 9 | point):
        // every wave must walk fewer than 2^23 chunks of 512 points
        const int64_t nchunks = (m + 511) / 512;
        const int64_t want = (nchunks + 3) / 4;
        const int64_t grid = want < L.max_blocks ? want : L.max_blocks;
        const int64_t waves = 4 * (grid > 0 ? grid : 1);
        if ((nchunks + waves - 1) / waves >= (int64_t(1) << 23))
            return fail(PIP_EUNSUPPORTED, "m = %lld points is too large for one launch on this device; "
                        "split the point array", (long long)m);
    }
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
    {  // this device's scratch array (only pip_voronoi_batched_noalloc needs it)
        DeviceGuard g(hip_device);
        c->scratch_err = g.err != hipSuccess ? g.err : scratch_address(hip_device, &c->scratch);
        if (c->scratch_err != hipSuccess) c->scratch = nullptr;
    }
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

pip_status pip_voronoi_radial_bounds(pip_ctx ctx, const double* V, int32_t n, float* out,
                                     hipStream_t stream) {
    if (!ctx) return fail(PIP_EINVAL, "ctx is NULL");
    pip_status s = check_polygon(V, n);
    if (s != PIP_OK) return s;
    if (!out) return fail(PIP_EINVAL, "out is NULL");
    if (!aligned(out, 4)) return fail(PIP_EINVAL, "out is not 4-byte aligned");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipError_t e = pipdev::launch_radial_bounds(V, n, out, stream);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return PIP_OK;
}

pip_status pip_screen_table(pip_ctx ctx, int32_t test, int32_t matrix, const double* V, int32_t n,
                            float* out, hipStream_t stream) {
    if (!ctx) return fail(PIP_EINVAL, "ctx is NULL");
    pip_status s = check_polygon(V, n);
    if (s != PIP_OK) return s;
    if (test != 0 && test != 1) return fail(PIP_EINVAL, "test = %d must be 0 or 1", (int)test);
    if (matrix != 0 && matrix != 1) return fail(PIP_EINVAL, "matrix = %d must be 0 or 1", (int)matrix);
    if (!out || !aligned(out, 4)) return fail(PIP_EINVAL, "out is NULL or not 4-byte aligned");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipError_t e = pipdev::launch_screen_table(V, n, test ? pipdev::K_SOO : pipdev::K_VORONOI,
                                               matrix ? pipdev::kMfmaScreenFactor : 4.05, out,
                                               stream);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return PIP_OK;
}

pip_status pip_mfma_margin_probe(pip_ctx ctx, const float* in, int64_t count, float* out,
                                 hipStream_t stream) {
    if (!ctx) return fail(PIP_EINVAL, "ctx is NULL");
    if (count < 0) return fail(PIP_EINVAL, "count is negative");
    if (count > (int64_t(1) << 40)) return fail(PIP_EUNSUPPORTED, "count is too large");
    if (count > 0 && (!in || !out || !aligned(in, 4) || !aligned(out, 4)))
        return fail(PIP_EINVAL, "in / out is NULL or misaligned");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipError_t e = pipdev::launch_mfma_probe(in, count, out, stream);
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

pip_status pip_voronoi_raster(pip_ctx ctx, const double* V, int32_t n, double x0, double y0,
                              double dx, double dy, int64_t width, int64_t height,
                              uint32_t* labels, int32_t* status, hipStream_t stream) {
    if (!ctx) return fail(PIP_EINVAL, "ctx is NULL");
    pip_status s = check_polygon(V, n);
    if (s != PIP_OK) return s;
    if (!std::isfinite(x0) || !std::isfinite(y0) || !std::isfinite(dx) || !std::isfinite(dy))
        return fail(PIP_EINVAL, "x0, y0, dx and dy must be finite");
    if (width < 0 || height < 0)
        return fail(PIP_EINVAL, "width = %lld, height = %lld: negative size", (long long)width,
                    (long long)height);
    if (width > (int64_t(1) << 24) || height > (int64_t(1) << 31))
        return fail(PIP_EUNSUPPORTED, "raster %lld x %lld exceeds 2^24 columns or 2^31 rows",
                    (long long)width, (long long)height);
    const bool empty = width == 0 || height == 0;
    if (!empty && !labels) return fail(PIP_EINVAL, "labels is NULL");
    if (!empty && !aligned(labels, 4)) return fail(PIP_EINVAL, "labels is not 4-byte aligned");
    if (status && !aligned(status, 4)) return fail(PIP_EINVAL, "status is not 4-byte aligned");
    if (empty && !status) return PIP_OK;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    const int radial = ctx->radial_min_edges > 0 && n >= ctx->radial_min_edges ? 1 : 0;
    int blocks;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (ctx->raster_blocks[radial] == 0) {
            int per_cu = 0;
            if (pipdev::raster_max_blocks_per_cu(radial, &per_cu) != hipSuccess || per_cu < 1)
                per_cu = 1;
            ctx->raster_blocks[radial] = per_cu * ctx->cu_count;
        }
        blocks = ctx->raster_blocks[radial];
    }
    pipdev::RasterGrid G{x0, y0, dx, dy, empty ? 0 : width, empty ? 0 : height};
    hipError_t e = pipdev::launch_raster(V, n, G, labels, status, radial, ctx->early_exit, blocks,
                                         stream);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return PIP_OK;
}


// ---------------------------------------------------------------------------
// batched
// ---------------------------------------------------------------------------
size_t pip_voronoi_batched_workspace_bytes(int32_t P, int64_t total_vertices,
                                           int64_t total_points) {
    if (P < 0 || total_vertices < 0 || total_points < 0) return 0;
    pipdev::BatchedLayout L;
    return pipdev::batched_workspace_layout(P, total_vertices, total_points, &L);
}

}  // extern "C"

namespace {

pip_status check_batched(pip_ctx ctx, int32_t P, const int64_t* vtx_off, const double* V,
                         int64_t total_vertices, const int64_t* pt_off, const float* Q,
                         int64_t total_points, const int64_t* lbl_word_off, uint32_t* labels,
                         int32_t* status) {
    if (!ctx) return fail(PIP_EINVAL, "ctx is NULL");
    if (P < 0) return fail(PIP_EINVAL, "P = %d is negative", (int)P);
    if (total_vertices < 0 || total_points < 0)
        return fail(PIP_EINVAL, "total_vertices / total_points must be >= 0");
    if (P > 0 && (!vtx_off || !pt_off || !lbl_word_off))
        return fail(PIP_EINVAL, "vtx_off, pt_off and lbl_word_off must not be NULL");
    if (P > 0 && (!aligned(vtx_off, 8) || !aligned(pt_off, 8) || !aligned(lbl_word_off, 8)))
        return fail(PIP_EINVAL, "offset arrays must be 8-byte aligned");
    if (total_vertices > 0 && (!V || !aligned(V, 8))) return fail(PIP_EINVAL, "V is NULL or misaligned");
    if (total_points > 0 && (!Q || !aligned(Q, 8))) return fail(PIP_EINVAL, "Q is NULL or not 8-byte aligned");
    if (total_points > 0 && (!labels || !aligned(labels, 4)))
        return fail(PIP_EINVAL, "labels is NULL or not 4-byte aligned");
    if (status && !aligned(status, 4)) return fail(PIP_EINVAL, "status is not 4-byte aligned");
    if (total_points > (int64_t(1) << 46)) return fail(PIP_EUNSUPPORTED, "too many points");
    return PIP_OK;
}

pipdev::BatchedDev make_dev(int32_t P, const int64_t* vtx_off, const double* V,
                            int64_t total_vertices, const int64_t* pt_off, const float* Q,
                            int64_t total_points, const int64_t* lbl_word_off, uint32_t* labels,
                            int32_t* status, void* ws, int radial_min) {
    pipdev::BatchedLayout L;
    pipdev::batched_workspace_layout(P, total_vertices, total_points, &L);
    char* b = static_cast<char*>(ws);
    pipdev::BatchedDev D{};
    D.P = P;
    D.vtx_off = vtx_off;
    D.V = V;
    D.total_vertices = total_vertices;
    D.pt_off = pt_off;
    D.Q = Q;
    D.total_points = total_points;
    D.lbl_word_off = lbl_word_off;
    D.labels = labels;
    D.status = status;
    D.hdr = reinterpret_cast<pipdev::PolyHdr*>(b + L.hdr);
    D.coef = reinterpret_cast<float4*>(b + L.coef);
    D.gen = reinterpret_cast<double2*>(b + L.gen);
    D.chunk_cnt = reinterpret_cast<int64_t*>(b + L.chunk_cnt);
    D.chunk_off = reinterpret_cast<int64_t*>(b + L.chunk_off);
    D.desc = b + L.desc;
    D.misc = reinterpret_cast<int64_t*>(b + L.misc);
    D.max_chunks = L.max_chunks;
    D.radial = reinterpret_cast<float*>(b + L.radial);
    D.radial_min = radial_min;
    return D;
}

int batched_blocks_per_cu(pip_ctx ctx) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->batched_blocks_per_cu == 0) {
        int b = 0;
        if (pipdev::batched_max_blocks_per_cu(&b) != hipSuccess || b < 1) b = 1;
        ctx->batched_blocks_per_cu = b;
    }
    return ctx->batched_blocks_per_cu;
}

pip_status resolve_config(pip_ctx ctx, const pip_batched_config* in, pip_batched_config* out) {
    const int occ = batched_blocks_per_cu(ctx);
    pip_batched_config c;
    c.chunks_per_tile = 16;
    c.blocks_per_cu = occ;
    if (in) {
        if (in->chunks_per_tile < 1) return fail(PIP_EINVAL, "chunks_per_tile must be >= 1");
        if (in->blocks_per_cu < 1 || in->blocks_per_cu > 64)
            return fail(PIP_EINVAL, "blocks_per_cu must be in [1, 64]");
        c = *in;
    }
    *out = c;
    return PIP_OK;
}

pip_status launch_batched_cfg(pip_ctx ctx, const pipdev::BatchedDev& D,
                              const pip_batched_config& c, hipStream_t stream) {
    hipError_t e = pipdev::launch_batched(D, c.chunks_per_tile, c.blocks_per_cu * ctx->cu_count, stream);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return PIP_OK;
}

}  // namespace

extern "C" {

pip_status pip_voronoi_batched(pip_ctx ctx, int32_t P, const int64_t* vtx_off, const double* V,
                               int64_t total_vertices, const int64_t* pt_off, const float* Q,
                               int64_t total_points, const int64_t* lbl_word_off,
                               uint32_t* labels, int32_t* status, void* workspace,
                               size_t workspace_bytes, const pip_batched_config* config,
                               hipStream_t stream) {
    pip_status s = check_batched(ctx, P, vtx_off, V, total_vertices, pt_off, Q, total_points,
                                 lbl_word_off, labels, status);
    if (s != PIP_OK) return s;
    if (P == 0) return PIP_OK;
    const size_t need = pip_voronoi_batched_workspace_bytes(P, total_vertices, total_points);
    if (!workspace || workspace_bytes < need)
        return fail(PIP_EINVAL, "workspace of %zu bytes needed (got %zu)", need, workspace_bytes);
    if (!aligned(workspace, 256)) return fail(PIP_EINVAL, "workspace is not 256-byte aligned");
    pip_batched_config c;
    if ((s = resolve_config(ctx, config, &c)) != PIP_OK) return s;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    const pipdev::BatchedDev D = make_dev(P, vtx_off, V, total_vertices, pt_off, Q, total_points,
                                          lbl_word_off, labels, status, workspace,
                                          ctx->radial_min_edges);
    return launch_batched_cfg(ctx, D, c, stream);
}

pip_status pip_voronoi_batched_noalloc(pip_ctx ctx, int32_t P, const int64_t* vtx_off,
                                       const double* V, int64_t total_vertices,
                                       const int64_t* pt_off, const float* Q,
                                       int64_t total_points, const int64_t* lbl_word_off,
                                       uint32_t* labels, int32_t* status,
                                       const pip_batched_config* config, hipStream_t stream) {
    pip_status s = check_batched(ctx, P, vtx_off, V, total_vertices, pt_off, Q, total_points,
                                 lbl_word_off, labels, status);
    if (s != PIP_OK) return s;
    if (P == 0) return PIP_OK;
    const size_t need = pip_voronoi_batched_workspace_bytes(P, total_vertices, total_points);
    if (need > PIP_BATCHED_SCRATCH_BYTES)
        return fail(PIP_EUNSUPPORTED,
                    "the batch needs %zu workspace bytes, more than the %zu of the library's "
                    "scratch array; use pip_voronoi_batched with a workspace",
                    need, (size_t)PIP_BATCHED_SCRATCH_BYTES);
    if (!ctx->scratch)
        return hip_fail(ctx->scratch_err, "device address of the scratch array (at pip_create)");
    pip_batched_config c;
    if ((s = resolve_config(ctx, config, &c)) != PIP_OK) return s;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    const pipdev::BatchedDev D = make_dev(P, vtx_off, V, total_vertices, pt_off, Q, total_points,
                                          lbl_word_off, labels, status, ctx->scratch,
                                          ctx->radial_min_edges);
    return launch_batched_cfg(ctx, D, c, stream);
}

// ---------------------------------------------------------------------------
// non-convex polygons: union of convex pieces
// ---------------------------------------------------------------------------
size_t pip_voronoi_pieces_workspace_bytes(int32_t K, int64_t idx_count) {
    if (K < 1 || idx_count < 0) return 0;
    pipdev::PiecesLayout L;
    return pipdev::pieces_workspace_layout(K, idx_count, &L);
}

pip_status pip_voronoi_pieces(pip_ctx ctx, const double* V, int64_t n, int32_t K,
                              const int32_t* piece_off, const int32_t* piece_idx,
                              int64_t idx_count, const void* Q, pip_dtype qdt, int64_t m,
                              uint32_t* labels, int32_t* status, void* workspace,
                              size_t workspace_bytes, hipStream_t stream) {
    if (!ctx) return fail(PIP_EINVAL, "ctx is NULL");
    if (!V || !aligned(V, 8)) return fail(PIP_EINVAL, "V is NULL or not 8-byte aligned");
    if (n < 3 || n > (int64_t(1) << 30)) return fail(PIP_EINVAL, "n = %lld is out of range", (long long)n);
    if (K < 1) return fail(PIP_EINVAL, "K = %d: at least one piece", (int)K);
    if (idx_count < 0) return fail(PIP_EINVAL, "idx_count is negative");
    if (!piece_off || !aligned(piece_off, 4)) return fail(PIP_EINVAL, "piece_off is NULL or misaligned");
    if (idx_count > 0 && (!piece_idx || !aligned(piece_idx, 4)))
        return fail(PIP_EINVAL, "piece_idx is NULL or misaligned");
    pip_status s = check_points(Q, qdt, m);
    if (s != PIP_OK) return s;
    if (m > 0 && (!labels || !aligned(labels, 4))) return fail(PIP_EINVAL, "labels is NULL or misaligned");
    if (status && !aligned(status, 4)) return fail(PIP_EINVAL, "status is not 4-byte aligned");
    const size_t lds = pipdev::pieces_lds_bytes(K, idx_count);
    if (lds > PIP_PIECES_MAX_TABLE_BYTES)
        return fail(PIP_EUNSUPPORTED,
                    "%d pieces with %lld vertex entries need %zu bytes of piece tables "
                    "(limit %d): split the polygon", (int)K, (long long)idx_count, lds,
                    (int)PIP_PIECES_MAX_TABLE_BYTES);
    const size_t need = pip_voronoi_pieces_workspace_bytes(K, idx_count);
    if (!workspace || !aligned(workspace, 256) || workspace_bytes < need)
        return fail(PIP_EINVAL, "workspace of %zu bytes (256-byte aligned) needed, got %zu", need,
                    workspace_bytes);
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    int per_cu = 0;
    if (pipdev::pieces_max_blocks_per_cu((int)qdt, lds, &per_cu) != hipSuccess || per_cu < 1)
        per_cu = 1;
    pipdev::PiecesLaunch A;
    A.V = V;
    A.n = n;
    A.K = K;
    A.off = piece_off;
    A.idx = piece_idx;
    A.idx_count = idx_count;
    A.Q = Q;
    A.qdt = (int)qdt;
    A.m = m;
    A.labels = labels;
    A.status = status;
    A.ws = workspace;
    A.max_blocks = per_cu * ctx->cu_count;
    // recheck queue codes hold 2^23 chunks per wave
    const int64_t waves = 4 * (int64_t)A.max_blocks;
    if (((m + 511) / 512 + waves - 1) / waves >= (int64_t(1) << 23))
        return fail(PIP_EUNSUPPORTED, "m = %lld points is too large for one launch", (long long)m);
    hipError_t e = pipdev::launch_pieces(A, stream);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return PIP_OK;
}

pip_status pip_convex_decompose(const double* V, int32_t n, int32_t max_piece_vertices,
                                int32_t* piece_off, int32_t* piece_idx, int32_t* num_pieces,
                                int64_t* idx_count) {
    if (!V || !piece_off || !piece_idx || !num_pieces || !idx_count)
        return fail(PIP_EINVAL, "a pointer argument is NULL");
    if (n < 3 || n > (1 << 20)) return fail(PIP_EINVAL, "n = %d is out of range [3, 2^20]", (int)n);
    if (max_piece_vertices < 3 || max_piece_vertices > PIP_MAX_EDGES)
        return fail(PIP_EINVAL, "max_piece_vertices must lie in [3, %d]", PIP_MAX_EDGES);
    std::vector<int32_t> off, idx;
    const int r = pipdev::convex_decompose_host(V, n, max_piece_vertices, off, idx);
    if (r == 1) return fail(PIP_EINVAL, "non-finite vertex or zero area");
    if (r == 2) return fail(PIP_EINVAL, "the polygon is not simple (no ear left to cut)");
    if (r != 0 || off.size() > (size_t)n - 1 || idx.size() > 3 * (size_t)(n - 2))
        return fail(PIP_EINVAL, "decomposition failed");
    for (size_t i = 0; i < off.size(); ++i) piece_off[i] = off[i];
    for (size_t i = 0; i < idx.size(); ++i) piece_idx[i] = idx[i];
    *num_pieces = (int32_t)off.size() - 1;
    *idx_count = (int64_t)idx.size();
    return PIP_OK;
}

// ---------------------------------------------------------------------------
// plans: autotuned tile shape + captured hipGraph
// ---------------------------------------------------------------------------
void pip_plan_destroy(pip_plan p) {
    if (!p) return;
    DeviceGuard g(p->ctx->device);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    if (p->ws) (void)hipFree(p->ws);
    if (p->ref_labels) (void)hipFree(p->ref_labels);
    if (p->ref_counts) (void)hipFree(p->ref_counts);
    if (p->d_diff) (void)hipFree(p->d_diff);
    delete p;
}

pip_status pip_plan_create_allpairs(pip_ctx ctx, int32_t P, int32_t n, const double* V,
                                    const float* Q, int64_t m, uint32_t* labels, int32_t* counts,
                                    int32_t* status, pip_plan* out) {
    if (!out) return fail(PIP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctx) return fail(PIP_EINVAL, "ctx is NULL");
    if (P < 1) return fail(PIP_EINVAL, "a plan needs P >= 1");
    if (n < 3) return fail(PIP_EINVAL, "n = %d: a polygon needs at least 3 vertices", (int)n);
    if (n > PIP_MAX_EDGES) return fail(PIP_EUNSUPPORTED, "n = %d exceeds %d", (int)n, PIP_MAX_EDGES);
    if (!V || !aligned(V, 8)) return fail(PIP_EINVAL, "V is NULL or misaligned");
    pip_status s = check_points(Q, PIP_F32, m);
    if (s != PIP_OK) return s;
    if (m > 0 && (!labels || !aligned(labels, 4)))
        return fail(PIP_EINVAL, "labels is NULL or not 4-byte aligned");
    if (!counts || !aligned(counts, 4)) return fail(PIP_EINVAL, "counts is NULL or misaligned");
    if (status && !aligned(status, 4)) return fail(PIP_EINVAL, "status is not 4-byte aligned");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    pip_plan p = new (std::nothrow) pip_plan_s();
    if (!p) return fail(PIP_ENOMEM, "out of host memory");
    p->ctx = ctx;
    p->kind = 1;
    p->A = AllpairsArgs{P, n, V, Q, m, labels, counts, status};
    p->acfg.cull = ctx->allpairs_cull;
    p->acfg.pair = ctx->allpairs_pair;
    p->label_words = (int64_t)P * ((m + 31) / 32);
    p->ws_bytes = pip_voronoi_allpairs_workspace_bytes(P, n);
    hipError_t e = hipMalloc(&p->ws, p->ws_bytes);
    if (e != hipSuccess) {
        pip_plan_destroy(p);
        return fail(PIP_ENOMEM, "hipMalloc of %zu workspace bytes failed", p->ws_bytes);
    }
    e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        pip_plan_destroy(p);
        return hip_fail(e, "hipStreamCreateWithFlags");
    }
    *out = p;
    return PIP_OK;
}

pip_status pip_plan_create_batched(pip_ctx ctx, int32_t P, const int64_t* vtx_off,
                                   const double* V, int64_t total_vertices,
                                   const int64_t* pt_off, const float* Q, int64_t total_points,
                                   const int64_t* lbl_word_off, uint32_t* labels,
                                   int32_t* status, pip_plan* out) {
    if (!out) return fail(PIP_EINVAL, "out is NULL");
    *out = nullptr;
    pip_status s = check_batched(ctx, P, vtx_off, V, total_vertices, pt_off, Q, total_points,
                                 lbl_word_off, labels, status);
    if (s != PIP_OK) return s;
    if (P < 1) return fail(PIP_EINVAL, "a plan needs P >= 1");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    pip_plan p = new (std::nothrow) pip_plan_s();
    if (!p) return fail(PIP_ENOMEM, "out of host memory");
    p->ctx = ctx;
    p->ws_bytes = pip_voronoi_batched_workspace_bytes(P, total_vertices, total_points);
    hipError_t e = hipMalloc(&p->ws, p->ws_bytes);
    if (e != hipSuccess) {
        pip_plan_destroy(p);
        return fail(PIP_ENOMEM, "hipMalloc of %zu workspace bytes failed", p->ws_bytes);
    }
    int64_t words = 0;
    e = hipMemcpy(&words, lbl_word_off + P, sizeof(int64_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        pip_plan_destroy(p);
        return hip_fail(e, "reading lbl_word_off[P]");
    }
    if (words < 0 || words > total_points / 32 + P + 1) {
        pip_plan_destroy(p);
        return fail(PIP_EINVAL, "lbl_word_off[P] = %lld is inconsistent with the point count",
                    (long long)words);
    }
    p->label_words = words;
    e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        pip_plan_destroy(p);
        return hip_fail(e, "hipStreamCreateWithFlags");
    }
    p->D = make_dev(P, vtx_off, V, total_vertices, pt_off, Q, total_points, lbl_word_off, labels,
                    status, p->ws, ctx->radial_min_edges);
    resolve_config(ctx, nullptr, &p->cfg);
    *out = p;
    return PIP_OK;
}

}  // extern "C"

namespace {

// One launch of the plan's work with its current configuration.
hipError_t launch_plan_once(pip_plan p, hipStream_t stream) {
    const CostArgs& C = p->Cst;
    switch (p->kind) {
        case 1:
            return pipdev::launch_allpairs(p->A.P, p->A.n, p->A.V, p->A.Q, p->A.m, p->A.labels,
                                           p->A.counts, p->A.status, p->ws, p->acfg.cull,
                                           p->acfg.pair, stream);
        case 2:
            return pipdev::launch_cost(false, C.F, C.n, C.pose, C.K, C.Q, C.m, nullptr, C.cost,
                                       nullptr, nullptr, nullptr, p->ws, p->acfg.cull, p->acfg.pair,
                                       stream);
        case 3:
            return pipdev::launch_cost(true, C.F, C.n, C.pose, C.K, C.Q, C.m, C.grad_cost, nullptr,
                                       C.grad_pose, C.grad_F, C.residual, p->ws, p->acfg.cull,
                                       p->acfg.pair, stream);
        default:
            return pipdev::launch_batched(p->D, p->cfg.chunks_per_tile,
                                          p->cfg.blocks_per_cu * p->ctx->cu_count, stream);
    }
}

pip_status capture_plan(pip_plan p) {
    if (p->exec) {
        (void)hipGraphExecDestroy(p->exec);
        p->exec = nullptr;
    }
    if (p->graph) {
        (void)hipGraphDestroy(p->graph);
        p->graph = nullptr;
    }
    hipError_t e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t le = launch_plan_once(p, p->cap);
    e = hipStreamEndCapture(p->cap, &p->graph);
    if (le != hipSuccess) return hip_fail(le, "kernel launch during capture");
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    return PIP_OK;
}

}  // namespace

extern "C" {

namespace {

// The output words a variant must reproduce: (pointer, 32-bit words) pairs.
int plan_outputs(pip_plan p, uint32_t** ptr, int64_t* words) {
    const CostArgs& C = p->Cst;
    switch (p->kind) {
        case 1:
            ptr[0] = p->A.labels;
            words[0] = p->label_words;
            ptr[1] = reinterpret_cast<uint32_t*>(p->A.counts);
            words[1] = p->A.P;
            return 2;
        case 2:
            ptr[0] = reinterpret_cast<uint32_t*>(C.cost);
            words[0] = C.K;
            return 1;
        case 3:
            ptr[0] = reinterpret_cast<uint32_t*>(C.grad_pose);
            words[0] = 3 * C.K;
            ptr[1] = reinterpret_cast<uint32_t*>(C.grad_F);
            words[1] = 2 * (int64_t)C.n;
            return 2;
        default:
            return 0;
    }
}

// All pairs and cost: the exact variants (all pairs: dense, culled, paired,
// both; cost: culled or not, pairing as configured); each must reproduce the
// first one's outputs word for word.
pip_status autotune_variants(pip_plan p, int32_t reps, hipStream_t stream) {
    hipError_t e;
    uint32_t* out[2] = {nullptr, nullptr};
    int64_t words[2] = {0, 0};
    const int nout = plan_outputs(p, out, words);
    if (!p->ref_labels && words[0] > 0 &&
        (e = hipMalloc(&p->ref_labels, sizeof(uint32_t) * words[0])) != hipSuccess)
        return fail(PIP_ENOMEM, "hipMalloc of the reference outputs failed");
    if (nout > 1 && !p->ref_counts && words[1] > 0 &&
        (e = hipMalloc(&p->ref_counts, sizeof(uint32_t) * words[1])) != hipSuccess)
        return fail(PIP_ENOMEM, "hipMalloc of the reference outputs failed");
    if (!p->d_diff && (e = hipMalloc(&p->d_diff, sizeof(unsigned long long))) != hipSuccess)
        return fail(PIP_ENOMEM, "hipMalloc failed");
    hipEvent_t a, b;
    if ((e = hipEventCreate(&a)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&b)) != hipSuccess) {
        (void)hipEventDestroy(a);
        return hip_fail(e, "hipEventCreate");
    }
    auto run = [&](const pip_variant_config& c) {
        const pip_variant_config keep = p->acfg;
        p->acfg = c;
        const hipError_t r = launch_plan_once(p, stream);
        p->acfg = keep;
        return r;
    };
    uint32_t* ref[2] = {p->ref_labels, p->ref_counts};
    auto differ = [&](const uint32_t* ref, const uint32_t* cur, int64_t words,
                      unsigned long long* out) -> hipError_t {
        hipError_t r = pipdev::launch_count_diff(ref, cur, words, p->d_diff, stream);
        if (r == hipSuccess) r = hipMemcpyAsync(out, p->d_diff, sizeof *out, hipMemcpyDeviceToHost, stream);
        if (r == hipSuccess) r = hipStreamSynchronize(stream);
        return r;
    };
    pip_status st = PIP_OK;
    float best = -1.f;
    pip_variant_config best_cfg = p->acfg;
    // all pairs: (cull, pair) in {0,1}^2; cost: cull in {0,1}, pair as configured
    const int nvar = p->kind == 1 ? 4 : 2;
    for (int v = 0; v < nvar && st == PIP_OK; ++v) {
        pip_variant_config c;
        c.cull = v & 1;
        c.pair = p->kind == 1 ? v >> 1 : p->acfg.pair;
        if ((e = run(c)) != hipSuccess) { st = hip_fail(e, "kernel launch"); break; }  // warm-up
        if (v == 0) {
            for (int o = 0; o < nout && e == hipSuccess; ++o)
                if (words[o] > 0)
                    e = hipMemcpyAsync(ref[o], out[o], sizeof(uint32_t) * words[o],
                                       hipMemcpyDeviceToDevice, stream);
            if (e != hipSuccess) { st = hip_fail(e, "hipMemcpyAsync"); break; }
        } else {
            unsigned long long d[2] = {0, 0};
            for (int o = 0; o < nout && e == hipSuccess; ++o)
                if (words[o] > 0) e = differ(ref[o], out[o], words[o], &d[o]);
            if (e != hipSuccess) { st = hip_fail(e, "output comparison"); break; }
            if (d[0] != 0 || d[1] != 0) {
                st = fail(PIP_EHIP, "autotune: variant (cull %d, pair %d) changed %llu + %llu "
                          "output words", c.cull, c.pair, d[0], d[1]);
                break;
            }
        }
        (void)hipEventRecord(a, stream);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = run(c);
        (void)hipEventRecord(b, stream);
        if (e != hipSuccess) { st = hip_fail(e, "kernel launch"); break; }
        if ((e = hipEventSynchronize(b)) != hipSuccess) { st = hip_fail(e, "hipEventSynchronize"); break; }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        ms /= reps;
        if (best < 0.f || ms < best) {
            best = ms;
            best_cfg = c;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st != PIP_OK) return st;
    p->acfg = best_cfg;
    p->best_ms = best;
    return capture_plan(p);
}

}  // namespace

pip_status pip_plan_autotune(pip_plan p, int32_t reps, hipStream_t stream) {
    if (!p) return fail(PIP_EINVAL, "plan is NULL");
    if (reps < 1) reps = 3;
    if (p->kind != 0) {
        DeviceGuard g(p->ctx->device);
        if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
        return autotune_variants(p, reps, stream);
    }
    DeviceGuard g(p->ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipError_t e;
    if (!p->ref_labels && p->label_words > 0) {
        if ((e = hipMalloc(&p->ref_labels, sizeof(uint32_t) * p->label_words)) != hipSuccess)
            return fail(PIP_ENOMEM, "hipMalloc of the reference labels failed");
    }
    if (!p->d_diff && (e = hipMalloc(&p->d_diff, sizeof(unsigned long long))) != hipSuccess)
        return fail(PIP_ENOMEM, "hipMalloc failed");
    const int occ = batched_blocks_per_cu(p->ctx);
    const int tiles[] = {1, 4, 16, 64, 1 << 30};  // 1 << 30: one contiguous range per wave
    int bpcs[3] = {occ, occ > 2 ? occ - 2 : occ, occ > 1 ? occ / 2 : occ};
    hipEvent_t a, b;
    if ((e = hipEventCreate(&a)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&b)) != hipSuccess) {
        (void)hipEventDestroy(a);
        return hip_fail(e, "hipEventCreate");
    }
    pip_status st = PIP_OK;
    float best = -1.f;
    pip_batched_config best_cfg = p->cfg;
    bool have_ref = false;
    for (int ti = 0; ti < 5 && st == PIP_OK; ++ti) {
        for (int bi = 0; bi < 3 && st == PIP_OK; ++bi) {
            if (bi > 0 && bpcs[bi] == bpcs[bi - 1]) continue;
            pip_batched_config c;
            c.chunks_per_tile = tiles[ti];
            c.blocks_per_cu = bpcs[bi];
            if ((st = launch_batched_cfg(p->ctx, p->D, c, stream)) != PIP_OK) break;  // warm-up
            if (p->label_words > 0) {
                if (!have_ref) {
                    e = hipMemcpyAsync(p->ref_labels, p->D.labels, sizeof(uint32_t) * p->label_words,
                                       hipMemcpyDeviceToDevice, stream);
                    if (e != hipSuccess) { st = hip_fail(e, "hipMemcpyAsync"); break; }
                    have_ref = true;
                } else {
                    unsigned long long diff = 0;
                    e = pipdev::launch_count_diff(p->ref_labels, p->D.labels, p->label_words,
                                                  p->d_diff, stream);
                    if (e == hipSuccess)
                        e = hipMemcpyAsync(&diff, p->d_diff, sizeof diff, hipMemcpyDeviceToHost, stream);
                    if (e == hipSuccess) e = hipStreamSynchronize(stream);
                    if (e != hipSuccess) { st = hip_fail(e, "label comparison"); break; }
                    if (diff != 0) {
                        st = fail(PIP_EHIP, "autotune: tile shape (%d chunks, %d blocks/CU) changed %llu label words",
                                  c.chunks_per_tile, c.blocks_per_cu, diff);
                        break;
                    }
                }
            }
            (void)hipEventRecord(a, stream);
            for (int r = 0; r < reps; ++r)
                if ((st = launch_batched_cfg(p->ctx, p->D, c, stream)) != PIP_OK) break;
            (void)hipEventRecord(b, stream);
            if ((e = hipEventSynchronize(b)) != hipSuccess) { st = hip_fail(e, "hipEventSynchronize"); break; }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, a, b);
            ms /= reps;
            if (best < 0.f || ms < best) {
                best = ms;
                best_cfg = c;
            }
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st != PIP_OK) return st;
    p->cfg = best_cfg;
    p->best_ms = best;
    return capture_plan(p);
}

pip_status pip_plan_launch(pip_plan p, hipStream_t stream) {
    if (!p) return fail(PIP_EINVAL, "plan is NULL");
    DeviceGuard g(p->ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    if (!p->exec) {
        pip_status s = capture_plan(p);
        if (s != PIP_OK) return s;
    }
    hipError_t e = hipGraphLaunch(p->exec, stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return PIP_OK;
}

pip_status pip_plan_variant(pip_plan p, pip_variant_config* cfg, float* best_ms) {
    if (!p || p->kind == 0) return fail(PIP_EINVAL, "plan is NULL or a batched plan");
    if (cfg) *cfg = p->acfg;
    if (best_ms) *best_ms = p->best_ms;
    return PIP_OK;
}

pip_status pip_plan_set_variant(pip_plan p, const pip_variant_config* cfg) {
    if (!p || p->kind == 0 || !cfg) return fail(PIP_EINVAL, "plan is NULL or batched, or cfg is NULL");
    if ((cfg->cull != 0 && cfg->cull != 1) || (cfg->pair != 0 && cfg->pair != 1))
        return fail(PIP_EINVAL, "cull and pair must be 0 or 1");
    DeviceGuard g(p->ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    p->acfg = *cfg;
    return capture_plan(p);
}

pip_status pip_plan_config(pip_plan p, pip_batched_config* cfg, float* best_ms) {
    if (!p) return fail(PIP_EINVAL, "plan is NULL");
    if (p->kind != 0) return fail(PIP_EINVAL, "not a batched plan");
    if (cfg) *cfg = p->cfg;
    if (best_ms) *best_ms = p->best_ms;
    return PIP_OK;
}

pip_status pip_plan_set_config(pip_plan p, const pip_batched_config* cfg) {
    if (!p || !cfg) return fail(PIP_EINVAL, "plan or cfg is NULL");
    if (p->kind != 0) return fail(PIP_EINVAL, "not a batched plan");
    pip_batched_config c;
    pip_status s = resolve_config(p->ctx, cfg, &c);
    if (s != PIP_OK) return s;
    DeviceGuard g(p->ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    p->cfg = c;
    return capture_plan(p);
}


// ---------------------------------------------------------------------------
// poses and all pairs
// ---------------------------------------------------------------------------
pip_status pip_poses_to_polygons(pip_ctx ctx, const double* footprint, int32_t n, const float* pose,
                                 const double* cs, int64_t K, double* V_out, hipStream_t stream) {
    if (!ctx) return fail(PIP_EINVAL, "ctx is NULL");
    pip_status s = check_polygon(footprint, n);
    if (s != PIP_OK) return s;
    if (K < 0) return fail(PIP_EINVAL, "K = %lld is negative", (long long)K);
    if (K > 0 && (!pose || !aligned(pose, 4))) return fail(PIP_EINVAL, "pose is NULL or misaligned");
    if (K > 0 && (!cs || !aligned(cs, 8))) return fail(PIP_EINVAL, "cs is NULL or misaligned");
    if (K > 0 && (!V_out || !aligned(V_out, 8))) return fail(PIP_EINVAL, "V_out is NULL or misaligned");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipError_t e = pipdev::launch_poses_to_polygons(footprint, n, pose, cs, K, V_out, stream);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return PIP_OK;
}

size_t pip_voronoi_allpairs_workspace_bytes(int32_t P, int32_t n) {
    if (P < 0 || n < 3 || n > PIP_MAX_EDGES) return 0;
    pipdev::AllpairsLayout L;
    return pipdev::allpairs_workspace_layout(P, n, &L);
}

pip_status pip_voronoi_allpairs(pip_ctx ctx, int32_t P, int32_t n, const double* V, const float* Q,
                                int64_t m, uint32_t* labels, int32_t* counts, int32_t* status,
                                void* workspace, size_t workspace_bytes, hipStream_t stream) {
    if (!ctx) return fail(PIP_EINVAL, "ctx is NULL");
    if (P < 0) return fail(PIP_EINVAL, "P = %d is negative", (int)P);
    if (n < 3) return fail(PIP_EINVAL, "n = %d: a polygon needs at least 3 vertices", (int)n);
    if (n > PIP_MAX_EDGES) return fail(PIP_EUNSUPPORTED, "n = %d exceeds %d", (int)n, PIP_MAX_EDGES);
    if (P > 0 && (!V || !aligned(V, 8))) return fail(PIP_EINVAL, "V is NULL or misaligned");
    pip_status s = check_points(Q, PIP_F32, m);
    if (s != PIP_OK) return s;
    if (P > 0 && m > 0 && (!labels || !aligned(labels, 4)))
        return fail(PIP_EINVAL, "labels is NULL or not 4-byte aligned");
    if (counts && !aligned(counts, 4)) return fail(PIP_EINVAL, "counts is not 4-byte aligned");
    if (status && !aligned(status, 4)) return fail(PIP_EINVAL, "status is not 4-byte aligned");
    if (P == 0) return PIP_OK;
    const size_t need = pip_voronoi_allpairs_workspace_bytes(P, n);
    if (!workspace || workspace_bytes < need)
        return fail(PIP_EINVAL, "workspace of %zu bytes needed (got %zu)", need, workspace_bytes);
    if (!aligned(workspace, 256)) return fail(PIP_EINVAL, "workspace is not 256-byte aligned");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipError_t e = pipdev::launch_allpairs(P, n, V, Q, m, labels, counts, status, workspace,
                                           ctx->allpairs_cull,
                                           ctx->allpairs_pair, stream);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return PIP_OK;
}


size_t pip_voronoi_allpairs_csr_workspace_bytes(int32_t P, int64_t total_vertices) {
    if (P < 0 || total_vertices < 0) return 0;
    pipdev::AllpairsLayout L;
    return pipdev::allpairs_csr_workspace_layout(P, total_vertices, &L);
}

pip_status pip_voronoi_allpairs_csr(pip_ctx ctx, int32_t P, const int64_t* vtx_off,
                                    const double* V, int64_t total_vertices, const float* Q,
                                    int64_t m, uint32_t* labels, int32_t* counts,
                                    int32_t* status, void* workspace, size_t workspace_bytes,
                                    hipStream_t stream) {
    if (!ctx) return fail(PIP_EINVAL, "ctx is NULL");
    if (P < 0) return fail(PIP_EINVAL, "P = %d is negative", (int)P);
    if (total_vertices < 0) return fail(PIP_EINVAL, "total_vertices is negative");
    if (total_vertices + 3 * (int64_t)P >= (int64_t(1) << 31))
        return fail(PIP_EUNSUPPORTED, "total_vertices + 3 P must stay below 2^31");
    if (P > 0 && (!vtx_off || !aligned(vtx_off, 8)))
        return fail(PIP_EINVAL, "vtx_off is NULL or not 8-byte aligned");
    if (total_vertices > 0 && (!V || !aligned(V, 8))) return fail(PIP_EINVAL, "V is NULL or misaligned");
    pip_status s = check_points(Q, PIP_F32, m);
    if (s != PIP_OK) return s;
    if (P > 0 && m > 0 && (!labels || !aligned(labels, 4)))
        return fail(PIP_EINVAL, "labels is NULL or not 4-byte aligned");
    if (counts && !aligned(counts, 4)) return fail(PIP_EINVAL, "counts is not 4-byte aligned");
    if (status && !aligned(status, 4)) return fail(PIP_EINVAL, "status is not 4-byte aligned");
    if (P == 0) return PIP_OK;
    const size_t need = pip_voronoi_allpairs_csr_workspace_bytes(P, total_vertices);
    if (!workspace || workspace_bytes < need)
        return fail(PIP_EINVAL, "workspace of %zu bytes needed (got %zu)", need, workspace_bytes);
    if (!aligned(workspace, 256)) return fail(PIP_EINVAL, "workspace is not 256-byte aligned");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipError_t e = pipdev::launch_allpairs_csr(P, vtx_off, V, total_vertices, Q, m, labels, counts,
                                               status, workspace, ctx->allpairs_cull,
                                               ctx->allpairs_pair, stream);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return PIP_OK;
}

// ---------------------------------------------------------------------------
// differentiable collision cost
// ---------------------------------------------------------------------------
size_t pip_cost_workspace_bytes(int32_t n, int64_t K, int64_t m) {
    if (n < 3 || n > pipdev::cost_max_edges() || K < 0 || m < 0) return 0;
    pipdev::CostLayout L;
    return pipdev::cost_workspace_layout(n, K, m, &L);
}

}  // extern "C"

namespace {
pip_status check_cost_args(pip_ctx ctx, const float* F, int32_t n, const float* pose, int64_t K,
                           const float* Q, int64_t m) {
    if (!ctx) return fail(PIP_EINVAL, "ctx is NULL");
    if (!F || !aligned(F, 4)) return fail(PIP_EINVAL, "footprint is NULL or misaligned");
    if (n < 3) return fail(PIP_EINVAL, "n = %d: a polygon needs at least 3 vertices", (int)n);
    if (n > pipdev::cost_max_edges())
        return fail(PIP_EUNSUPPORTED, "n = %d exceeds the cost path's limit of %d edges", (int)n,
                    pipdev::cost_max_edges());
    if (K < 0 || m < 0) return fail(PIP_EINVAL, "K and m must be >= 0");
    if (K > 0 && (!pose || !aligned(pose, 4))) return fail(PIP_EINVAL, "pose is NULL or misaligned");
    if (m > 0 && (!Q || !aligned(Q, 8))) return fail(PIP_EINVAL, "Q is NULL or not 8-byte aligned");
    if (K > ((int64_t)1 << 31) || m > ((int64_t)1 << 40)) return fail(PIP_EUNSUPPORTED, "too large");
    return PIP_OK;
}

pip_status check_cost(pip_ctx ctx, const float* F, int32_t n, const float* pose, int64_t K,
                      const float* Q, int64_t m, void* ws, size_t ws_bytes) {
    pip_status s = check_cost_args(ctx, F, n, pose, K, Q, m);
    if (s != PIP_OK) return s;
    const size_t need = pip_cost_workspace_bytes(n, K, m);
    if (!ws || ws_bytes < need)
        return fail(PIP_EINVAL, "workspace of %zu bytes needed (got %zu)", need, ws_bytes);
    if (!aligned(ws, 256)) return fail(PIP_EINVAL, "workspace is not 256-byte aligned");
    return PIP_OK;
}
}  // namespace

extern "C" {

pip_status pip_cost_fwd(pip_ctx ctx, const float* footprint, int32_t n, const float* pose, int64_t K,
                        const float* Q, int64_t m, float* cost, void* workspace,
                        size_t workspace_bytes, hipStream_t stream) {
    pip_status s = check_cost(ctx, footprint, n, pose, K, Q, m, workspace, workspace_bytes);
    if (s != PIP_OK) return s;
    if (K > 0 && (!cost || !aligned(cost, 4))) return fail(PIP_EINVAL, "cost is NULL or misaligned");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipError_t e = pipdev::launch_cost(false, footprint, n, pose, K, Q, m, nullptr, cost, nullptr,
                                       nullptr, nullptr, workspace, ctx->cost_cull,
                                       ctx->cost_pair, stream);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return PIP_OK;
}

pip_status pip_cost_bwd(pip_ctx ctx, const float* footprint, int32_t n, const float* pose, int64_t K,
                        const float* Q, int64_t m, const float* grad_cost, float* grad_pose,
                        float* grad_footprint, float* residual, void* workspace,
                        size_t workspace_bytes, hipStream_t stream) {
    pip_status s = check_cost(ctx, footprint, n, pose, K, Q, m, workspace, workspace_bytes);
    if (s != PIP_OK) return s;
    if (K > 0 && (!grad_cost || !aligned(grad_cost, 4)))
        return fail(PIP_EINVAL, "grad_cost is NULL or misaligned");
    if (K > 0 && (!grad_pose || !aligned(grad_pose, 4)))
        return fail(PIP_EINVAL, "grad_pose is NULL or misaligned");
    if (!grad_footprint || !aligned(grad_footprint, 4))
        return fail(PIP_EINVAL, "grad_footprint is NULL or misaligned");
    if (residual && !aligned(residual, 4)) return fail(PIP_EINVAL, "residual is misaligned");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipError_t e = pipdev::launch_cost(true, footprint, n, pose, K, Q, m, grad_cost, nullptr, grad_pose,
                                       grad_footprint, residual, workspace, ctx->cost_cull,
                                       ctx->cost_pair, stream);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return PIP_OK;
}


pip_status pip_plan_create_cost(pip_ctx ctx, int32_t backward, const float* footprint, int32_t n,
                                const float* pose, int64_t K, const float* Q, int64_t m, float* cost,
                                const float* grad_cost, float* grad_pose, float* grad_footprint,
                                float* residual, pip_plan* out) {
    if (!out) return fail(PIP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctx) return fail(PIP_EINVAL, "ctx is NULL");
    if (K < 1) return fail(PIP_EINVAL, "a plan needs K >= 1");
    pip_status s = check_cost_args(ctx, footprint, n, pose, K, Q, m);
    if (s != PIP_OK) return s;
    const size_t need = pip_cost_workspace_bytes(n, K, m);
    if (!backward && (!cost || !aligned(cost, 4))) return fail(PIP_EINVAL, "cost is NULL or misaligned");
    if (backward) {
        if (!grad_cost || !aligned(grad_cost, 4)) return fail(PIP_EINVAL, "grad_cost is NULL or misaligned");
        if (!grad_pose || !aligned(grad_pose, 4)) return fail(PIP_EINVAL, "grad_pose is NULL or misaligned");
        if (!grad_footprint || !aligned(grad_footprint, 4))
            return fail(PIP_EINVAL, "grad_footprint is NULL or misaligned");
        if (residual && !aligned(residual, 4)) return fail(PIP_EINVAL, "residual is misaligned");
    }
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    pip_plan p = new (std::nothrow) pip_plan_s();
    if (!p) return fail(PIP_ENOMEM, "out of host memory");
    p->ctx = ctx;
    p->kind = backward ? 3 : 2;
    p->Cst = CostArgs{footprint, n, pose, K, Q, m, cost, grad_cost, grad_pose, grad_footprint, residual};
    p->acfg.cull = ctx->cost_cull;
    p->acfg.pair = ctx->cost_pair;
    p->ws_bytes = need;
    hipError_t e = hipMalloc(&p->ws, p->ws_bytes);
    if (e != hipSuccess) {
        pip_plan_destroy(p);
        return fail(PIP_ENOMEM, "hipMalloc of %zu workspace bytes failed", p->ws_bytes);
    }
    e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        pip_plan_destroy(p);
        return hip_fail(e, "hipStreamCreateWithFlags");
    }
    *out = p;
    return PIP_OK;
}


// ---------------------------------------------------------------------------
// point location index
// ---------------------------------------------------------------------------
void pip_index_destroy(pip_index x) {
    if (!x) return;
    DeviceGuard g(x->ctx->device);
    if (x->mem) (void)hipFree(x->mem);
    if (x->list_mem) (void)hipFree(x->list_mem);
    delete x;
}

pip_status pip_index_create(pip_ctx ctx, int32_t P, const int64_t* vtx_off, const double* V,
                            int64_t total_vertices, int64_t cells, int32_t* status,
                            hipStream_t stream, pip_index* out) {
    if (!out) return fail(PIP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctx) return fail(PIP_EINVAL, "ctx is NULL");
    if (P < 0) return fail(PIP_EINVAL, "P = %d is negative", (int)P);
    if (!vtx_off || !aligned(vtx_off, 8)) return fail(PIP_EINVAL, "vtx_off is NULL or misaligned");
    if (total_vertices < 0) return fail(PIP_EINVAL, "total_vertices is negative");
    if (total_vertices > 0 && (!V || !aligned(V, 8))) return fail(PIP_EINVAL, "V is NULL or misaligned");
    if (status && !aligned(status, 4)) return fail(PIP_EINVAL, "status is not 4-byte aligned");
    if (cells < 0 || cells > (int64_t(1) << 24))
        return fail(PIP_EINVAL, "cells = %lld must be in [0, 2^24]", (long long)cells);
    if (cells == 0) cells = P < 1 ? 1 : (P > (1 << 24) ? (1 << 24) : P);
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    // the caller's offsets must end at total_vertices
    int64_t last = -1;
    hipError_t e = hipMemcpy(&last, vtx_off + P, sizeof(int64_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "reading vtx_off[P]");
    if (last != total_vertices)
        return fail(PIP_EINVAL, "vtx_off[P] = %lld differs from total_vertices = %lld",
                    (long long)last, (long long)total_vertices);
    if (total_vertices + 5 * (int64_t)P >= (int64_t(1) << 31))
        return fail(PIP_EUNSUPPORTED, "%lld vertices in %d polygons exceed the 32-bit record offsets",
                    (long long)total_vertices, (int)P);
    pip_index x = new (std::nothrow) pip_index_s();
    if (!x) return fail(PIP_ENOMEM, "out of host memory");
    x->ctx = ctx;
    x->P = P;
    x->cells = cells;
    auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
    const size_t o_rec = 0;
    const size_t o_qrec = up(o_rec + sizeof(pipdev::LocRec) * (size_t)(P > 0 ? P : 1));
    const size_t o_gen = up(o_qrec + 16 * (size_t)(total_vertices + 5 * (int64_t)P + 1));
    const size_t o_grid = up(o_gen + 16 * (size_t)(total_vertices + P + 1));
    const size_t o_flag = up(o_grid + sizeof(pipdev::LocGrid));
    const size_t o_total = up(o_flag + 8);
    const size_t o_cnt = up(o_total + 8);
    const size_t o_off = up(o_cnt + 4 * (size_t)(cells + 1));
    const size_t o_end = up(o_off + 4 * (size_t)(cells + 2));
    char* b = nullptr;
    if ((e = hipMalloc(&x->mem, o_end)) != hipSuccess) {
        pip_index_destroy(x);
        return fail(PIP_ENOMEM, "hipMalloc of %zu index bytes failed", o_end);
    }
    b = static_cast<char*>(x->mem);
    x->rec = reinterpret_cast<pipdev::LocRec*>(b + o_rec);
    x->qrec = reinterpret_cast<float4*>(b + o_qrec);
    x->gen = reinterpret_cast<double2*>(b + o_gen);
    x->grid = reinterpret_cast<pipdev::LocGrid*>(b + o_grid);
    int32_t* flag = reinterpret_cast<int32_t*>(b + o_flag);
    auto* total = reinterpret_cast<unsigned long long*>(b + o_total);
    int32_t* cnt = reinterpret_cast<int32_t*>(b + o_cnt);
    x->cell_off = reinterpret_cast<int32_t*>(b + o_off);
    e = pipdev::index_prepare(P, vtx_off, V, x->rec, x->qrec, x->gen, status, flag, stream);
    if (e == hipSuccess) e = pipdev::index_grid(P, x->rec, cells, x->grid, cnt, total, stream);
    int32_t hflag = 0;
    unsigned long long htotal = 0;
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = hipMemcpy(&hflag, flag, 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&htotal, total, 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        pip_index_destroy(x);
        return hip_fail(e, "building the index");
    }
    if (hflag) {
        pip_index_destroy(x);
        return fail(PIP_EUNSUPPORTED, "a polygon has more than %d vertices", PIP_MAX_EDGES);
    }
    {  // super-cells for binned queries, about square in cells: at most 256 while
       // sf <= 32 (the binned kernel's in-tile sort takes up to 32 x 32 cells;
       // fewer, larger bins give longer write runs in the scatter pass:
       // 3.14 -> 3.01 ms for 2^26 points against 98,317 cells), then at most
       // 1024
        pipdev::LocGrid hg;
        if ((e = hipMemcpy(&hg, x->grid, sizeof(hg), hipMemcpyDeviceToHost)) != hipSuccess) {
            pip_index_destroy(x);
            return hip_fail(e, "reading the grid");
        }
        int sf = 1;
        auto bins = [&](int f) { return (int64_t)((hg.gx + f - 1) / f) * ((hg.gy + f - 1) / f); };
        while (sf < 32 && bins(sf) > 256) ++sf;
        while (bins(sf) > 1024) ++sf;
        x->sf = sf;
        x->sgx = (hg.gx + sf - 1) / sf;
        x->nbins = x->sgx * ((hg.gy + sf - 1) / sf);
    }
    if (htotal >= (1ull << 31)) {
        pip_index_destroy(x);
        return fail(PIP_EUNSUPPORTED, "%llu cell entries: use fewer cells", htotal);
    }
    x->entries = (int64_t)htotal;
    if ((e = hipMalloc(&x->list_mem, sizeof(pipdev::LocEntry) * (size_t)(htotal > 0 ? htotal : 1))) !=
        hipSuccess) {
        pip_index_destroy(x);
        return fail(PIP_ENOMEM, "hipMalloc of the cell lists failed");
    }
    x->list = static_cast<pipdev::LocEntry*>(x->list_mem);
    e = pipdev::index_fill(P, x->rec, x->grid, cells, cnt, x->cell_off, x->list, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        pip_index_destroy(x);
        return hip_fail(e, "filling the index");
    }
    int per_cu = 0;
    if (pipdev::locate_max_blocks_per_cu(&per_cu) != hipSuccess || per_cu < 1) per_cu = 1;
    x->blocks = per_cu * ctx->cu_count;
    *out = x;
    return PIP_OK;
}

pip_status pip_index_locate(pip_index x, const float* Q, int64_t m, int32_t* ids,
                            hipStream_t stream) {
    if (!x) return fail(PIP_EINVAL, "index is NULL");
    if (m < 0) return fail(PIP_EINVAL, "m = %lld is negative", (long long)m);
    if (m > 0 && (!Q || !aligned(Q, 8))) return fail(PIP_EINVAL, "Q is NULL or not 8-byte aligned");
    if (m > 0 && (!ids || !aligned(ids, 4))) return fail(PIP_EINVAL, "ids is NULL or misaligned");
    if (m == 0) return PIP_OK;
    DeviceGuard g(x->ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipError_t e = pipdev::launch_locate(x->rec, x->P, x->qrec, x->gen, x->grid, x->cell_off, x->list, Q, m, ids,
                                         x->blocks, stream);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return PIP_OK;
}

size_t pip_index_locate_workspace_bytes(pip_index x, int64_t m) {
    if (!x || m < 0) return 0;
    size_t a, b, c, d;
    return pipdev::locate_binned_workspace(x->nbins, m, &a, &b, &c, &d);
}

pip_status pip_index_locate_binned(pip_index x, const float* Q, int64_t m, int32_t* ids,
                                   void* workspace, size_t ws_bytes, hipStream_t stream) {
    if (!x) return fail(PIP_EINVAL, "index is NULL");
    if (m < 0) return fail(PIP_EINVAL, "m = %lld is negative", (long long)m);
    // the binned copy is indexed with int32 offsets
    if (m >= (int64_t(1) << 31)) return fail(PIP_EUNSUPPORTED, "m = %lld is too large", (long long)m);
    if (m > 0 && (!Q || !aligned(Q, 8))) return fail(PIP_EINVAL, "Q is NULL or not 8-byte aligned");
    if (m > 0 && (!ids || !aligned(ids, 4))) return fail(PIP_EINVAL, "ids is NULL or misaligned");
    if (m == 0) return PIP_OK;
    const size_t need = pip_index_locate_workspace_bytes(x, m);
    if (!workspace || !aligned(workspace, 256) || ws_bytes < need)
        return fail(PIP_EINVAL, "workspace must be 256-byte aligned with >= %zu bytes", need);
    DeviceGuard g(x->ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipError_t e = pipdev::launch_locate_binned(x->rec, x->P, x->qrec, x->gen, x->grid, x->cell_off, x->list, x->sf,
                                                x->sgx, x->nbins, Q, m, ids, workspace,
                                                x->ctx->cu_count, stream);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return PIP_OK;
}

pip_status pip_index_info(pip_index x, int64_t* cells, int64_t* entries) {
    if (!x) return fail(PIP_EINVAL, "index is NULL");
    if (cells) *cells = x->cells;
    if (entries) *entries = x->entries;
    return PIP_OK;
}

pip_status pip_set_option(pip_ctx ctx, pip_option opt, int64_t value) {
    if (!ctx) return fail(PIP_EINVAL, "ctx is NULL");
    switch (opt) {
        case PIP_OPT_MFMA_MIN_EDGES:
            if (value < 0 || value > PIP_MAX_EDGES + 1)
                return fail(PIP_EINVAL, "PIP_OPT_MFMA_MIN_EDGES must be in [0, %d]", PIP_MAX_EDGES + 1);
            ctx->mfma_min_edges = (int)value;
            return PIP_OK;
        case PIP_OPT_ALLPAIRS_CULL:
            if (value != 0 && value != 1)
                return fail(PIP_EINVAL, "PIP_OPT_ALLPAIRS_CULL must be 0 or 1");
            ctx->allpairs_cull = (int)value;
            return PIP_OK;
        case PIP_OPT_COST_CULL:
            if (value != 0 && value != 1) return fail(PIP_EINVAL, "PIP_OPT_COST_CULL must be 0 or 1");
            ctx->cost_cull = (int)value;
            return PIP_OK;
        case PIP_OPT_ALLPAIRS_PAIR:
            if (value != 0 && value != 1)
                return fail(PIP_EINVAL, "PIP_OPT_ALLPAIRS_PAIR must be 0 or 1");
            ctx->allpairs_pair = (int)value;
            return PIP_OK;
        case PIP_OPT_COST_PAIR:
            if (value != 0 && value != 1) return fail(PIP_EINVAL, "PIP_OPT_COST_PAIR must be 0 or 1");
            ctx->cost_pair = (int)value;
            return PIP_OK;
        case PIP_OPT_RADIAL_MIN_EDGES:
            if (value < 0 || value > PIP_MAX_EDGES + 1)
                return fail(PIP_EINVAL, "PIP_OPT_RADIAL_MIN_EDGES must be in [0, %d]", PIP_MAX_EDGES + 1);
            ctx->radial_min_edges = (int)value;
            return PIP_OK;
        case PIP_OPT_EARLY_EXIT:
            if (value != 0 && value != 1) return fail(PIP_EINVAL, "PIP_OPT_EARLY_EXIT must be 0 or 1");
            ctx->early_exit = (int)value;
            return PIP_OK;
    }
    return fail(PIP_EINVAL, "unknown option %d", (int)opt);
}

pip_status pip_plan_create(pip_ctx ctx, pip_plan_kind kind, const void* desc, pip_plan* out) {
    if (!ctx) return fail(PIP_EINVAL, "ctx is NULL");
    if (!desc || !out) return fail(PIP_EINVAL, "desc or out is NULL");
    switch (kind) {
        case PIP_PLAN_BATCHED: {
            const pip_batched_desc& d = *static_cast<const pip_batched_desc*>(desc);
            return pip_plan_create_batched(ctx, d.P, d.vtx_off, d.V, d.total_vertices, d.pt_off,
                                           d.Q, d.total_points, d.lbl_word_off, d.labels,
                                           d.status, out);
        }
        case PIP_PLAN_ALLPAIRS: {
            const pip_allpairs_desc& d = *static_cast<const pip_allpairs_desc*>(desc);
            return pip_plan_create_allpairs(ctx, d.P, d.n, d.V, d.Q, d.m, d.labels, d.counts,
                                            d.status, out);
        }
        case PIP_PLAN_COST_FWD:
        case PIP_PLAN_COST_BWD: {
            const pip_cost_desc& d = *static_cast<const pip_cost_desc*>(desc);
            return pip_plan_create_cost(ctx, kind == PIP_PLAN_COST_BWD ? 1 : 0, d.footprint, d.n,
                                        d.pose, d.K, d.Q, d.m, d.cost, d.grad_cost, d.grad_pose,
                                        d.grad_footprint, d.residual, out);
        }
    }
    return fail(PIP_EINVAL, "unknown plan kind %d", (int)kind);
}

pip_status pip_get_option(pip_ctx ctx, pip_option opt, int64_t* value) {
    if (!ctx || !value) return fail(PIP_EINVAL, "ctx or value is NULL");
    switch (opt) {
        case PIP_OPT_MFMA_MIN_EDGES:
            *value = ctx->mfma_min_edges;
            return PIP_OK;
        case PIP_OPT_ALLPAIRS_CULL:
            *value = ctx->allpairs_cull;
            return PIP_OK;
        case PIP_OPT_COST_CULL:
            *value = ctx->cost_cull;
            return PIP_OK;
        case PIP_OPT_ALLPAIRS_PAIR:
            *value = ctx->allpairs_pair;
            return PIP_OK;
        case PIP_OPT_COST_PAIR:
            *value = ctx->cost_pair;
            return PIP_OK;
        case PIP_OPT_RADIAL_MIN_EDGES:
            *value = ctx->radial_min_edges;
            return PIP_OK;
        case PIP_OPT_EARLY_EXIT:
            *value = ctx->early_exit;
            return PIP_OK;
    }
    return fail(PIP_EINVAL, "unknown option %d", (int)opt);
}

}  // extern "C"
