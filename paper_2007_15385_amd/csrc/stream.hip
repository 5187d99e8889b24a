// Single-polygon streaming kernels: one polygon, a very large point array.
//
// Each workgroup first derives the polygon's generators (Section 3) into LDS,
// then every wave walks its own chunks of points.  float32 points for the
// Voronoi, sign-of-offset and plain tests take k_stream32 (512-point chunks,
// see stream32.hpp); binary64 points, ray crossing and the largest-margin
// output take k_stream, whose chunks are 256 points (4 per lane, lane l
// holding points l, l+64, l+128, l+192 of the chunk, so each 8- or 16-byte
// load of a wave covers one contiguous span of memory).  Results are packed
// with wave ballots: the mask of slot j covers points [64 j, 64 j + 64) of
// the chunk, i.e. two consecutive little-endian label words.
//
// Voronoi and sign of offset decide a point in float32 only when the margin
// clears the proven band; the remaining points are queued per wave in LDS
// and re-decided in binary64 (all 64 lanes busy) when the queue fills and at
// the end.  A queued point's label bit is left 0 by the chunk's store and set
// afterwards with an atomic OR by the same wave, after a fence.
#include "device.hpp"
#include "kernels.hpp"
#include "radial.hpp"
#include "stream32.hpp"

using namespace pipdev;

namespace {

template <typename PT>
struct PointIO;

template <>
struct PointIO<float> {
    using V2 = float2;
    __device__ static float2 load(const void* Q, int64_t i) {
        return static_cast<const float2*>(Q)[i];
    }
};

template <>
struct PointIO<double> {
    using V2 = double2;
    __device__ static double2 load(const void* Q, int64_t i) {
        return static_cast<const double2*>(Q)[i];
    }
};

// Loads of one chunk.  The loads are unconditional (indices past the end
// are clamped to the last point, m >= 1), so the compiler can wait for
// exactly the previous chunk's loads and keep this chunk's in flight while
// the previous one is processed; out-of-range slots are masked later.
template <typename PT>
__device__ __forceinline__ void load_chunk(const void* Q, int64_t m, int64_t chunk, int lane,
                                           PT (&x)[kPPL], PT (&y)[kPPL]) {
    const int64_t last = m - 1;
#pragma unroll
    for (int j = 0; j < kPPL; ++j) {
        int64_t idx = chunk * kChunk + lane + kWave * j;
        idx = idx < last ? idx : last;
        const auto p = PointIO<PT>::load(Q, idx);
        x[j] = p.x;
        y[j] = p.y;
    }
}

// Local float32 coordinate: fl32(p - o).  For float32 input this is one
// rounded float32 subtraction; for binary64 input the difference is taken
// in binary64 and rounded once more to float32.
__device__ __forceinline__ float to_local(float p, float o) { return p - o; }
__device__ __forceinline__ float to_local(double p, float o) { return (float)(p - (double)o); }

// Lane k (k < 8) stores label word k of the chunk.  The masks are
// wave-uniform; a select tree on the lane's bits picks the word (plain
// selects between scalar values, no per-lane array indexing).
// Re-decide the queued points in binary64 and set their inside bits.  The
// queue holds each point's index and its coordinates as loaded (no second
// read of the point from HBM).
//
// Only the wave that owns a chunk ever writes its label words: first the
// chunk store (undecided bits 0), later these ORs, issued after wave_drain()
// so no OR can be overtaken by the store it modifies.
template <int KIND, typename PT>
__device__ void flush_queue(const PolyLds& S, const int64_t* qi, const PT* qx, const PT* qy,
                            int count, uint32_t* labels, int lane) {
    wave_drain();
    for (int e = lane; e < count; e += kWave) {
        const int64_t idx = qi[e];
        const double x = (double)qx[e], y = (double)qy[e];
        bool in;
        if constexpr (KIND == K_VORONOI)
            in = voronoi64(x, y, S.gen, S.n);
        else
            in = sign_of_offset64(x, y, S.vtx, S.n);
        if (in) or_label_bit(labels, idx >> 5, (uint32_t)(idx & 31));
    }
    __builtin_amdgcn_wave_barrier();
}

// float32, binary64-free preparation (Algorithms 3-4 evaluated in float32 in
// the global frame) for the plain reference kernel.
__device__ void prepare_plain(PolyLds& S, int lane) {
    const int n = S.n;
    float Ss = 0.f, Sx = 0.f, Sy = 0.f;
    for (int i = 0; i < n; ++i) {
        const int j = prev_edge(i, n);
        const float vx = (float)S.vtx[i].x, vy = (float)S.vtx[i].y;
        const float wx = (float)S.vtx[j].x, wy = (float)S.vtx[j].y;
        const float Ai = wx * vy - vx * wy;
        Ss += Ai;
        Sx += (vx + wx) * Ai;
        Sy += (vy + wy) * Ai;
    }
    const float a = 0.5f * Ss;
    const float cx = Sx / (6.f * a), cy = Sy / (6.f * a);
    const int i = lane < n ? lane : 0;
    const int j = prev_edge(i, n);
    const float vx = (float)S.vtx[i].x, vy = (float)S.vtx[i].y;
    const float wx = (float)S.vtx[j].x, wy = (float)S.vtx[j].y;
    const float ea = vy - wy, eb = wx - vx;
    const float ec = -(ea * vx + eb * vy);
    const float den = ea * ea + eb * eb;
    const float gx = ((eb * eb - ea * ea) * cx + (-2.f * ea) * eb * cy + (-2.f * ec) * ea) / den;
    const float gy = ((-2.f * ea) * eb * cx + (ea * ea - eb * eb) * cy + (-2.f * ec) * eb) / den;
    const float A = 2.f * (gx - cx), B = 2.f * (gy - cy);
    const float C = (gx * gx + gy * gy) - (cx * cx + cy * cy);
    S.coef[lane] = make_float4(A, B, -C, 0.f);
    if (lane == 0) {
        S.ox = 0.f;
        S.oy = 0.f;
        S.n4 = (n + 3) & ~3;
        S.status = ST_OK;
    }
}

template <int KIND, typename PT>
__global__ __launch_bounds__(kBlock) void k_stream(const double* __restrict__ V, int n,
                                                  const void* __restrict__ Q, int64_t m,
                                                  uint32_t* __restrict__ labels,
                                                  float* __restrict__ margin,
                                                  int32_t* __restrict__ status) {
    constexpr bool kQueue = (KIND == K_VORONOI || KIND == K_SOO);
    __shared__ PolyLds S;
    __shared__ int64_t queue[kWavesPerBlock][kQueue ? kQueueCap : 1];
    __shared__ PT queue_x[kWavesPerBlock][kQueue ? kQueueCap : 1];
    __shared__ PT queue_y[kWavesPerBlock][kQueue ? kQueueCap : 1];

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = tid / kWave;
    const int64_t nchunks = (m + kChunk - 1) / kChunk;
    const int64_t nwords = (m + 31) / 32;
    const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
    int64_t chunk = (int64_t)blockIdx.x * kWavesPerBlock + wv;

    double2 vt = make_double2(0.0, 0.0);
    if (tid < n) vt = make_double2(V[2 * tid], V[2 * tid + 1]);
    PT px[kPPL], py[kPPL];
    if (m > 0) load_chunk<PT>(Q, m, chunk, lane, px, py);  // in flight during preparation

    if (tid < n) S.vtx[tid] = vt;
    if (tid == 0) S.n = n;
    __syncthreads();
    if (wv == 0) {
        if constexpr (KIND == K_PLAIN)
            prepare_plain(S, lane);
        else
            prepare_polygon(S, KIND, lane);
    }
    __syncthreads();
    if (status && blockIdx.x == 0 && tid == 0) *status = S.status;

    const float ox = S.ox, oy = S.oy;
    const float KQ = S.KQ, KA = S.KA, KB = S.KB, KC = S.KC;
    (void)KQ; (void)KA; (void)KB; (void)KC;
    const int n4 = __builtin_amdgcn_readfirstlane(S.n4);
    const int nv = __builtin_amdgcn_readfirstlane(S.n);
    int qcount = 0;

    for (; chunk < nchunks; chunk += stride) {
        PT nx[kPPL], ny[kPPL];
        load_chunk<PT>(Q, m, chunk + stride, lane, nx, ny);
        const int64_t base = chunk * kChunk;
        uint64_t inm[kPPL];
        bool valid[kPPL];
#pragma unroll
        for (int j = 0; j < kPPL; ++j) valid[j] = base + lane + kWave * j < m;

        if constexpr (KIND == K_RAY) {
            // Algorithm 1 in binary64 directly (exact replay, no band).
            double x[kPPL], y[kPPL];
            bool cross[kPPL];
#pragma unroll
            for (int j = 0; j < kPPL; ++j) {
                x[j] = (double)px[j];
                y[j] = (double)py[j];
                cross[j] = false;
            }
            for (int e = 0; e < nv; ++e) {
                const double4 r = S.ray[e];  // (V'_y, V_y, dV_x, dV_y)
                const double R = S.rhs[e];
                const bool up = r.y > r.x;
#pragma unroll
                for (int j = 0; j < kPPL; ++j) {
                    const bool inr = (r.y > y[j]) != (r.x > y[j]);
                    const double L = y[j] * r.z - x[j] * r.w;
                    const bool left = up ? (L > R) : (L < R);
                    cross[j] = cross[j] != (inr && left);
                }
            }
#pragma unroll
            for (int j = 0; j < kPPL; ++j) {
                const bool fin = isfinite(x[j]) && isfinite(y[j]);
                inm[j] = __ballot(valid[j] && fin && cross[j]);
            }
            store_chunk_words(labels, base / 32, nwords - base / 32, lane, inm);
        } else if constexpr (KIND == K_MARGIN || KIND == K_PLAIN) {
            float X[kPPL], Y[kPPL], Mx[kPPL];
#pragma unroll
            for (int j = 0; j < kPPL; ++j) {
                X[j] = to_local(px[j], ox);
                Y[j] = to_local(py[j], oy);
                Mx[j] = -__builtin_huge_valf();
            }
            for (int e = 0; e < n4; e += 4) {
                const float4 c0 = S.coef[e + 0], c1 = S.coef[e + 1];
                const float4 c2 = S.coef[e + 2], c3 = S.coef[e + 3];
#pragma unroll
                for (int j = 0; j < kPPL; ++j) {
                    const float m0 = fmaf(c0.x, X[j], fmaf(c0.y, Y[j], c0.z));
                    const float m1 = fmaf(c1.x, X[j], fmaf(c1.y, Y[j], c1.z));
                    const float m2 = fmaf(c2.x, X[j], fmaf(c2.y, Y[j], c2.z));
                    const float m3 = fmaf(c3.x, X[j], fmaf(c3.y, Y[j], c3.z));
                    Mx[j] = fmaxf(fmaxf(Mx[j], m0), m1);
                    Mx[j] = fmaxf(fmaxf(Mx[j], m2), m3);
                }
            }
            if constexpr (KIND == K_MARGIN) {
#pragma unroll
                for (int j = 0; j < kPPL; ++j)
                    if (valid[j]) margin[base + lane + kWave * j] = Mx[j];
            } else {
#pragma unroll
                for (int j = 0; j < kPPL; ++j) inm[j] = __ballot(valid[j] && Mx[j] <= 0.0f);
                store_chunk_words(labels, base / 32, nwords - base / 32, lane, inm);
            }
        } else {
            float X[kPPL], Y[kPPL];
#pragma unroll
            for (int j = 0; j < kPPL; ++j) {
                X[j] = to_local(px[j], ox);
                Y[j] = to_local(py[j], oy);
            }
            uint64_t unc[kPPL];
            screen_chunk<KIND>(S.coef, n4, KQ, KA, KB, KC, X, Y, valid, inm, unc);
            const int nunc = __popcll(unc[0]) + __popcll(unc[1]) + __popcll(unc[2]) + __popcll(unc[3]);
            if (nunc != 0 && qcount + nunc > kQueueCap) {  // flush before push
                flush_queue<KIND, PT>(S, queue[wv], queue_x[wv], queue_y[wv], qcount, labels, lane);
                qcount = 0;
            }
            store_chunk_words(labels, base / 32, nwords - base / 32, lane, inm);
            if (nunc != 0) {
                const uint64_t lt = lanemask_lt();
#pragma unroll
                for (int j = 0; j < kPPL; ++j) {
                    if (unc[j] == 0) continue;  // wave-uniform: no undecided point in this slot
                    if ((unc[j] >> lane) & 1ull) {
                        const int slot = qcount + __popcll(unc[j] & lt);
                        queue[wv][slot] = base + lane + kWave * j;
                        queue_x[wv][slot] = px[j];
                        queue_y[wv][slot] = py[j];
                    }
                    qcount += __popcll(unc[j]);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < kPPL; ++j) {
            px[j] = nx[j];
            py[j] = ny[j];
        }
    }
    if constexpr (kQueue) {
        if (qcount > 0)
            flush_queue<KIND, PT>(S, queue[wv], queue_x[wv], queue_y[wv], qcount, labels, lane);
    }
}

template <int KIND>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5))) void k_stream32(const double* __restrict__ V, int n,
                                                    const float2* __restrict__ Q, int64_t m,
                                                    uint32_t* __restrict__ labels,
                                                    int32_t* __restrict__ status) {
    constexpr bool kQueue = KIND != K_PLAIN;
    __shared__ PolyLds S;
    __shared__ uint32_t queue_c[kWavesPerBlock][kQueue ? kQueue32 : 1];
    __shared__ float queue_x[kWavesPerBlock][kQueue ? kQueue32 : 1];
    __shared__ float queue_y[kWavesPerBlock][kQueue ? kQueue32 : 1];

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int64_t nfull = m / kChunk32;
    const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
    const int64_t c0 = (int64_t)blockIdx.x * kWavesPerBlock + wv;
    int64_t chunk = c0;
    uint32_t k = 0;  // chunks of this wave so far

    double2 vt = make_double2(0.0, 0.0);
    if (tid < n) vt = make_double2(V[2 * tid], V[2 * tid + 1]);
    float2 pa[kP32], pb[kP32];
    if (nfull > 0) load_full32(Q, chunk < nfull ? chunk : nfull - 1, lane, pa);

    if (tid < n) S.vtx[tid] = vt;
    if (tid == 0) S.n = n;
    __syncthreads();
    if (wv == 0) {
        if constexpr (KIND == K_PLAIN)
            prepare_plain(S, lane);
        else
            prepare_polygon(S, KIND == K_RAY ? K_RAY32 : KIND, lane);
    }
    __syncthreads();
    if (status && blockIdx.x == 0 && tid == 0) *status = S.status;

    const float ox = S.ox, oy = S.oy;
    const float KQ = S.KQ, KA = S.KA, KB = S.KB, KC = S.KC, RQ = S.RQ, KS = fmaxf(KA, KB);
    const float SO = S.SO;
    const int n4 = __builtin_amdgcn_readfirstlane(S.n4);
    const int nv = __builtin_amdgcn_readfirstlane(S.n);
    int qcount = 0;

    // Screen the 8 points of every lane of this wave's k-th chunk `ch`;
    // `rem` points of it exist (>= 512 for a full chunk).
    auto process = [&](const float2(&p)[kP32], int64_t ch, int64_t rem) {
        const bool full = rem >= kChunk32;
        uint64_t inm[kP32], unc[kP32];
        if constexpr (KIND == K_RAY) {
            // Ray crossing (Algorithm 1).  In range: the vertex-above flags
            // c > Q_y with c the vertex height rounded up to float32 (exact
            // for float32 Q_y).  On the left: the sign-of-offset margin s of
            // the edge (its row negated for an edge going down) against its
            // band, decided when |s| > E; a point with an undecided edge goes
            // to binary64.  Flags, parities and the undecided set are wave
            // masks, four slots per pass over the edges.
            float X[kP32], Y[kP32], E[kP32];
            const float clast = S.coef[nv - 1].w;  // start vertex of edge 0
#pragma unroll
            for (int j = 0; j < kP32; ++j) {
                X[j] = p[j].x - ox;
                Y[j] = p[j].y - oy;
                const float r2 = fmaf(X[j], X[j], Y[j] * Y[j]);
                E[j] = fmaf(KQ, r2, fmaf(KA, fabsf(X[j]), fmaf(KB, fabsf(Y[j]), KC)));
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                uint64_t above[4], cross[4], amb[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    above[t] = __ballot(clast > p[4 * h + t].y);
                    cross[t] = 0;
                    amb[t] = 0;
                }
                // one edge: its end vertex's above flags into `ab`; an
                // undecided line test marks the point whether the edge is in
                // range or not (a superset: only points within the band of
                // an edge's line)
                auto edge = [&](const float4& c, const uint64_t(&prev)[4], uint64_t(&ab)[4]) {
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int j = 4 * h + t;
                        ab[t] = __ballot(c.w > p[j].y);
                        const float sm = fmaf(c.x, X[j], fmaf(c.y, Y[j], c.z));
                        amb[t] |= __ballot(!(fabsf(sm) > E[j]));
                        cross[t] ^= (ab[t] ^ prev[t]) & __ballot(sm > E[j]);
                    }
                };
                int e = 0;
                for (; e + 2 <= nv; e += 2) {  // rows negated for edges going down
                    uint64_t mid[4];
                    edge(S.coef[e], above, mid);
                    edge(S.coef[e + 1], mid, above);
                }
                if (e < nv) {
                    uint64_t last[4];
                    edge(S.coef[e], above, last);
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int j = 4 * h + t;
                    // a non-finite point is outside (never queued)
                    const uint64_t fin = __ballot(isfinite(p[j].x) && isfinite(p[j].y));
                    unc[j] = amb[t] & fin;
                    inm[j] = cross[t] & fin & ~amb[t];
                }
            }
        } else {
            // Voronoi: the largest margin; sign of offset (rows oriented so
            // that the inner side is s > 0): the smallest offset only
            float X[kP32], Y[kP32], Mx[kP32];
            {  // edges 0-3 (n4 >= 4) start the max / min
                const float4 c0 = S.coef[0], c1 = S.coef[1], c2 = S.coef[2], c3 = S.coef[3];
    #pragma unroll
                for (int j = 0; j < kP32; ++j) {
                    X[j] = p[j].x - ox;
                    Y[j] = p[j].y - oy;
                    const float m0 = fmaf(c0.x, X[j], fmaf(c0.y, Y[j], c0.z));
                    const float m1 = fmaf(c1.x, X[j], fmaf(c1.y, Y[j], c1.z));
                    const float m2 = fmaf(c2.x, X[j], fmaf(c2.y, Y[j], c2.z));
                    const float m3 = fmaf(c3.x, X[j], fmaf(c3.y, Y[j], c3.z));
                    if constexpr (KIND == K_SOO)
                        Mx[j] = fminf(fminf(fminf(m0, m1), m2), m3);
                    else
                        Mx[j] = fmaxf(fmaxf(fmaxf(m0, m1), m2), m3);
                }
            }
            for (int e = 4; e < n4; e += 4) {
                const float4 c0 = S.coef[e + 0], c1 = S.coef[e + 1];
                const float4 c2 = S.coef[e + 2], c3 = S.coef[e + 3];
    #pragma unroll
                for (int j = 0; j < kP32; ++j) {
                    const float m0 = fmaf(c0.x, X[j], fmaf(c0.y, Y[j], c0.z));
                    const float m1 = fmaf(c1.x, X[j], fmaf(c1.y, Y[j], c1.z));
                    const float m2 = fmaf(c2.x, X[j], fmaf(c2.y, Y[j], c2.z));
                    const float m3 = fmaf(c3.x, X[j], fmaf(c3.y, Y[j], c3.z));
                    if constexpr (KIND == K_SOO) {
                        Mx[j] = fminf(fminf(Mx[j], m0), m1);
                        Mx[j] = fminf(fminf(Mx[j], m2), m3);
                    } else {
                        Mx[j] = fmaxf(fmaxf(Mx[j], m0), m1);
                        Mx[j] = fmaxf(fmaxf(Mx[j], m2), m3);
                    }
                }
            }
            // When |X| + |Y| <= RQ for every point of the chunk, the band's
            // quadratic term is inside its linear constants and
            // E = KS (|X| + |Y|) + KC with KS = max(KA, KB) (wave-uniform branch;
            // a NaN sum is dropped by the max and gives a NaN band: undecided)
            bool fold = false;
            float sxy[kP32];
            if constexpr (KIND == K_VORONOI || KIND == K_SOO) {
                float acc = 0.0f;
    #pragma unroll
                for (int j = 0; j < kP32; ++j) {
                    sxy[j] = fabsf(X[j]) + fabsf(Y[j]);
                    acc = fmaxf(acc, sxy[j]);
                }
                fold = __ballot(acc > RQ) == 0;
            }
            if (fold) {
    #pragma unroll
                for (int j = 0; j < kP32; ++j) {
                    const float E = fmaf(KS, sxy[j], KC);
                    uint64_t in, out;
                    if constexpr (KIND == K_SOO) {
                        // inside: every offset on the inner side; outside: one
                        // on the outer side, and fl32(|X| + |Y|) < SO proves
                        // one on the inner side
                        in = __ballot(Mx[j] > E);
                        out = __ballot(Mx[j] < -E) & __ballot(sxy[j] < SO);
                    } else {
                        in = __ballot(Mx[j] < -E);
                        out = __ballot(Mx[j] > E);
                    }
                    inm[j] = in;
                    unc[j] = ~(in | out);
                }
            } else {
    #pragma unroll
                for (int j = 0; j < kP32; ++j) {
                    if constexpr (KIND == K_PLAIN) {
                        inm[j] = __ballot(Mx[j] <= 0.0f);
                        unc[j] = 0;
                    } else {
                        const float r2 = fmaf(X[j], X[j], Y[j] * Y[j]);
                        const float E = fmaf(KQ, r2, fmaf(KA, fabsf(X[j]), fmaf(KB, fabsf(Y[j]), KC)));
                        uint64_t in, out;
                        if constexpr (KIND == K_SOO) {
                            in = __ballot(Mx[j] > E);
                            out = __ballot(Mx[j] < -E) & __ballot(sxy[j] < SO);
                        } else {
                            in = __ballot(Mx[j] < -E);
                            out = __ballot(Mx[j] > E);
                        }
                        inm[j] = in;
                        unc[j] = ~(in | out);
                    }
                }
            }
        }
        if (!full) {
#pragma unroll
            for (int j = 0; j < kP32; ++j) {
                const uint64_t vm = __ballot(lane + kWave * j < rem);
                inm[j] &= vm;
                unc[j] &= vm;
            }
        }
        const uint32_t w = chunk_word32(inm);
        const int64_t nw = full ? kWords32 : (rem + 31) / 32;
        if (lane < nw) labels[ch * kWords32 + lane] = w;
        if constexpr (kQueue) {
            int nunc = 0;
#pragma unroll
            for (int j = 0; j < kP32; ++j) nunc += __popcll(unc[j]);
            if (nunc != 0) {
                if (qcount + nunc > kQueue32) {  // flush before push (drains the store above)
                    flush_queue32<KIND>(S, queue_c[wv], queue_x[wv], queue_y[wv], qcount, labels,
                                        lane, c0, stride);
                    qcount = 0;
                }
                const uint64_t lt = lanemask_lt();
#pragma unroll
                for (int j = 0; j < kP32; ++j) {
                    if (unc[j] == 0) continue;  // wave-uniform: no undecided point in this slot
                    if ((unc[j] >> lane) & 1ull) {
                        const int slot = qcount + __popcll(unc[j] & lt);
                        queue_c[wv][slot] = (k << 9) | (uint32_t)(lane + kWave * j);
                        queue_x[wv][slot] = p[j].x;
                        queue_y[wv][slot] = p[j].y;
                    }
                    qcount += __popcll(unc[j]);
                }
            }
        }
        ++k;
    };

    for (;;) {
        if (chunk >= nfull) break;
        load_full32(Q, chunk + stride < nfull ? chunk + stride : chunk, lane, pb);
        process(pa, chunk, kChunk32);
        chunk += stride;
        if (chunk >= nfull) break;
        load_full32(Q, chunk + stride < nfull ? chunk + stride : chunk, lane, pa);
        process(pb, chunk, kChunk32);
        chunk += stride;
    }
    if (chunk == nfull && nfull * kChunk32 < m) {  // the partial chunk
        const int64_t base = nfull * kChunk32;
        const int rem = (int)(m - base);
        float2 pt[kP32];
#pragma unroll
        for (int j = 0; j < kP32; ++j) {
            const int r = lane + kWave * j;
            pt[j] = Q[base + (r < rem ? r : rem - 1)];
        }
        process(pt, chunk, rem);
    }
    if constexpr (kQueue) {
        if (qcount > 0)
            flush_queue32<KIND>(S, queue_c[wv], queue_x[wv], queue_y[wv], qcount, labels, lane,
                                c0, stride);
    }
}

// ----------------------------------------------------------------------------
// Voronoi with the radial pre-screen (radial.hpp).  The fast path of a chunk
// costs a few operations per point: r2 = fl32(X^2 + Y^2), the octant's two
// thresholds from LDS and three compares decide every point closer to p_0
// than the octant's inner radius (inside) or beyond its outer radius
// (outside).  The other points (coordinates as loaded and a position code)
// enter a per-wave ring in LDS.
//
// The label words of the wave's last eight chunks stay in LDS (in the
// polygon block's space for the ray-crossing test, unused here).  The ring
// is consumed in rounds of 64 entries, one per lane: a lane screens its point
// against the candidate edges of the point's octant (radial.hpp) with the
// band of the float32 screen, re-decides it in binary64 over the same edges
// when the band leaves it undecided, and sets its inside bit in the LDS copy
// of the word with an LDS atomic OR.  A full round runs whenever 64 entries
// wait; a chunk's words go to memory with one plain store seven chunks later,
// after its remaining entries have been settled (in a partial round if the
// full rounds have not reached them).  No global read-modify-write is needed
// and a chunk costs a fixed set of memory operations (its loads and one
// store).
// ----------------------------------------------------------------------------
constexpr int kSlots = 8;  // chunks whose label words stay in LDS
static_assert(kWavesPerBlock * kSlots * kWords32 <= kMaxEdges * 10,
              "the word rings fit the polygon block's free space");

__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
    return v;
}

// One round: entries head .. head + cnt - 1 of the ring (cnt <= 64), entry
// head + l on lane l.  Every lane walks the wave's longest candidate list;
// a shorter list is padded with repeats, so no lane needs a mask.  An entry's
// code is (slot << 9) | r for point r of the chunk in word-ring slot `slot`.
__device__ __forceinline__ void radial_round(const PolyLds& S, const RadialTab& R, const uint32_t* qc,
                                             const float2* qp, uint32_t head, int cnt,
                                             uint32_t (*words)[kWords32], int lane) {
    const bool valid = lane < cnt;
    const uint32_t slot = (head + (uint32_t)lane) & (kQueue32 - 1);
    const float2 q = qp[slot];
    const uint32_t cd = qc[slot];
    const float X = q.x - S.ox, Y = q.y - S.oy;
    const int c = radial_class(R, X, Y);
    const uint8_t* list = R.list[c];
    const int len = wave_max_int(valid ? R.len4[c] : 0);
    float M = -__builtin_huge_valf();
    for (int t = 0; t < len; t += 4) {
        const uint32_t ix = *reinterpret_cast<const uint32_t*>(list + t);  // 4 edge indices
        const float4 k0 = S.coef[ix & 255u], k1 = S.coef[(ix >> 8) & 255u];
        const float4 k2 = S.coef[(ix >> 16) & 255u], k3 = S.coef[ix >> 24];
        const float m0 = fmaf(k0.x, X, fmaf(k0.y, Y, k0.z));
        const float m1 = fmaf(k1.x, X, fmaf(k1.y, Y, k1.z));
        const float m2 = fmaf(k2.x, X, fmaf(k2.y, Y, k2.z));
        const float m3 = fmaf(k3.x, X, fmaf(k3.y, Y, k3.z));
        M = fmaxf(fmaxf(M, m0), m1);
        M = fmaxf(fmaxf(M, m2), m3);
    }
    const float r2 = fmaf(X, X, Y * Y);
    const float E = fmaf(S.KQ, r2, fmaf(S.KA, fabsf(X), fmaf(S.KB, fabsf(Y), S.KC)));
    bool in = valid && M < -E;
    if (valid && !(M < -E) && !(M > E))  // inside the band: binary64, Algorithm 5
        in = voronoi64_list((double)q.x, (double)q.y, S.gen, list, R.len4[c]);
    if (in) atomicOr(&words[(cd >> 9) & (kSlots - 1)][(cd & 511u) >> 5], 1u << (cd & 31u));
}

__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5))) void k_stream32_radial(
    const double* __restrict__ V, int n, const float2* __restrict__ Q, int64_t m,
    uint32_t* __restrict__ labels, int32_t* __restrict__ status) {
    __shared__ PolyLds S;
    __shared__ RadialTab R;
    __shared__ uint32_t queue_c[kWavesPerBlock][kQueue32];
    __shared__ float2 queue_p[kWavesPerBlock][kQueue32];
    __shared__ uint32_t ring_end[kWavesPerBlock][kSlots];  // ring tail after each slot's push
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int64_t nfull = m / kChunk32;
    const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
    const int64_t c0 = (int64_t)blockIdx.x * kWavesPerBlock + wv;
    int64_t chunk = c0;
    uint32_t k = 0;  // chunks of this wave so far

    double2 vt = make_double2(0.0, 0.0);
    if (tid < n) vt = make_double2(V[2 * tid], V[2 * tid + 1]);
    float2 pa[kP32], pb[kP32];
    if (nfull > 0) load_full32(Q, chunk < nfull ? chunk : nfull - 1, lane, pa);

    if (tid < n) S.vtx[tid] = vt;
    if (tid == 0) S.n = n;
    __syncthreads();
    if (wv == 0) {
        prepare_polygon(S, K_VORONOI, lane);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        prepare_radial(S, lane, R);
    }
    __syncthreads();
    if (status && blockIdx.x == 0 && tid == 0) *status = S.status;
    const float ox = S.ox, oy = S.oy;
    const float tfar = R.tfar;
    const char* tab = reinterpret_cast<const char*>(R.t);
    uint32_t* qc = queue_c[wv];
    float2* qp = queue_p[wv];
    uint32_t(*words)[kWords32] =
        reinterpret_cast<uint32_t(*)[kWords32]>(S.aux + wv * kSlots * kWords32);
    uint32_t* ends = ring_end[wv];
    // ring positions (wave-uniform, counting pushes modulo 2^32): entries
    // head .. tail - 1; tail - head never exceeds the ring size
    uint32_t head = 0, tail = 0;

    // settle every entry pushed before `end` (partial rounds allowed)
    auto settle = [&](uint32_t end) {
        while ((int)(end - head) > 0) {
            const int cnt = min((int)(end - head), kWave);
            radial_round(S, R, qc, qp, head, cnt, words, lane);
            head += (uint32_t)cnt;
        }
    };
    // words of the wave's i-th chunk (i < k) from LDS to memory
    auto store_chunk = [&](uint32_t i) {
        const int64_t ch = c0 + (int64_t)i * stride;
        const int64_t nw = ch < nfull ? kWords32 : ((m - nfull * kChunk32) + 31) / 32;
        __builtin_amdgcn_wave_barrier();
        if (lane < nw) labels[ch * kWords32 + lane] = words[i & (kSlots - 1)][lane];
    };
    auto process = [&](const float2(&p)[kP32], int64_t rem) {
        const bool full = rem >= kChunk32;
        const uint32_t sl = k & (kSlots - 1);
        uint64_t inm[kP32], amb[kP32];
#pragma unroll
        for (int j = 0; j < kP32; ++j) {
            const float X = p[j].x - ox, Y = p[j].y - oy;
            const float r2 = fmaf(X, X, Y * Y);
            // octant byte offset: 32 sign(X) + 16 sign(Y) + 8 (|Y| > |X|)
            const uint32_t off = ((__float_as_uint(X) >> 31) << 5) | ((__float_as_uint(Y) >> 31) << 4) |
                                 (fabsf(Y) > fabsf(X) ? 8u : 0u);
            const float2 t = *reinterpret_cast<const float2*>(tab + off);
            const bool in = r2 < t.x;
            const bool out = (r2 > t.y) & (r2 < tfar);
            inm[j] = __ballot(in);
            amb[j] = ~(inm[j] | __ballot(out));
        }
        if (!full) {
#pragma unroll
            for (int j = 0; j < kP32; ++j) {
                const uint64_t vm = __ballot(lane + kWave * j < rem);
                inm[j] &= vm;
                amb[j] &= vm;
            }
        }
        const uint32_t w = chunk_word32(inm);
        if (lane < kWords32) words[sl][lane] = w;
        int na = 0;
#pragma unroll
        for (int j = 0; j < kP32; ++j) na += __popcll(amb[j]);
        if (na != 0) {
            while (tail - head + (uint32_t)na > (uint32_t)kQueue32) {  // make room
                const int cnt = min((int)(tail - head), kWave);
                radial_round(S, R, qc, qp, head, cnt, words, lane);
                head += (uint32_t)cnt;
            }
            const uint64_t lt = lanemask_lt();
#pragma unroll
            for (int j = 0; j < kP32; ++j) {
                if ((amb[j] >> lane) & 1ull) {
                    const uint32_t slot = (tail + (uint32_t)__popcll(amb[j] & lt)) & (kQueue32 - 1);
                    // the lane index from the hardware, not a register kept live
                    qc[slot] = (sl << 9) | ((uint32_t)__lane_id() + kWave * j);
                    qp[slot] = p[j];
                }
                tail += (uint32_t)__popcll(amb[j]);
            }
        }
        if (lane == 0) ends[sl] = tail;
        if (tail - head >= (uint32_t)kWave) {  // a full round
            radial_round(S, R, qc, qp, head, kWave, words, lane);
            head += kWave;
        }
        if (k + 1 >= kSlots) {  // chunk k - 7 leaves the word ring before chunk k + 1 reuses its slot
            const uint32_t old = k + 1 - kSlots;
            __builtin_amdgcn_wave_barrier();
            settle(ends[old & (kSlots - 1)]);
            store_chunk(old);
        }
        ++k;
    };
    for (;;) {
        if (chunk >= nfull) break;
        load_full32(Q, chunk + stride < nfull ? chunk + stride : chunk, lane, pb);
        process(pa, kChunk32);
        chunk += stride;
        if (chunk >= nfull) break;
        load_full32(Q, chunk + stride < nfull ? chunk + stride : chunk, lane, pa);
        process(pb, kChunk32);
        chunk += stride;
    }
    if (chunk == nfull && nfull * kChunk32 < m) {  // the partial chunk
        const int64_t base = nfull * kChunk32;
        const int rem = (int)(m - base);
        float2 pt[kP32];
#pragma unroll
        for (int j = 0; j < kP32; ++j) {
            const int r = lane + kWave * j;
            pt[j] = Q[base + (r < rem ? r : rem - 1)];
        }
        process(pt, rem);
    }
    settle(tail);  // every entry, then the chunks still in the word ring
    for (uint32_t i = k >= kSlots - 1 ? k - (kSlots - 1) : 0; i < k; ++i) store_chunk(i);
}

// Thresholds of the radial pre-screen, for tests and diagnostics: one wave
// prepares the polygon and writes T_in[8], T_out[8], T_far.
__global__ __launch_bounds__(kWave) void k_radial_bounds(const double* __restrict__ V, int n,
                                                        float* __restrict__ out) {
    __shared__ PolyLds S;
    __shared__ RadialTab R;
    const int lane = threadIdx.x;
    if (lane < n) S.vtx[lane] = make_double2(V[2 * lane], V[2 * lane + 1]);
    if (lane == 0) S.n = n;
    __syncthreads();
    prepare_polygon(S, K_VORONOI, lane);
    __syncthreads();
    prepare_radial(S, lane, R);
    __syncthreads();
    if (lane < 8) {
        out[lane] = R.t[lane].x;
        out[8 + lane] = R.t[lane].y;
    }
    if (lane == 0) out[16] = R.tfar;
}

// polygon_to_generators: one wave derives p_0 and the n outer generators.
// The float32 screen table of one polygon as the streaming screens derive
// it: out[0..12) = ox, oy, KQ, KA, KB, KC, n4, status, RQ, 0, 0, 0; then n4
// rows (A, B, -C, 0) (Voronoi) or (-dV_y, dV_x, -R, 0) (sign of offset).
__global__ __launch_bounds__(kWave) void k_screen_table(const double* __restrict__ V, int n,
                                                       int kind, double factor,
                                                       float* __restrict__ out) {
    __shared__ PolyLds S;
    const int lane = threadIdx.x;
    if (lane < n) S.vtx[lane] = make_double2(V[2 * lane], V[2 * lane + 1]);
    if (lane == 0) S.n = n;
    __syncthreads();
    prepare_polygon(S, kind, lane, false, factor);
    __syncthreads();
    if (lane == 0) {
        out[0] = S.ox;
        out[1] = S.oy;
        out[2] = S.KQ;
        out[3] = S.KA;
        out[4] = S.KB;
        out[5] = S.KC;
        out[6] = (float)S.n4;
        out[7] = (float)S.status;
        out[8] = S.RQ;
        out[9] = S.SO;
        out[10] = out[11] = 0.0f;
    }
    for (int r = lane; r < S.n4; r += kWave) {
        const float4 c = S.coef[r];
        out[12 + 4 * r] = c.x;
        out[13 + 4 * r] = c.y;
        out[14 + 4 * r] = c.z;
        out[15 + 4 * r] = c.w;
    }
}

__global__ __launch_bounds__(kWave) void k_generators_one(const double* __restrict__ V, int n,
                                                         double* __restrict__ P,
                                                         int32_t* __restrict__ status) {
    __shared__ PolyLds S;
    const int lane = threadIdx.x;
    if (lane < n) S.vtx[lane] = make_double2(V[2 * lane], V[2 * lane + 1]);
    if (lane == 0) S.n = n;
    __syncthreads();
    prepare_polygon(S, K_VORONOI, lane);
    __syncthreads();
    for (int k = lane; k <= n; k += kWave) {
        P[2 * k] = S.gen[k].x;
        P[2 * k + 1] = S.gen[k].y;
    }
    if (status && lane == 0) *status = S.status;
}

template <int KIND>
hipError_t launch_stream32_t(const StreamLaunch& L) {
    const int64_t nchunks = (L.m + kChunk32 - 1) / kChunk32;
    const int64_t want = (nchunks + kWavesPerBlock - 1) / kWavesPerBlock;
    int grid = (int)(want < L.max_blocks ? want : L.max_blocks);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL((k_stream32<KIND>), dim3(grid), dim3(kBlock), 0, L.stream, L.V, L.n,
                       static_cast<const float2*>(L.Q), L.m, L.labels, L.status);
    return hipGetLastError();
}

hipError_t launch_stream32_radial(const StreamLaunch& L) {
    const int64_t nchunks = (L.m + kChunk32 - 1) / kChunk32;
    const int64_t want = (nchunks + kWavesPerBlock - 1) / kWavesPerBlock;
    int grid = (int)(want < L.max_blocks ? want : L.max_blocks);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_stream32_radial, dim3(grid), dim3(kBlock), 0, L.stream, L.V, L.n,
                       static_cast<const float2*>(L.Q), L.m, L.labels, L.status);
    return hipGetLastError();
}

template <int KIND, typename PT>
hipError_t launch_stream_t(const StreamLaunch& L) {
    const int64_t nchunks = (L.m + kChunk - 1) / kChunk;
    const int64_t want = (nchunks + kWavesPerBlock - 1) / kWavesPerBlock;
    int grid = (int)(want < L.max_blocks ? want : L.max_blocks);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL((k_stream<KIND, PT>), dim3(grid), dim3(kBlock), 0, L.stream, L.V, L.n, L.Q,
                       L.m, L.labels, L.margin, L.status);
    return hipGetLastError();
}

}  // namespace

namespace pipdev {

hipError_t launch_stream(const StreamLaunch& L) {
    const bool f64 = L.qdt == 1;
    if (L.radial && !f64 && L.kind == K_VORONOI) return launch_stream32_radial(L);
    if (L.mfma && !f64 && (L.kind == K_VORONOI || L.kind == K_SOO)) return launch_stream_mfma(L);
    switch (L.kind) {
        case K_VORONOI:
            return f64 ? launch_stream_t<K_VORONOI, double>(L) : launch_stream32_t<K_VORONOI>(L);
        case K_SOO:
            return f64 ? launch_stream_t<K_SOO, double>(L) : launch_stream32_t<K_SOO>(L);
        case K_RAY:
            return f64 ? launch_stream_t<K_RAY, double>(L) : launch_stream32_t<K_RAY>(L);
        case K_PLAIN:
            return f64 ? launch_stream_t<K_PLAIN, double>(L) : launch_stream32_t<K_PLAIN>(L);
        case K_MARGIN:
            return f64 ? launch_stream_t<K_MARGIN, double>(L) : launch_stream_t<K_MARGIN, float>(L);
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_screen_table(const double* V, int n, int kind, double factor, float* out,
                               hipStream_t stream) {
    hipLaunchKernelGGL(k_screen_table, dim3(1), dim3(kWave), 0, stream, V, n, kind, factor, out);
    return hipGetLastError();
}

hipError_t launch_generators_one(const double* V, int n, double* P, int32_t* status,
                                 hipStream_t stream) {
    hipLaunchKernelGGL(k_generators_one, dim3(1), dim3(kWave), 0, stream, V, n, P, status);
    return hipGetLastError();
}

hipError_t stream_max_blocks_per_cu(int kind, int qdt, int* out) {
    const void* f = nullptr;
    const bool f64 = qdt == 1;
    switch (kind) {
        case K_VORONOI: f = f64 ? (const void*)k_stream<K_VORONOI, double> : (const void*)k_stream32<K_VORONOI>; break;
        case K_SOO: f = f64 ? (const void*)k_stream<K_SOO, double> : (const void*)k_stream32<K_SOO>; break;
        case K_RAY: f = f64 ? (const void*)k_stream<K_RAY, double> : (const void*)k_stream32<K_RAY>; break;
        case K_PLAIN: f = f64 ? (const void*)k_stream<K_PLAIN, double> : (const void*)k_stream32<K_PLAIN>; break;
        case K_MARGIN: f = f64 ? (const void*)k_stream<K_MARGIN, double> : (const void*)k_stream<K_MARGIN, float>; break;
        default: return hipErrorInvalidValue;
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, f, kBlock, 0);
}

hipError_t radial_max_blocks_per_cu(int* out) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, (const void*)k_stream32_radial, kBlock, 0);
}

hipError_t launch_radial_bounds(const double* V, int n, float* out, hipStream_t stream) {
    hipLaunchKernelGGL(k_radial_bounds, dim3(1), dim3(kWave), 0, stream, V, n, out);
    return hipGetLastError();
}

}  // namespace pipdev
