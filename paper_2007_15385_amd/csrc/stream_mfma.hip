// Single-polygon streaming screen on the matrix cores (float32 points).
//
// The n margins of 32 points form one dense product: with rows = edges and
// columns = points,
//     M[i][j] = A_i X_j + B_i Y_j + (-C_i)      (Eq. 11 rearranged, local frame)
// is exactly v_mfma_f32_32x32x2f32 with A = [A_i, B_i] (32 x 2), B = [X_j; Y_j]
// (2 x 32) and the accumulator input preset to -C_i; polygons of up to 64
// edges take two such products per 32 points.  The vector units then only
// reduce each point's margins (max over edges; max and min for sign of
// offset), evaluate the band and pack the labels.
//
// Operand layout (gfx950, verified on the device): lane l supplies A[l%32][l/32]
// and B[l/32][l%32]; accumulator register r of lane l holds row
// 8(r/4) + 4(l/32) + r%4 of column l%32.  Lanes l and l + 32 both load point
// l%32 (x and y) and feed X or Y into the product; every lane computes the
// band of its point itself.  Rows beyond n repeat edge 0 (the max is
// unchanged).  Both lanes of a point end with the same max and band, so they
// take the same decision and the low 32 bits of a ballot are that point
// group's label word.
//
// Band: as for the two-fma screen with 6.05 u instead of 4.05 u (the matrix
// core's sum of three terms is bounded by 4 u of the sum of |terms|; measured
// worst 1.96 u).  Undecided points are queued with their coordinates and
// re-decided in binary64 exactly as in the vector kernel.
#include "device.hpp"
#include "kernels.hpp"

using namespace pipdev;

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kGroups = kChunk / 32;  // 8 point groups of 32 per 256-point chunk
constexpr double kMfmaFactor = 6.05;

// The two outputs of the swap hold the two half-wave values of a column in
// both halves; a compare-select (no NaN canonicalisation needed: a NaN margin
// only occurs with a NaN band, which already forces the binary64 path).
__device__ __forceinline__ float pair_max(float v) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false,
                                                    false);
    const float a = __uint_as_float(r[0]), b = __uint_as_float(r[1]);
    return a > b ? a : b;
}
__device__ __forceinline__ float pair_min(float v) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false,
                                                    false);
    const float a = __uint_as_float(r[0]), b = __uint_as_float(r[1]);
    return a < b ? a : b;
}
template <int KIND>
__device__ void flush_mfma(const PolyLds& S, const int64_t* qi, const float2* qp, int count,
                           uint32_t* labels, int lane) {
    wave_drain();
    for (int e = lane; e < count; e += kWave) {
        const int64_t idx = qi[e];
        const double x = (double)qp[e].x, y = (double)qp[e].y;
        bool in;
        if constexpr (KIND == K_VORONOI)
            in = voronoi64(x, y, S.gen, S.n);
        else
            in = sign_of_offset64(x, y, S.vtx, S.n);
        if (in) or_label_bit(labels, idx >> 5, (uint32_t)(idx & 31));
    }
    __builtin_amdgcn_wave_barrier();
}

// NE: edge capacity (8, 16, 32, 64).  For NE <= 16 the edges are placed in
// both row halves (row -> edge 4 (row / 8) + row % 4), so register r of every
// lane holds edge r and each lane sees all margins of its point; NE = 32 uses
// row = edge (two lanes per point, combined by one swap); NE = 64 uses two
// products.
template <int KIND, int NE>
__global__ __launch_bounds__(kBlock) void k_stream_mfma(const double* __restrict__ V, int n,
                                                      const float* __restrict__ Qf, int64_t m,
                                                      uint32_t* __restrict__ labels,
                                                      int32_t* __restrict__ status) {
    constexpr int NB = NE > 32 ? 2 : 1;
    constexpr bool kDup = NE <= 16;
    constexpr int RR = kDup ? NE : 16;  // registers reduced per product
    __shared__ PolyLds S;
    __shared__ int64_t qidx[kWavesPerBlock][kQueueCap];
    __shared__ float2 qpt[kWavesPerBlock][kQueueCap];

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int half = lane >> 5, col = lane & 31;
    const int64_t nchunks = (m + kChunk - 1) / kChunk;
    const int64_t nwords = (m + 31) / 32;
    const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
    int64_t chunk = (int64_t)blockIdx.x * kWavesPerBlock + wv;
    const float2* __restrict__ Q2 = reinterpret_cast<const float2*>(Qf);

    double2 vt = make_double2(0.0, 0.0);
    if (tid < n) vt = make_double2(V[2 * tid], V[2 * tid + 1]);
    // lane l loads point (group start + l % 32) of each of the 8 groups; full
    // chunks need no clamping (immediate offsets), the last one is clamped
    float2 v[kGroups];
    auto load_chunk = [&](int64_t c, float2 (&dst)[kGroups]) {
        if ((c + 1) * kChunk <= m) {
            const float2* a = Q2 + c * kChunk + col;
#pragma unroll
            for (int t = 0; t < kGroups; ++t) dst[t] = a[32 * t];
        } else {
            const int64_t last = m - 1;
#pragma unroll
            for (int t = 0; t < kGroups; ++t) {
                int64_t p = c * kChunk + 32 * t + col;
                p = p < last ? p : last;
                dst[t] = Q2[p];
            }
        }
    };
    if (m > 0) load_chunk(chunk, v);

    if (tid < n) S.vtx[tid] = vt;
    if (tid == 0) S.n = n;
    __syncthreads();
    if (wv == 0) prepare_polygon(S, KIND, lane, false, kMfmaFactor);
    __syncthreads();
    if (status && blockIdx.x == 0 && tid == 0) *status = S.status;

    // constant operands of this polygon
    auto edge_of_row = [&](int row) -> int {
        const int e = kDup ? 4 * (row / 8) + row % 4 : row;
        return e < n ? e : 0;
    };
    float a_op[NB];
    floatx16 c_op[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const float4 ce = S.coef[edge_of_row(32 * b + col)];
        a_op[b] = half ? ce.y : ce.x;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = 32 * b + 8 * (r / 4) + 4 * half + (r % 4);
            c_op[b][r] = S.coef[edge_of_row(row)].z;
        }
    }
    const float ox = S.ox, oy = S.oy;
    const float KQ = S.KQ, KA = S.KA, KB = S.KB, KC = S.KC;
    int qcount = 0;

    for (; chunk < nchunks; chunk += stride) {
        float2 nv[kGroups];
        load_chunk(chunk + stride, nv);
        const int64_t base = chunk * kChunk;
        // lanes of points past the end (partial last chunk only)
        const uint32_t vmask = (base + kChunk <= m) ? 0xffffffffu : 0u;
        uint32_t inw[kGroups], uncw[kGroups];
        float X[kGroups], Y[kGroups];
#pragma unroll
        for (int t = 0; t < kGroups; ++t) {
            X[t] = v[t].x - ox;
            Y[t] = v[t].y - oy;
        }
        floatx16 dnext[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b)
            dnext[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(a_op[b], half ? Y[0] : X[0], c_op[b], 0,
                                                            0, 0);
#pragma unroll
        for (int t = 0; t < kGroups; ++t) {
            floatx16 d[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) d[b] = dnext[b];
            if (t + 1 < kGroups) {  // next group's products before this group's reduction
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    dnext[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                        a_op[b], half ? Y[t + 1] : X[t + 1], c_op[b], 0, 0, 0);
            }
            float mx = -__builtin_huge_valf(), mn = __builtin_huge_valf();
#pragma unroll
            for (int b = 0; b < NB; ++b) {
#pragma unroll
                for (int r = 0; r < RR; ++r) {
                    mx = fmaxf(mx, d[b][r]);
                    if constexpr (KIND == K_SOO) mn = fminf(mn, d[b][r]);
                }
            }
            if constexpr (!kDup) {
                mx = pair_max(mx);
                if constexpr (KIND == K_SOO) mn = pair_min(mn);
            }
            const float ax = fabsf(X[t]), ay = fabsf(Y[t]);
            const float r2 = fmaf(X[t], X[t], Y[t] * Y[t]);
            const float E = fmaf(KQ, r2, fmaf(KA, ax, fmaf(KB, ay, KC)));
            uint32_t ins, outs;
            if constexpr (KIND == K_SOO) {
                ins = (uint32_t)__ballot(mx < -E) | (uint32_t)__ballot(mn > E);
                outs = (uint32_t)__ballot(mx > E) & (uint32_t)__ballot(mn < -E);
            } else {
                ins = (uint32_t)__ballot(mx < -E);
                outs = (uint32_t)__ballot(mx > E);
            }
            uint32_t valid = vmask;
            if (!vmask) {
                const int64_t rem = m - (base + 32 * t);
                valid = rem >= 32 ? 0xffffffffu : (rem <= 0 ? 0u : ((1u << rem) - 1u));
            }
            inw[t] = ins & valid;
            uncw[t] = ~(ins | outs) & valid;
        }
        int nunc = 0;
#pragma unroll
        for (int t = 0; t < kGroups; ++t) nunc += __popc(uncw[t]);
        if (nunc != 0 && qcount + nunc > kQueueCap) {  // flush before push
            flush_mfma<KIND>(S, qidx[wv], qpt[wv], qcount, labels, lane);
            qcount = 0;
        }
        // lane k (< 8) stores word k of the chunk
        uint32_t w = 0;
#pragma unroll
        for (int t = 0; t < kGroups; ++t) w = (lane == t) ? inw[t] : w;
        const int64_t widx = base / 32 + lane;
        if (lane < kWordsPerChunk && widx < nwords) labels[widx] = w;
        if (nunc != 0) {
            const uint32_t lt = (uint32_t)lanemask_lt();
#pragma unroll
            for (int t = 0; t < kGroups; ++t) {
                if (uncw[t]) {
                    if (half == 0 && ((uncw[t] >> col) & 1u)) {
                        const int slot = qcount + __popc(uncw[t] & lt);
                        qidx[wv][slot] = base + 32 * t + col;
                        qpt[wv][slot] = v[t];
                    }
                    qcount += __popc(uncw[t]);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < kGroups; ++t) v[t] = nv[t];
    }
    if (qcount > 0) flush_mfma<KIND>(S, qidx[wv], qpt[wv], qcount, labels, lane);
}

template <int KIND, int R>
hipError_t launch_t(const StreamLaunch& L) {
    const int64_t nchunks = (L.m + kChunk - 1) / kChunk;
    const int64_t want = (nchunks + kWavesPerBlock - 1) / kWavesPerBlock;
    int grid = (int)(want < L.max_blocks ? want : L.max_blocks);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL((k_stream_mfma<KIND, R>), dim3(grid), dim3(kBlock), 0, L.stream, L.V, L.n,
                       static_cast<const float*>(L.Q), L.m, L.labels, L.status);
    return hipGetLastError();
}

template <int KIND>
hipError_t launch_kind(const StreamLaunch& L) {
    if (L.n <= 8) return launch_t<KIND, 8>(L);
    if (L.n <= 16) return launch_t<KIND, 16>(L);
    if (L.n <= 32) return launch_t<KIND, 32>(L);
    return launch_t<KIND, 64>(L);
}

template <int KIND>
const void* kernel_for(int n) {
    if (n <= 8) return (const void*)k_stream_mfma<KIND, 8>;
    if (n <= 16) return (const void*)k_stream_mfma<KIND, 16>;
    if (n <= 32) return (const void*)k_stream_mfma<KIND, 32>;
    return (const void*)k_stream_mfma<KIND, 64>;
}

}  // namespace

namespace pipdev {

hipError_t launch_stream_mfma(const StreamLaunch& L) {
    return L.kind == K_SOO ? launch_kind<K_SOO>(L) : launch_kind<K_VORONOI>(L);
}

hipError_t stream_mfma_max_blocks_per_cu(int kind, int n, int* out) {
    const void* f = kind == K_SOO ? kernel_for<K_SOO>(n) : kernel_for<K_VORONOI>(n);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, f, kBlock, 0);
}

}  // namespace pipdev
