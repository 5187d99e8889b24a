// Single-polygon streaming screen on the matrix cores (float32 points).
//
// The n margins of 32 points form one dense product: with rows = edges and
// columns = points,
//     M[i][j] = A_i X_j + B_i Y_j + (-C_i)      (Eq. 11 rearranged, local frame)
// is exactly v_mfma_f32_32x32x2f32 with A = [A_i, B_i] (32 x 2), B = [X_j; Y_j]
// (2 x 32) and the accumulator input preset to -C_i; polygons of up to 64
// edges take two such products per 32 points.  The vector units then only
// reduce each point's margins (max over edges; for sign of offset, whose rows
// are oriented so that the inner side is positive, the min), evaluate the
// band and pack the labels.
//
// Operand layout (gfx950, verified on the device): lane l supplies A[l%32][l/32]
// and B[l/32][l%32]; accumulator register r of lane l holds row
// 8(r/4) + 4(l/32) + r%4 of column l%32.  Points are loaded exactly as in the
// vector kernel (lane l holds point 64 j + l of slot j, 512 contiguous bytes
// per load instruction).  One v_permlane32_swap of the local X and Y
// registers yields the B operands of both 32-point groups of a slot: group A
// (points 0-31: X of lane l, Y of lane l - 32) and group B (points 32-63: X of
// lane l + 32, Y of lane l).  After the reductions, one more swap pairs the two
// half-wave maxima so that lane l ends with the full max of its own point
// (group A in lanes 0-31, group B in lanes 32-63); the band, the decision and
// the ballot are then per lane as in the vector kernel, and the ballot is the
// slot's 64 label bits.
//
// Band: as for the two-fma screen with 6.05 u instead of 4.05 u (the matrix
// core's sum of three terms is bounded by 4 u of the sum of |terms|; measured
// worst 1.96 u).  Undecided points are queued with their coordinates and
// re-decided in binary64 exactly as in the vector kernel.
#include "device.hpp"
#include "kernels.hpp"
#include "stream32.hpp"

using namespace pipdev;

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr double kMfmaFactor = kMfmaScreenFactor;

// max / min of the first R accumulator registers of one product, written as
// a chain whose every step combines three values, so it compiles to v_max3 /
// v_min3 without canonicalising the matrix-core results first (an odd
// remainder repeats register 0).  A NaN margin comes with a NaN or infinite
// band and goes to the binary64 path, so NaN propagation does not matter.
template <int R>
__device__ __forceinline__ float reg_max(const floatx16& d) {
    float r = fmaxf(fmaxf(d[0], d[1]), d[2]);
#pragma unroll
    for (int i = 3; i < R; i += 2) r = fmaxf(fmaxf(r, d[i]), d[i + 1 < R ? i + 1 : 0]);
    return r;
}
// the first product's max continued over the second product (one chain)
__device__ __forceinline__ float reg_max_cont(float r, const floatx16& d) {
#pragma unroll
    for (int i = 0; i < 16; i += 2) r = fmaxf(fmaxf(r, d[i]), d[i + 1]);
    return r;
}
template <int R>
__device__ __forceinline__ float reg_min(const floatx16& d) {
    float r = fminf(fminf(d[0], d[1]), d[2]);
#pragma unroll
    for (int i = 3; i < R; i += 2) r = fminf(fminf(r, d[i]), d[i + 1 < R ? i + 1 : 0]);
    return r;
}
__device__ __forceinline__ float reg_min_cont(float r, const floatx16& d) {
#pragma unroll
    for (int i = 0; i < 16; i += 2) r = fminf(fminf(r, d[i]), d[i + 1]);
    return r;
}

// lane l < 32: (a[l], a[l + 32]); lane l >= 32: (b[l - 32], b[l])
__device__ __forceinline__ void swap_halves(float a, float b, float& lo, float& hi) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                    false);
    lo = __uint_as_float(r[0]);
    hi = __uint_as_float(r[1]);
}

// NE: edge capacity (8, 16, 32, 64).  For NE <= 16 the edges are placed in
// both row halves (row -> edge 4 (row / 8) + row % 4), so register r of every
// lane holds edge r and each lane sees all margins of its column; NE = 32
// uses the natural row -> edge map (the two halves hold different edges of
// the column); NE = 64 takes two products per group.
template <int KIND, int NE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4)))
void k_stream_mfma(const double* __restrict__ V, int n, const float2* __restrict__ Q, int64_t m,
                   uint32_t* __restrict__ labels, int32_t* __restrict__ status) {
    constexpr int NB = NE == 64 ? 2 : 1;
    constexpr bool kDup = NE <= 16;
    constexpr int RR = kDup ? NE : 16;  // registers reduced per product
    __shared__ PolyLds S;
    __shared__ uint32_t queue_c[kWavesPerBlock][kQueue32];
    __shared__ float queue_x[kWavesPerBlock][kQueue32];
    __shared__ float queue_y[kWavesPerBlock][kQueue32];

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int half = lane >> 5, col = lane & 31;
    const int64_t nfull = m / kChunk32;
    const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
    const int64_t c0 = (int64_t)blockIdx.x * kWavesPerBlock + wv;
    int64_t chunk = c0;
    uint32_t k = 0;

    double2 vt = make_double2(0.0, 0.0);
    if (tid < n) vt = make_double2(V[2 * tid], V[2 * tid + 1]);
    float2 pa[kP32], pb[kP32];
    if (nfull > 0) load_full32(Q, chunk < nfull ? chunk : nfull - 1, lane, pa);

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
    const float KQ = S.KQ, KA = S.KA, KB = S.KB, KC = S.KC, SO = S.SO;
    int qcount = 0;

    // Screen the 8 slots of 64 points of chunk `ch` (this wave's k-th); rem
    // points of it exist (>= 512 for a full chunk).
    auto process = [&](const float2(&p)[kP32], int64_t ch, int64_t rem) {
        const bool full = rem >= kChunk32;
        uint64_t inm[kP32], unc[kP32];
#pragma unroll
        for (int j = 0; j < kP32; ++j) {
            const float X = p[j].x - ox, Y = p[j].y - oy;
            // the band first: X and Y are then free for the operand swap
            const float r2 = fmaf(X, X, Y * Y);
            const float E = fmaf(KQ, r2, fmaf(KA, fabsf(X), fmaf(KB, fabsf(Y), KC)));
            const float sxy = fabsf(X) + fabsf(Y);  // sign of offset's one-sided test
            float bA, bB;  // operands of groups A and B
            swap_halves(X, Y, bA, bB);
            float xA = 0.f, xB = 0.f, nA = 0.f, nB = 0.f;
            if constexpr (NB == 1) {
                floatx16 dA = __builtin_amdgcn_mfma_f32_32x32x2f32(a_op[0], bA, c_op[0], 0, 0, 0);
                floatx16 dB = __builtin_amdgcn_mfma_f32_32x32x2f32(a_op[0], bB, c_op[0], 0, 0, 0);
                // both products in flight before the reductions start
                __builtin_amdgcn_sched_barrier(0);
                if constexpr (KIND == K_SOO) {
                    nA = reg_min<RR>(dA);
                    nB = reg_min<RR>(dB);
                } else {
                    xA = reg_max<RR>(dA);
                    xB = reg_max<RR>(dB);
                }
                if constexpr (kDup && RR < 16) {  // keep every product register live
#if defined(__HIP_DEVICE_COMPILE__)
                    asm volatile("" ::"v"(dA), "v"(dB));
#endif
                }
            } else {
                // 64 edges: the two products of group A, then those of group B
                // (two accumulator sets live at a time, for occupancy)
                auto group = [&](float bop, float& mx, float& mn) {
                    const floatx16 d0 =
                        __builtin_amdgcn_mfma_f32_32x32x2f32(a_op[0], bop, c_op[0], 0, 0, 0);
                    const floatx16 d1 =
                        __builtin_amdgcn_mfma_f32_32x32x2f32(a_op[1], bop, c_op[1], 0, 0, 0);
                    __builtin_amdgcn_sched_barrier(0);
                    if constexpr (KIND == K_SOO)
                        mn = reg_min_cont(reg_min<RR>(d0), d1);
                    else
                        mx = reg_max_cont(reg_max<RR>(d0), d1);
                };
                group(bA, xA, nA);
                group(bB, xB, nB);
            }
            // max over all edges of this lane's own point (sign of offset,
            // rows oriented so that the inner side is s > 0: the min)
            float mx = 0.f, mn = 0.f;
            if constexpr (kDup) {
                if constexpr (KIND == K_SOO)
                    mn = half ? nB : nA;
                else
                    mx = half ? xB : xA;
            } else {
                float u, w;
                if constexpr (KIND == K_SOO) {
                    swap_halves(nA, nB, u, w);
                    mn = u < w ? u : w;
                } else {
                    swap_halves(xA, xB, u, w);
                    mx = u > w ? u : w;
                }
            }
            uint64_t in, out;
            if constexpr (KIND == K_SOO) {
                // inside: every offset on the inner side; outside: one on the
                // outer side, and fl32(|X| + |Y|) < SO proves one on the inner
                // side (the bound of the polygon's preparation)
                in = __ballot(mn > E);
                out = __ballot(mn < -E) & __ballot(sxy < SO);
            } else {
                in = __ballot(mx < -E);
                out = __ballot(mx > E);
            }
            inm[j] = in;
            unc[j] = ~(in | out);
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
        int nunc = 0;
#pragma unroll
        for (int j = 0; j < kP32; ++j) nunc += __popcll(unc[j]);
        if (nunc != 0) {
            if (qcount + nunc > kQueue32) {  // flush before push (drains the store above)
                flush_queue32<KIND>(S, queue_c[wv], queue_x[wv], queue_y[wv], qcount, labels, lane,
                                    c0, stride);
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
    if (qcount > 0)
        flush_queue32<KIND>(S, queue_c[wv], queue_x[wv], queue_y[wv], qcount, labels, lane, c0,
                            stride);
}

// Diagnostic: the float32 matrix-core multiply-add of the screen above on
// caller-chosen operands.  Entry e (5 floats: A, B, c, X, Y) is row e % 32 of
// the A operand and column e % 32 of the B operand of its group's product,
// with c in the accumulator row e % 32; out[e] is the product's diagonal
// element, A X + B Y + c as v_mfma_f32_32x32x2f32 forms it.
__global__ __launch_bounds__(kWave) void k_mfma_probe(const float* __restrict__ in, int64_t count,
                                                      float* __restrict__ out) {
    const int lane = threadIdx.x;
    const int col = lane & 31, half = lane >> 5;
    const int64_t g0 = (int64_t)blockIdx.x * 32;
    const int64_t e = g0 + col;
    const bool ok = e < count;
    const float* r = in + 5 * (ok ? e : 0);
    const float a = ok ? (half ? r[1] : r[0]) : 0.f;  // A[row col][k = half]
    const float b = ok ? (half ? r[4] : r[3]) : 0.f;  // B[k = half][column col]
    floatx16 c;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int64_t row = g0 + 8 * (q / 4) + 4 * half + (q % 4);
        c[q] = row < count ? in[5 * row + 2] : 0.f;
    }
    const floatx16 d = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
    // the diagonal element (row col, column col) sits in the lane of column
    // col whose half holds row col, register 4 (col / 8) + col % 4
    const int q = 4 * (col / 8) + col % 4;
    float v = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) v = i == q ? d[i] : v;
    if (ok && half == (col % 8) / 4) out[e] = v;
}

template <int KIND, int R>
hipError_t launch_t(const StreamLaunch& L) {
    const int64_t nchunks = (L.m + kChunk32 - 1) / kChunk32;
    const int64_t want = (nchunks + kWavesPerBlock - 1) / kWavesPerBlock;
    int grid = (int)(want < L.max_blocks ? want : L.max_blocks);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL((k_stream_mfma<KIND, R>), dim3(grid), dim3(kBlock), 0, L.stream, L.V, L.n,
                       static_cast<const float2*>(L.Q), L.m, L.labels, L.status);
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

hipError_t launch_mfma_probe(const float* in, int64_t count, float* out, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mfma_probe, dim3((unsigned)((count + 31) / 32)), dim3(kWave), 0, stream,
                       in, count, out);
    return hipGetLastError();
}

hipError_t stream_mfma_max_blocks_per_cu(int kind, int n, int* out) {
    const void* f = kind == K_SOO ? kernel_for<K_SOO>(n) : kernel_for<K_VORONOI>(n);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, f, kBlock, 0);
}

}  // namespace pipdev
