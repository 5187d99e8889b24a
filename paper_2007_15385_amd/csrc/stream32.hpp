// Shared pieces of the float32 single-polygon streaming kernels (vector and
// matrix-core screens): chunk geometry, loads, label-word packing and the
// binary64 recheck queue.
#pragma once
#include "device.hpp"

namespace pipdev {

// ----------------------------------------------------------------------------
// float32 points, Voronoi / sign of offset / plain: the bandwidth-bound case.
//
// Each wave owns chunks of kP32 * 64 = 512 points (lane l holds points
// l + 64 j, j < 8, so every 8-byte load instruction of the wave covers 512
// contiguous bytes).  The chunk index is wave-uniform, so addresses are a
// scalar base plus the lane's constant offset; full chunks load without
// clamping and the one partial chunk (if any) is handled after the loop.
// The next chunk is loaded into the other of two register buffers while the
// current one is screened (4 KiB per wave in flight); the last prefetch of a
// wave re-reads its own chunk instead of branching, so every load is
// unconditional and the compiler waits for exactly the previous chunk.
// Ballots come straight from the float32 compares; lane k < 16 stores label
// word k of the chunk (slot j's 64-bit mask is words 2j, 2j + 1).
// ----------------------------------------------------------------------------
constexpr int kP32 = 8;
constexpr int kChunk32 = kWave * kP32;   // 512 points
constexpr int kWords32 = kChunk32 / 32;  // 16 label words
constexpr int kQueue32 = kChunk32;       // one whole chunk fits the queue

// Non-temporal loads: the points are read once, and streaming them with the
// nt hint measured about 13% more read bandwidth than ordinary loads.
__device__ __forceinline__ void load_full32(const float2* __restrict__ Q, int64_t chunk, int lane,
                                            float2 (&p)[kP32]) {
    const vfloat2* q = reinterpret_cast<const vfloat2*>(Q) + chunk * kChunk32 + lane;
#pragma unroll
    for (int j = 0; j < kP32; ++j) {
        const vfloat2 v = __builtin_nontemporal_load(q + kWave * j);
        p[j] = make_float2(v.x, v.y);
    }
}

// Label words of a chunk into one VGPR: lane k < 16 gets word k (slot j's
// 64-bit mask is words 2j, 2j + 1).  v_writelane_b32 copies a scalar into
// one lane, ignoring exec; the lane selects are constants.
#define PIP_WRITELANE(w, sv, L) \
    asm volatile("v_writelane_b32 %0, %1, " #L : "+v"(w) : "s"(sv))

__device__ __forceinline__ uint32_t chunk_word32(const uint64_t (&mk)[kP32]) {
    uint32_t w = 0;
    PIP_WRITELANE(w, (uint32_t)mk[0], 0);
    PIP_WRITELANE(w, (uint32_t)(mk[0] >> 32), 1);
    PIP_WRITELANE(w, (uint32_t)mk[1], 2);
    PIP_WRITELANE(w, (uint32_t)(mk[1] >> 32), 3);
    PIP_WRITELANE(w, (uint32_t)mk[2], 4);
    PIP_WRITELANE(w, (uint32_t)(mk[2] >> 32), 5);
    PIP_WRITELANE(w, (uint32_t)mk[3], 6);
    PIP_WRITELANE(w, (uint32_t)(mk[3] >> 32), 7);
    PIP_WRITELANE(w, (uint32_t)mk[4], 8);
    PIP_WRITELANE(w, (uint32_t)(mk[4] >> 32), 9);
    PIP_WRITELANE(w, (uint32_t)mk[5], 10);
    PIP_WRITELANE(w, (uint32_t)(mk[5] >> 32), 11);
    PIP_WRITELANE(w, (uint32_t)mk[6], 12);
    PIP_WRITELANE(w, (uint32_t)(mk[6] >> 32), 13);
    PIP_WRITELANE(w, (uint32_t)mk[7], 14);
    PIP_WRITELANE(w, (uint32_t)(mk[7] >> 32), 15);
    return w;
}
#undef PIP_WRITELANE

// Queue entries of the float32 kernel: code = (k << 9) | r for point r of the
// wave's k-th chunk (chunk c0 + k * stride), and the coordinates as loaded.
template <int KIND>
__device__ inline void flush_queue32(const PolyLds& S, const uint32_t* qc, const float* qx,
                              const float* qy, int count, uint32_t* labels, int lane, int64_t c0,
                              int64_t stride) {
    wave_drain();
    for (int e = lane; e < count; e += kWave) {
        const uint32_t code = qc[e];
        const int64_t idx = (c0 + (int64_t)(code >> 9) * stride) * kChunk32 + (code & 511u);
        const double x = (double)qx[e], y = (double)qy[e];
        bool in;
        if constexpr (KIND == K_VORONOI)
            in = voronoi64(x, y, S.gen, S.n);
        else if constexpr (KIND == K_RAY)
            in = ray_crossing64(x, y, S.ray, S.rhs, S.n);
        else
            in = sign_of_offset64(x, y, S.vtx, S.n);
        if (in) or_label_bit(labels, idx >> 5, (uint32_t)(idx & 31));
    }
    __builtin_amdgcn_wave_barrier();
}

}  // namespace pipdev
