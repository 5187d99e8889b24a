// Batched Voronoi inclusion: thousands of convex polygons of uneven vertex
// counts, each against its own point set of uneven size, in one persistent
// launch (plus three small set-up kernels).
//
//   k_prepare_batched  one wave per polygon: generators (Section 3,
//                      Algorithms 3-4, binary64), float32 coefficients and
//                      band into the polygon table; chunk count of its set.
//   k_scan_chunks      exclusive scan of the chunk counts (one workgroup).
//   k_fill_chunks      per chunk of 256 points: (first point, polygon, count).
//   k_batched_voronoi  persistent waves walk tiles of G consecutive chunks
//                      (tile t of wave w is t*W + w); polygon coefficients are
//                      staged in the wave's LDS when the polygon changes; the
//                      next chunk's points are always in flight while the
//                      current one is screened (Section 4, Algorithm 5 via
//                      the certified float32 margin), undecided points are
//                      queued and re-decided in binary64.
//
// The precomputed per-polygon tables are the storage the paper suggests for
// static polygons (Section 7: generators stored beside the vertices).
#include "device.hpp"
#include "kernels.hpp"
#include "radial.hpp"
#include "stream32.hpp"

using namespace pipdev;

namespace {

struct alignas(16) ChunkDesc {
    int64_t start;  // global index of the chunk's first point
    int32_t k;      // polygon
    int32_t count;  // points in the chunk (1..512)
};

// buffer resource word 3 of the gfx9 family (raw 32-bit data, no swizzle)
constexpr int kRsrcWord3 = 0x00020000;
constexpr int kLoadNT = 2;  // cache-policy bit of a non-temporal (streaming) load

__global__ __launch_bounds__(kBlock) void k_prepare_batched(BatchedDev D) {
    __shared__ PolyLds S[kWavesPerBlock];
    __shared__ RadialTab RT[kWavesPerBlock];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int64_t k = (int64_t)blockIdx.x * kWavesPerBlock + wv;
    if (k >= D.P) return;  // whole wave
    const int64_t v0 = D.vtx_off[k], v1 = D.vtx_off[k + 1];
    const int64_t p0 = D.pt_off[k], p1 = D.pt_off[k + 1];
    const int64_t nn = v1 - v0;
    // offsets outside the declared arrays: nothing of this polygon is touched
    const bool range_bad = v0 < 0 || v1 < v0 || v1 > D.total_vertices || p0 < 0 || p1 < p0 ||
                           p1 > D.total_points;
    int bad = ST_OK;
    if (range_bad || nn < 3) bad = ST_INVAL;
    else if (nn > kMaxEdges) bad = 6;  // PIP_EUNSUPPORTED
    else if (p1 - p0 > 0xffffffffll) bad = 6;  // recheck queue holds 32-bit point indices
    // an unusable polygon with a valid point range gets all-zero labels
    const int64_t s = range_bad ? 0 : p1 - p0;
    const int64_t chunks = (s + kChunk32 - 1) / kChunk32;
    PolyHdr* H = D.hdr + k;
    if (bad != ST_OK) {
        if (lane == 0) {
            H->n = 0;
            H->n4 = 0;
            H->status = bad;
            H->ox = H->oy = 0.f;
            H->KQ = H->KA = H->KB = H->KC = __builtin_huge_valf();
            H->RQ = 0.f;
            H->radial = 0;
            D.chunk_cnt[k] = chunks;
            if (D.status) D.status[k] = bad;
        }
        return;
    }
    const int n = (int)nn;
    PolyLds& L = S[wv];
    if (lane < n) L.vtx[lane] = make_double2(D.V[2 * (v0 + lane)], D.V[2 * (v0 + lane) + 1]);
    if (lane == 0) L.n = n;
    __builtin_amdgcn_wave_barrier();
    prepare_polygon(L, K_VORONOI, lane);
    __builtin_amdgcn_wave_barrier();
    const int n4 = L.n4;
    float4* C = D.coef + coef_base(D.vtx_off, k);
    if (lane < n4) C[lane] = L.coef[lane];
    double2* G = D.gen + gen_base(D.vtx_off, k);
    for (int i = lane; i <= n; i += kWave) G[i] = L.gen[i];
    // radial pre-screen thresholds (radial.hpp), for polygons large enough
    int radial = 0;
    if (D.radial_min > 0 && n >= D.radial_min) {
        RadialTab& T = RT[wv];
        prepare_radial(L, lane, T);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        float* row = D.radial + k * kRadialRow;
        if (lane < 8) {
            row[2 * lane] = T.t[lane].x;
            row[2 * lane + 1] = T.t[lane].y;
        }
        if (lane == 0) row[16] = T.tfar;
        radial = T.tfar > 0.0f ? 1 : 0;  // a usable table has a positive far limit
    }
    if (lane == 0) {
        H->radial = radial;
        H->ox = L.ox;
        H->oy = L.oy;
        H->KQ = L.KQ;
        H->KA = L.KA;
        H->KB = L.KB;
        H->KC = L.KC;
        H->RQ = L.RQ;
        H->n = n;
        H->n4 = n4;
        H->status = L.status;
        D.chunk_cnt[k] = chunks;
        if (D.status) D.status[k] = L.status;
    }
}

// Exclusive scan of chunk_cnt[P] into chunk_off[P+1]; chunk_off[P] = total.
__global__ __launch_bounds__(1024) void k_scan_chunks(BatchedDev D) {
    __shared__ int64_t wsum[16];
    __shared__ int64_t carry_s;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid == 0) carry_s = 0;
    __syncthreads();
    for (int64_t base = 0; base < D.P; base += 1024) {
        const int64_t i = base + tid;
        const int64_t v = i < D.P ? D.chunk_cnt[i] : 0;
        int64_t x = v;  // inclusive scan within the wave
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wv] = x;
        __syncthreads();
        if (wv == 0) {
            int64_t t = lane < 16 ? wsum[lane] : 0;
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) {
                const int64_t y = __shfl_up(t, o, 64);
                if (lane >= o) t += y;
            }
            if (lane < 16) wsum[lane] = t;  // inclusive over waves
        }
        __syncthreads();
        const int64_t before = (wv ? wsum[wv - 1] : 0) + carry_s;
        if (i < D.P) D.chunk_off[i] = before + x - v;
        __syncthreads();
        if (tid == 0) carry_s += wsum[15];
        __syncthreads();
    }
    if (tid == 0) {
        int64_t total = carry_s;
        if (total > D.max_chunks) total = D.max_chunks;  // never beyond the descriptor array
        D.chunk_off[D.P] = carry_s;
        D.misc[0] = total;
    }
}

__global__ __launch_bounds__(kBlock) void k_fill_chunks(BatchedDev D) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t k = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (k >= D.P) return;
    const int64_t c0 = D.chunk_off[k], c1 = D.chunk_off[k + 1];
    const int64_t p0 = D.pt_off[k];
    const int64_t s = (c1 - c0) > 0 ? D.pt_off[k + 1] - p0 : 0;
    ChunkDesc* desc = reinterpret_cast<ChunkDesc*>(D.desc);
    for (int64_t c = c0 + lane; c < c1 && c < D.max_chunks; c += kWave) {
        const int64_t first = (c - c0) * kChunk32;
        const int64_t cnt = s - first < kChunk32 ? s - first : kChunk32;
        ChunkDesc d;
        d.start = p0 + first;
        d.k = (int32_t)k;
        d.count = (int32_t)cnt;
        desc[c] = d;
    }
}

// Read-only tables of the main kernel, passed as separate __restrict__
// arguments so that loads at wave-uniform addresses become scalar loads.
struct MainArgs {
    const ChunkDesc* __restrict__ desc;
    const PolyHdr* __restrict__ hdr;
    const float4* __restrict__ coef;
    const double2* __restrict__ gen;
    const int64_t* __restrict__ vtx_off;
    const int64_t* __restrict__ pt_off;
    const int64_t* __restrict__ lbl_word_off;
};

// Queue of undecided points of a wave: polygon, index within the polygon's
// point set, and the coordinates as loaded (no second read from HBM).
struct QueueB {
    int32_t k[kQueueCap];
    uint32_t local[kQueueCap];
    float x[kQueueCap], y[kQueueCap];
};

// Re-decide queued (point, polygon) pairs in binary64 against the stored
// generators and set their inside bits.
__device__ void flush_batched(const int64_t* __restrict__ vtx_off,
                              const int64_t* __restrict__ lbl_word_off,
                              const PolyHdr* __restrict__ hdr, const double2* __restrict__ gen,
                              uint32_t* __restrict__ labels, const QueueB& q, int count, int lane) {
    wave_drain();
    for (int e = lane; e < count; e += kWave) {
        const int32_t k = q.k[e];
        const uint32_t local = q.local[e];
        const int n = hdr[k].n;
        const bool in = voronoi64((double)q.x[e], (double)q.y[e], gen + gen_base(vtx_off, k), n);
        if (in) or_label_bit(labels, lbl_word_off[k] + (local >> 5), local & 31u);
    }
    __builtin_amdgcn_wave_barrier();
}

// Points of one chunk: a buffer resource spanning exactly its count points,
// so lanes past the end read 0 without any per-lane address arithmetic.
__device__ __forceinline__ void load_chunk_b(const float2* __restrict__ Q, const ChunkDesc& d,
                                             int lane, float2 (&p)[kP32]) {
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float2*>(Q + d.start), (short)0, d.count * (int)sizeof(float2), kRsrcWord3);
#pragma unroll
    for (int j = 0; j < kP32; ++j) {
        const vfloat2 v = __builtin_bit_cast(
            vfloat2, __builtin_amdgcn_raw_buffer_load_b64(r, (lane + kWave * j) * (int)sizeof(float2),
                                                          0, kLoadNT));
        p[j] = make_float2(v.x, v.y);
    }
}

// RADIAL: the batch holds polygons that take the radial pre-screen; without
// them the kernel carries no radial state (fewer scalar registers live).
template <bool RADIAL>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5))) void k_batched_voronoi(
    const ChunkDesc* __restrict__ desc, const PolyHdr* __restrict__ hdr,
    const float4* __restrict__ coef, const double2* __restrict__ gen,
    const int64_t* __restrict__ vtx_off, const int64_t* __restrict__ pt_off,
    const int64_t* __restrict__ lbl_word_off, const float2* __restrict__ Q,
    uint32_t* __restrict__ labels, const int64_t* __restrict__ misc,
    const float* __restrict__ radial, int G) {
    __shared__ float4 coefs[kWavesPerBlock][2][kMaxEdges];  // current / next polygon
    __shared__ __align__(16) float rtab[kWavesPerBlock][2][kRadialRow];  // their radial thresholds
    __shared__ float2 cpt[kWavesPerBlock][kWave];             // compacted annulus points
    __shared__ int32_t cres[kWavesPerBlock][kWave];           // and their decisions
    __shared__ QueueB queue[kWavesPerBlock];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t W = (int64_t)gridDim.x * kWavesPerBlock;
    const int64_t w = (int64_t)blockIdx.x * kWavesPerBlock + wv;
    const int64_t nchunks = misc[0];
    // a tile never exceeds an even share of the chunks, so the largest tile
    // shape means one contiguous range per wave
    const int64_t share = (nchunks + W - 1) / W;
    if (G > share) G = (int)(share > 0 ? share : 1);

    int64_t tile = w;
    int64_t g = tile * G;
    if (g >= nchunks) return;  // whole wave, nothing to do
    ChunkDesc d = desc[g];
    float2 pa[kP32], pb[kP32];
    load_chunk_b(Q, d, lane, pa);
    int cb = 0;  // LDS table of the current polygon; rows past n4 are never read
    coefs[wv][1][lane] = coef[coef_base(vtx_off, d.k) + lane];
    if (RADIAL && lane < kRadialRow) rtab[wv][1][lane] = radial[(int64_t)d.k * kRadialRow + lane];

    int cur_k = -1;
    // band of the current polygon: KQ r2 + KS (|X| + |Y|) + KC with
    // KS = max(KA, KB) (at least the band), and its fold radius RQ
    float ox = 0.f, oy = 0.f, KQ = 0.f, KS = 0.f, KC = 0.f, RQ = 0.f;
    int n4 = 0, ne = 0;  // edge rows: padded to 4, and evaluated (n rounded up to 2)
    int use_radial = 0;
    int64_t ptk = 0, wk = 0;
    int qcount = 0;
    QueueB& q = queue[wv];

    // Screen chunk `cd` (points p) against polygon cur_k.
    auto process = [&](const float2(&p)[kP32], const ChunkDesc& cd) {
        const int cnt = __builtin_amdgcn_readfirstlane(cd.count);
        const bool full = cnt >= kChunk32;
        uint64_t inm[kP32], unc[kP32];
        if (RADIAL && use_radial) {
            // Radial pre-screen (radial.hpp): most points are decided from r2
            // against their octant's radii; the rest are compacted one per lane
            // and screened against every edge, 64 at a time.
            const float* T = rtab[wv][cb];
            const float tfar = T[16];
            uint64_t amb[kP32];
#pragma unroll
            for (int j = 0; j < kP32; ++j) {
                const float X = p[j].x - ox, Y = p[j].y - oy;
                const float r2 = fmaf(X, X, Y * Y);
                const uint32_t o = ((__float_as_uint(X) >> 31) << 2) | ((__float_as_uint(Y) >> 31) << 1) |
                                   (fabsf(Y) > fabsf(X) ? 1u : 0u);
                const float2 t = *reinterpret_cast<const float2*>(T + 2 * o);
                inm[j] = __ballot(r2 < t.x);
                amb[j] = ~(inm[j] | __ballot((r2 > t.y) & (r2 < tfar)));
                unc[j] = 0;
            }
            if (!full) {
#pragma unroll
                for (int j = 0; j < kP32; ++j) {
                    const uint64_t vm = __ballot(lane + kWave * j < cnt);
                    inm[j] &= vm;
                    amb[j] &= vm;
                }
            }
            int na = 0;
#pragma unroll
            for (int j = 0; j < kP32; ++j) na += __popcll(amb[j]);
            const uint64_t lt = lanemask_lt();
            for (int base = 0; base < na; base += kWave) {
                int run = 0;  // rank of a lane's point among the chunk's annulus points
#pragma unroll
                for (int j = 0; j < kP32; ++j) {
                    const int rank = run + __popcll(amb[j] & lt) - base;
                    if (((amb[j] >> lane) & 1ull) && rank >= 0 && rank < kWave) cpt[wv][rank] = p[j];
                    run += __popcll(amb[j]);
                }
                __builtin_amdgcn_wave_barrier();
                const int cntp = min(na - base, kWave);
                int res = 0;  // 1 inside, 2 inside the band
                if (lane < cntp) {
                    const float2 qq = cpt[wv][lane];
                    const float X = qq.x - ox, Y = qq.y - oy;
                    const float4* cf = coefs[wv][cb];
                    float M = -__builtin_huge_valf();
                    for (int e = 0; e < n4; e += 4) {
                        const float4 c0 = cf[e + 0], c1 = cf[e + 1], c2 = cf[e + 2], c3 = cf[e + 3];
                        const float m0 = fmaf(c0.x, X, fmaf(c0.y, Y, c0.z));
                        const float m1 = fmaf(c1.x, X, fmaf(c1.y, Y, c1.z));
                        const float m2 = fmaf(c2.x, X, fmaf(c2.y, Y, c2.z));
                        const float m3 = fmaf(c3.x, X, fmaf(c3.y, Y, c3.z));
                        M = fmaxf(fmaxf(M, m0), m1);
                        M = fmaxf(fmaxf(M, m2), m3);
                    }
                    const float r2 = fmaf(X, X, Y * Y);
                    const float E = fmaf(KQ, r2, fmaf(KS, fabsf(X) + fabsf(Y), KC));
                    res = M < -E ? 1 : (M > E ? 0 : 2);
                }
                cres[wv][lane] = res;
                __builtin_amdgcn_wave_barrier();
                run = 0;
#pragma unroll
                for (int j = 0; j < kP32; ++j) {
                    const int rank = run + __popcll(amb[j] & lt) - base;
                    const bool mine = ((amb[j] >> lane) & 1ull) && rank >= 0 && rank < kWave;
                    const int r = mine ? cres[wv][rank] : 0;
                    inm[j] |= __ballot(r == 1);
                    unc[j] |= __ballot(r == 2);
                    run += __popcll(amb[j]);
                }
                __builtin_amdgcn_wave_barrier();
            }
        } else if (ne > 0) {
            float X[kP32], Y[kP32], Mx[kP32];
            {  // edges 0-3 (n4 >= 4) start the max
                const float4* cf = coefs[wv][cb];
                const float4 c0 = cf[0], c1 = cf[1], c2 = cf[2], c3 = cf[3];
#pragma unroll
                for (int j = 0; j < kP32; ++j) {
                    X[j] = p[j].x - ox;
                    Y[j] = p[j].y - oy;
                    const float m0 = fmaf(c0.x, X[j], fmaf(c0.y, Y[j], c0.z));
                    const float m1 = fmaf(c1.x, X[j], fmaf(c1.y, Y[j], c1.z));
                    const float m2 = fmaf(c2.x, X[j], fmaf(c2.y, Y[j], c2.z));
                    const float m3 = fmaf(c3.x, X[j], fmaf(c3.y, Y[j], c3.z));
                    Mx[j] = fmaxf(fmaxf(fmaxf(m0, m1), m2), m3);
                }
            }
            // rows 4.. in fours, then a last pair: n rounded up to 2 rows are
            // evaluated (a pad row repeats edge 0 and leaves the max unchanged)
            int e = 4;
            for (; e + 4 <= ne; e += 4) {
                const float4* cf = coefs[wv][cb];
                const float4 c0 = cf[e + 0], c1 = cf[e + 1], c2 = cf[e + 2], c3 = cf[e + 3];
#pragma unroll
                for (int j = 0; j < kP32; ++j) {
                    const float m0 = fmaf(c0.x, X[j], fmaf(c0.y, Y[j], c0.z));
                    const float m1 = fmaf(c1.x, X[j], fmaf(c1.y, Y[j], c1.z));
                    const float m2 = fmaf(c2.x, X[j], fmaf(c2.y, Y[j], c2.z));
                    const float m3 = fmaf(c3.x, X[j], fmaf(c3.y, Y[j], c3.z));
                    Mx[j] = fmaxf(fmaxf(Mx[j], m0), m1);
                    Mx[j] = fmaxf(fmaxf(Mx[j], m2), m3);
                }
            }
            if (e < ne) {
                const float4* cf = coefs[wv][cb];
                const float4 c0 = cf[e + 0], c1 = cf[e + 1];
#pragma unroll
                for (int j = 0; j < kP32; ++j) {
                    const float m0 = fmaf(c0.x, X[j], fmaf(c0.y, Y[j], c0.z));
                    const float m1 = fmaf(c1.x, X[j], fmaf(c1.y, Y[j], c1.z));
                    Mx[j] = fmaxf(fmaxf(Mx[j], m0), m1);
                }
            }
            // band: when |X| + |Y| <= RQ for every point of the chunk, the
            // quadratic term is inside the linear constants and
            // E = max(KA, KB) (|X| + |Y|) + KC (wave-uniform branch; a NaN sum
            // is dropped by the max and gives a NaN band: undecided)
            float sxy[kP32];
            float acc = 0.0f;
#pragma unroll
            for (int j = 0; j < kP32; ++j) {
                sxy[j] = fabsf(X[j]) + fabsf(Y[j]);
                acc = fmaxf(acc, sxy[j]);
            }
            if (__ballot(acc > RQ) == 0) {
#pragma unroll
                for (int j = 0; j < kP32; ++j) {
                    const float E = fmaf(KS, sxy[j], KC);
                    const uint64_t in = __ballot(Mx[j] < -E), out = __ballot(Mx[j] > E);
                    inm[j] = in;
                    unc[j] = ~(in | out);
                }
            } else {
#pragma unroll
                for (int j = 0; j < kP32; ++j) {
                    const float r2 = fmaf(X[j], X[j], Y[j] * Y[j]);
                    const float E = fmaf(KQ, r2, fmaf(KS, sxy[j], KC));
                    const uint64_t in = __ballot(Mx[j] < -E), out = __ballot(Mx[j] > E);
                    inm[j] = in;
                    unc[j] = ~(in | out);
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < kP32; ++j) inm[j] = unc[j] = 0;  // invalid polygon: labels 0
        }
        if (!full) {
#pragma unroll
            for (int j = 0; j < kP32; ++j) {
                const uint64_t vm = __ballot(lane + kWave * j < cnt);
                inm[j] &= vm;
                unc[j] &= vm;
            }
        }
        const int64_t local = cd.start - ptk;  // multiple of 512
        const uint32_t wd = chunk_word32(inm);
        const int nw = full ? kWords32 : (cnt + 31) / 32;
        if (lane < nw) labels[wk + local / 32 + lane] = wd;
        // queue in two halves of at most 256 points (flush before push)
        const uint64_t lt = lanemask_lt();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            int c = 0;
#pragma unroll
            for (int j = 4 * h; j < 4 * h + 4; ++j) c += __popcll(unc[j]);
            if (c == 0) continue;
            if (qcount + c > kQueueCap) {  // drains this chunk's store too
                flush_batched(vtx_off, lbl_word_off, hdr, gen, labels, q, qcount, lane);
                qcount = 0;
            }
#pragma unroll
            for (int j = 4 * h; j < 4 * h + 4; ++j) {
                if (unc[j] == 0) continue;  // wave-uniform: no undecided point in this slot
                if ((unc[j] >> lane) & 1ull) {
                    const int slot = qcount + __popcll(unc[j] & lt);
                    q.k[slot] = cur_k;
                    q.local[slot] = (uint32_t)(local + lane + kWave * j);
                    q.x[slot] = p[j].x;
                    q.y[slot] = p[j].y;
                }
                qcount += __popcll(unc[j]);
            }
        }
    };
    // Polygon table of chunk `cd` (its coefficient rows are in the other LDS
    // table, written when its first chunk was prefetched).
    auto stage = [&](const ChunkDesc& cd) {
        const int k = __builtin_amdgcn_readfirstlane(cd.k);
        if (k == cur_k) return;
        const PolyHdr& H = hdr[k];
        ox = H.ox;
        oy = H.oy;
        KQ = H.KQ;
        KS = fmaxf(H.KA, H.KB);
        KC = H.KC;
        RQ = H.RQ;
        n4 = __builtin_amdgcn_readfirstlane(H.n4);
        ne = (__builtin_amdgcn_readfirstlane(H.n) + 1) & ~1;
        use_radial = RADIAL ? __builtin_amdgcn_readfirstlane(H.radial) : 0;
        ptk = pt_off[k];
        wk = lbl_word_off[k];
        cb ^= 1;
        __builtin_amdgcn_wave_barrier();
        cur_k = k;
    };
    // the chunk after gg in this wave's sequence; pos is gg's place in its
    // tile (a counter instead of a 64-bit remainder per chunk)
    auto next_chunk = [&](int64_t gg, int& pos) -> int64_t {
        if (pos + 1 < G && gg + 1 < nchunks) {
            ++pos;
            return gg + 1;
        }
        tile += W;
        pos = 0;
        return tile * G;
    };

    // Descriptors travel by vector load, issued after the point prefetch, so
    // that waiting for the next one coincides with waiting for the points
    // that are screened next (no scalar-load latency before each prefetch).
    auto load_desc_v = [&](int64_t gg) {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<ChunkDesc*>(desc + gg), (short)0, (int)sizeof(ChunkDesc), kRsrcWord3);
        return __builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0);
    };
    auto unpack = [&](const decltype(load_desc_v(0))& v) {
        ChunkDesc c;
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)v[0]);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)v[1]);
        c.start = (int64_t)(((uint64_t)hi << 32) | lo);
        c.k = __builtin_amdgcn_readfirstlane((int)v[2]);
        c.count = __builtin_amdgcn_readfirstlane((int)v[3]);
        return c;
    };
    const int64_t g0 = g;  // a valid index for the descriptor loads past the end
    int pos2 = 0;          // place of g2 (then g3) in its tile
    int64_t g2 = next_chunk(g, pos2);
    bool more = g2 < nchunks;
    auto d2v = load_desc_v(more ? g2 : g0);

    for (;;) {
        stage(d);
        ChunkDesc d2 = unpack(d2v);
        {  // a new polygon's rows go to the spare LDS table (load issued first)
            const bool newpoly = d2.k != d.k;
            float4 cn = make_float4(0.f, 0.f, 0.f, 0.f);
            float rn = 0.f;
            if (newpoly) cn = coef[coef_base(vtx_off, d2.k) + lane];
            if (RADIAL && newpoly && lane < kRadialRow) rn = radial[(int64_t)d2.k * kRadialRow + lane];
            load_chunk_b(Q, d2, lane, pb);
            if (newpoly) coefs[wv][cb ^ 1][lane] = cn;
            if (RADIAL && newpoly && lane < kRadialRow) rtab[wv][cb ^ 1][lane] = rn;
        }
        int64_t g3 = more ? next_chunk(g2, pos2) : g2;
        bool more3 = more && g3 < nchunks;
        d2v = load_desc_v(more3 ? g3 : (more ? g2 : g0));
        process(pa, d);
        if (!more) break;
        d = d2;
        g2 = g3;
        more = more3;

        stage(d);
        d2 = unpack(d2v);
        {
            const bool newpoly = d2.k != d.k;
            float4 cn = make_float4(0.f, 0.f, 0.f, 0.f);
            float rn = 0.f;
            if (newpoly) cn = coef[coef_base(vtx_off, d2.k) + lane];
            if (RADIAL && newpoly && lane < kRadialRow) rn = radial[(int64_t)d2.k * kRadialRow + lane];
            load_chunk_b(Q, d2, lane, pa);
            if (newpoly) coefs[wv][cb ^ 1][lane] = cn;
            if (RADIAL && newpoly && lane < kRadialRow) rtab[wv][cb ^ 1][lane] = rn;
        }
        g3 = more ? next_chunk(g2, pos2) : g2;
        more3 = more && g3 < nchunks;
        d2v = load_desc_v(more3 ? g3 : (more ? g2 : g0));
        process(pb, d);
        if (!more) break;
        d = d2;
        g2 = g3;
        more = more3;
    }
    if (qcount > 0) flush_batched(vtx_off, lbl_word_off, hdr, gen, labels, q, qcount, lane);
}

}  // namespace

namespace pipdev {

size_t batched_workspace_layout(int64_t P, int64_t total_vertices, int64_t total_points,
                                BatchedLayout* L) {
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t off = 0;
    L->hdr = off;
    off = up(off + sizeof(PolyHdr) * (size_t)P);
    L->coef = off;  // + 64 rows: a whole wave may read 64 rows from any polygon's base
    off = up(off + 16 * (size_t)(total_vertices + 3 * P + kWave));
    L->gen = off;
    off = up(off + 16 * (size_t)(total_vertices + P));
    L->chunk_cnt = off;
    off = up(off + 8 * (size_t)P);
    L->chunk_off = off;
    off = up(off + 8 * (size_t)(P + 1));
    L->max_chunks = total_points / kChunk32 + P + 1;
    L->desc = off;
    off = up(off + sizeof(ChunkDesc) * (size_t)L->max_chunks);
    L->misc = off;
    off = up(off + 64);
    L->radial = off;
    off = up(off + sizeof(float) * kRadialRow * (size_t)P);
    return off;
}

hipError_t launch_batched(const BatchedDev& D, int G, int blocks, hipStream_t stream) {
    const int pblocks = (int)((D.P + kWavesPerBlock - 1) / kWavesPerBlock);
    hipLaunchKernelGGL(k_prepare_batched, dim3(pblocks), dim3(kBlock), 0, stream, D);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_chunks, dim3(1), dim3(1024), 0, stream, D);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_fill_chunks, dim3(pblocks), dim3(kBlock), 0, stream, D);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    auto kern = D.radial_min > 0 ? k_batched_voronoi<true> : k_batched_voronoi<false>;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(kBlock), 0, stream,
                       reinterpret_cast<const ChunkDesc*>(D.desc), D.hdr, D.coef, D.gen, D.vtx_off,
                       D.pt_off, D.lbl_word_off, reinterpret_cast<const float2*>(D.Q), D.labels,
                       D.misc, D.radial, G);
    return hipGetLastError();
}

hipError_t batched_max_blocks_per_cu(int* out) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, (const void*)k_batched_voronoi<true>,
                                                        kBlock, 0);
}

}  // namespace pipdev

namespace {
__global__ void k_zero_u64(unsigned long long* out) { *out = 0ull; }

__global__ void k_count_diff(const uint32_t* a, const uint32_t* b, int64_t nwords,
                             unsigned long long* out) {
    unsigned long long local = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords;
         i += (int64_t)gridDim.x * blockDim.x)
        local += (a[i] != b[i]);
    if (local) atomicAdd(out, local);
}
}  // namespace

namespace pipdev {
// *out = number of differing words (the counter is cleared first, in-stream).
hipError_t launch_count_diff(const uint32_t* a, const uint32_t* b, int64_t nwords,
                             unsigned long long* out, hipStream_t stream) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, stream, out);
    hipLaunchKernelGGL(k_count_diff, dim3(1024), dim3(256), 0, stream, a, b, nwords, out);
    return hipGetLastError();
}
}  // namespace pipdev
