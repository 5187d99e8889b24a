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

using namespace pipdev;

namespace {

struct alignas(16) ChunkDesc {
    int64_t start;  // global index of the chunk's first point
    int32_t k;      // polygon
    int32_t count;  // points in the chunk (1..256)
};

__global__ __launch_bounds__(kBlock) void k_prepare_batched(BatchedDev D) {
    __shared__ PolyLds S[kWavesPerBlock];
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
    // an unusable polygon with a valid point range gets all-zero labels
    const int64_t s = range_bad ? 0 : p1 - p0;
    const int64_t chunks = (s + kChunk - 1) / kChunk;
    PolyHdr* H = D.hdr + k;
    if (bad != ST_OK) {
        if (lane == 0) {
            H->n = 0;
            H->n4 = 0;
            H->status = bad;
            H->ox = H->oy = 0.f;
            H->KQ = H->KA = H->KB = H->KC = __builtin_huge_valf();
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
    if (lane == 0) {
        H->ox = L.ox;
        H->oy = L.oy;
        H->KQ = L.KQ;
        H->KA = L.KA;
        H->KB = L.KB;
        H->KC = L.KC;
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
        const int64_t first = (c - c0) * kChunk;
        const int64_t cnt = s - first < kChunk ? s - first : kChunk;
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

// Re-decide queued (point, polygon) pairs in binary64 against the stored
// generators and set their inside bits.
__device__ void flush_batched(const int64_t* __restrict__ vtx_off, const int64_t* __restrict__ pt_off,
                              const int64_t* __restrict__ lbl_word_off,
                              const PolyHdr* __restrict__ hdr, const double2* __restrict__ gen,
                              const float2* __restrict__ Q, uint32_t* __restrict__ labels,
                              const int64_t* qi, const int32_t* qk, int count, int lane) {
    wave_drain();
    for (int e = lane; e < count; e += kWave) {
        const int64_t idx = qi[e];
        const int32_t k = qk[e];
        const float2 p = Q[idx];
        const int n = hdr[k].n;
        const bool in = voronoi64((double)p.x, (double)p.y, gen + gen_base(vtx_off, k), n);
        const int64_t local = idx - pt_off[k];
        if (in) or_label_bit(labels, lbl_word_off[k] + (local >> 5), (uint32_t)(local & 31));
    }
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void load_points(const float2* __restrict__ Q, int64_t start, int64_t last,
                                            int lane, float (&x)[kPPL], float (&y)[kPPL]) {
#pragma unroll
    for (int j = 0; j < kPPL; ++j) {
        int64_t i = start + lane + kWave * j;
        i = i < last ? i : last;
        const vfloat2 p = __builtin_nontemporal_load(reinterpret_cast<const vfloat2*>(Q) + i);
        x[j] = p.x;
        y[j] = p.y;
    }
}

__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const int hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__global__ __launch_bounds__(kBlock) void k_batched_voronoi(
    const ChunkDesc* __restrict__ desc, const PolyHdr* __restrict__ hdr,
    const float4* __restrict__ coef, const double2* __restrict__ gen,
    const int64_t* __restrict__ vtx_off, const int64_t* __restrict__ pt_off,
    const int64_t* __restrict__ lbl_word_off, const float2* __restrict__ Q,
    uint32_t* __restrict__ labels, const int64_t* __restrict__ misc, int G) {
    __shared__ float4 coefs[kWavesPerBlock][kMaxEdges];
    __shared__ int64_t qidx[kWavesPerBlock][kQueueCap];
    __shared__ int32_t qpoly[kWavesPerBlock][kQueueCap];
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
    float px[kPPL], py[kPPL];
    load_points(Q, d.start, d.start + d.count - 1, lane, px, py);

    int cur_k = -1;
    float ox = 0.f, oy = 0.f, KQ = 0.f, KA = 0.f, KB = 0.f, KC = 0.f;
    int n4 = 0;
    int64_t ptk = 0, wk = 0;
    int qcount = 0;
    for (;;) {
        // the chunk after g in this wave's sequence
        int64_t g2 = g + 1;
        if (g2 % G == 0 || g2 >= nchunks) {
            tile += W;
            g2 = tile * G;
        }
        const bool more = g2 < nchunks;
        const ChunkDesc d2 = desc[uniform64(more ? g2 : g)];

        const int k = __builtin_amdgcn_readfirstlane(d.k);
        if (k != cur_k) {  // stage the polygon's table (before the prefetch)
            const PolyHdr& H = hdr[k];
            ox = H.ox;
            oy = H.oy;
            KQ = H.KQ;
            KA = H.KA;
            KB = H.KB;
            KC = H.KC;
            n4 = __builtin_amdgcn_readfirstlane(H.n4);
            ptk = pt_off[k];
            wk = lbl_word_off[k];
            if (lane < n4) coefs[wv][lane] = coef[coef_base(vtx_off, k) + lane];
            __builtin_amdgcn_wave_barrier();
            cur_k = k;
        }
        float nx[kPPL], ny[kPPL];
        load_points(Q, d2.start, d2.start + d2.count - 1, lane, nx, ny);

        bool valid[kPPL];
        float X[kPPL], Y[kPPL];
#pragma unroll
        for (int j = 0; j < kPPL; ++j) {
            valid[j] = lane + kWave * j < d.count;
            X[j] = px[j] - ox;
            Y[j] = py[j] - oy;
        }
        uint64_t inm[kPPL], unc[kPPL];
        if (n4 > 0) {
            screen_chunk<K_VORONOI>(coefs[wv], n4, KQ, KA, KB, KC, X, Y, valid, inm, unc);
        } else {
#pragma unroll
            for (int j = 0; j < kPPL; ++j) inm[j] = unc[j] = 0;  // invalid polygon: labels 0
        }
        const int nunc = __popcll(unc[0]) + __popcll(unc[1]) + __popcll(unc[2]) + __popcll(unc[3]);
        if (nunc != 0 && qcount + nunc > kQueueCap) {
            flush_batched(vtx_off, pt_off, lbl_word_off, hdr, gen, Q, labels, qidx[wv], qpoly[wv],
                          qcount, lane);
            qcount = 0;
        }
        const int64_t local = d.start - ptk;  // multiple of 256
        store_chunk_words(labels, wk + local / 32, ((int64_t)d.count + 31) / 32, lane, inm);
        if (nunc != 0) {
            const uint64_t lt = lanemask_lt();
#pragma unroll
            for (int j = 0; j < kPPL; ++j) {
                if ((unc[j] >> lane) & 1ull) {
                    const int slot = qcount + __popcll(unc[j] & lt);
                    qidx[wv][slot] = d.start + lane + kWave * j;
                    qpoly[wv][slot] = k;
                }
                qcount += __popcll(unc[j]);
            }
        }
        if (!more) break;
        g = g2;
        d = d2;
#pragma unroll
        for (int j = 0; j < kPPL; ++j) {
            px[j] = nx[j];
            py[j] = ny[j];
        }
    }
    if (qcount > 0)
        flush_batched(vtx_off, pt_off, lbl_word_off, hdr, gen, Q, labels, qidx[wv], qpoly[wv], qcount,
                      lane);
}

}  // namespace

namespace pipdev {

size_t batched_workspace_layout(int64_t P, int64_t total_vertices, int64_t total_points,
                                BatchedLayout* L) {
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t off = 0;
    L->hdr = off;
    off = up(off + sizeof(PolyHdr) * (size_t)P);
    L->coef = off;
    off = up(off + 16 * (size_t)(total_vertices + 3 * P));
    L->gen = off;
    off = up(off + 16 * (size_t)(total_vertices + P));
    L->chunk_cnt = off;
    off = up(off + 8 * (size_t)P);
    L->chunk_off = off;
    off = up(off + 8 * (size_t)(P + 1));
    L->max_chunks = total_points / kChunk + P + 1;
    L->desc = off;
    off = up(off + sizeof(ChunkDesc) * (size_t)L->max_chunks);
    L->misc = off;
    off = up(off + 64);
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
    hipLaunchKernelGGL(k_batched_voronoi, dim3(blocks), dim3(kBlock), 0, stream,
                       reinterpret_cast<const ChunkDesc*>(D.desc), D.hdr, D.coef, D.gen, D.vtx_off,
                       D.pt_off, D.lbl_word_off, reinterpret_cast<const float2*>(D.Q), D.labels,
                       D.misc, G);
    return hipGetLastError();
}

hipError_t batched_max_blocks_per_cu(int* out) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, (const void*)k_batched_voronoi, kBlock, 0);
}

}  // namespace pipdev

namespace {
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
hipError_t launch_count_diff(const uint32_t* a, const uint32_t* b, int64_t nwords,
                             unsigned long long* out, hipStream_t stream) {
    hipLaunchKernelGGL(k_count_diff, dim3(1024), dim3(256), 0, stream, a, b, nwords, out);
    return hipGetLastError();
}
}  // namespace pipdev
