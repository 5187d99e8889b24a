// Non-convex polygons as unions of convex pieces.
//
// Section 7 of the paper names non-convex polygons as the extension of the
// method: the test of Section 4 needs a convex polygon, so a simple polygon
// is split into convex pieces whose vertices are vertices of the polygon,
// every piece gets its own inner and outer generators (Section 3, Algorithms
// 3-4) and a point is inside iff the closed Voronoi test (Algorithm 5) of at
// least one piece puts it inside.
//
//   k_prepare_pieces  one wave per piece: gathers the piece's vertices through
//                     its index list, derives its generators in binary64 and
//                     its float32 margin rows and band, all in one float32
//                     frame shared by the pieces (origin fl32(v_0)), so a
//                     point's local coordinates are formed once, not per piece.
//   k_pieces          persistent waves over chunks of 512 points (8 per lane,
//                     the layout of the single-polygon float32 kernel); the
//                     rows and bands of every piece sit in LDS.  Per point and
//                     piece: the largest margin against the piece's band; the
//                     point is inside when some piece clears it below, outside
//                     when every piece clears it above, else it is queued and
//                     re-decided in binary64 against every piece (Algorithm 5
//                     replayed operation by operation).
#include "device.hpp"
#include "kernels.hpp"
#include "stream32.hpp"

using namespace pipdev;

namespace {

// Workspace: headers [K], then margin rows (piece k at row off[k] + 3k,
// n4 <= n_k + 3 rows), then generators (piece k at off[k] + k, n_k + 1).
struct alignas(32) PieceHdr {
    float KQ, KA, KB, KC;  // band of the piece in the shared frame
    int n4;                // margin rows (multiple of 4); 0: the piece contains no point
    int row;               // first row
    int n;                 // edges (binary64 recheck)
    int gen;               // index of the piece's p_0 in the generator array
};
static_assert(sizeof(PieceHdr) == 32, "PieceHdr is 32 bytes");

__device__ __forceinline__ float frame_coord(double v) { return (float)v; }

__global__ __launch_bounds__(kBlock) void k_prepare_pieces(const double* __restrict__ V, int64_t n,
                                                           int K, const int32_t* __restrict__ off,
                                                           const int32_t* __restrict__ idx,
                                                           int64_t idx_count, PieceHdr* hdr,
                                                           float4* rows, double2* gens,
                                                           int32_t* status) {
    __shared__ PolyLds S[kWavesPerBlock];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int k = blockIdx.x * kWavesPerBlock + wv;
    if (k >= K) return;  // whole wave
    const int64_t o0 = off[k], o1 = off[k + 1];
    const int64_t nk = o1 - o0;
    bool bad_range = o0 < 0 || o1 < o0 || o1 > idx_count;
    int32_t vi = 0;
    if (!bad_range && lane < nk && lane < kMaxEdges) {
        vi = idx[o0 + lane];
        if (vi < 0 || vi >= n) vi = -1;
    }
    bad_range = bad_range || __ballot(vi < 0) != 0;
    int st = ST_OK;
    if (bad_range || nk < 3) st = ST_INVAL;
    else if (nk > kMaxEdges) st = 6;  // PIP_EUNSUPPORTED
    PieceHdr h;
    h.row = (int)(bad_range ? 0 : o0 + 3 * k);
    h.gen = (int)(bad_range ? 0 : o0 + k);
    if (st != ST_OK) {
        if (lane == 0) {
            h.KQ = h.KA = h.KB = h.KC = __builtin_huge_valf();
            h.n4 = 0;
            h.n = 0;
            hdr[k] = h;
            if (status) status[k] = st;
        }
        return;
    }
    const int nn = (int)nk;
    PolyLds& L = S[wv];
    if (lane < nn) L.vtx[lane] = make_double2(V[2 * (int64_t)vi], V[2 * (int64_t)vi + 1]);
    if (lane == 0) L.n = nn;
    __builtin_amdgcn_wave_barrier();
    const float fox = frame_coord(V[0]), foy = frame_coord(V[1]);
    prepare_polygon(L, K_VORONOI, lane, false, 4.05, true, fox, foy);
    __builtin_amdgcn_wave_barrier();
    const int n4 = L.n4;
    if (lane < n4) rows[h.row + lane] = L.coef[lane];
    for (int i = lane; i <= nn; i += kWave) gens[h.gen + i] = L.gen[i];
    if (lane == 0) {
        h.KQ = L.KQ;
        h.KA = L.KA;
        h.KB = L.KB;
        h.KC = L.KC;
        h.n4 = n4;
        h.n = nn;
        hdr[k] = h;
        if (status) status[k] = L.status;
    }
}

typedef double vdouble2 __attribute__((ext_vector_type(2)));
template <typename PT>
struct Pt2;
template <>
struct Pt2<float> {
    using T = vfloat2;
};
template <>
struct Pt2<double> {
    using T = vdouble2;
};

__device__ __forceinline__ float local_coord(float p, float o) { return p - o; }
__device__ __forceinline__ float local_coord(double p, float o) { return (float)(p - (double)o); }

// Queue entries: code = (c << 9) | r for point r of the wave's c-th chunk,
// and the coordinates as loaded.
template <typename PT>
__device__ void flush_pieces(const PieceHdr* hs, int K, const double2* __restrict__ gens,
                             const uint32_t* qc, const PT* qx, const PT* qy, int count,
                             uint32_t* labels, int lane, int64_t c0, int64_t stride) {
    wave_drain();
    for (int e = lane; e < count; e += kWave) {
        const uint32_t code = qc[e];
        const int64_t i = (c0 + (int64_t)(code >> 9) * stride) * kChunk32 + (code & 511u);
        const double x = (double)qx[e], y = (double)qy[e];
        bool in = false;
        for (int k = 0; k < K && !in; ++k) {
            const PieceHdr& h = hs[k];
            if (h.n4 > 0) in = voronoi64(x, y, gens + h.gen, h.n);
        }
        if (in) or_label_bit(labels, i >> 5, (uint32_t)(i & 31));
    }
    __builtin_amdgcn_wave_barrier();
}

template <typename PT>
__global__ __launch_bounds__(kBlock) void k_pieces(const double* __restrict__ V, int K, int nrows,
                                                   const PieceHdr* __restrict__ hdr_g,
                                                   const float4* __restrict__ rows_g,
                                                   const double2* __restrict__ gens,
                                                   const void* __restrict__ Qv, int64_t m,
                                                   uint32_t* __restrict__ labels) {
    using P2 = typename Pt2<PT>::T;
    extern __shared__ __align__(32) unsigned char lds[];
    PieceHdr* hs = reinterpret_cast<PieceHdr*>(lds);
    float4* rs = reinterpret_cast<float4*>(lds + sizeof(PieceHdr) * (size_t)K);
    __shared__ uint32_t queue_c[kWavesPerBlock][kQueue32];
    __shared__ PT queue_x[kWavesPerBlock][kQueue32];
    __shared__ PT queue_y[kWavesPerBlock][kQueue32];

    const P2* Q = static_cast<const P2*>(Qv);
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int64_t nfull = m / kChunk32;
    const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
    const int64_t c0 = (int64_t)blockIdx.x * kWavesPerBlock + wv;
    int64_t chunk = c0;
    uint32_t kc = 0;  // chunks of this wave so far

    auto load = [&](int64_t ch, P2(&p)[kP32]) {
#pragma unroll
        for (int j = 0; j < kP32; ++j)
            p[j] = __builtin_nontemporal_load(Q + ch * kChunk32 + lane + kWave * j);
    };
    P2 pa[kP32], pb[kP32];
    if (nfull > 0) load(chunk < nfull ? chunk : nfull - 1, pa);
    for (int i = tid; i < K; i += kBlock) hs[i] = hdr_g[i];
    for (int i = tid; i < nrows; i += kBlock) rs[i] = rows_g[i];
    __syncthreads();
    const float fox = frame_coord(V[0]), foy = frame_coord(V[1]);
    int qcount = 0;

    auto process = [&](const P2(&p)[kP32], int64_t ch, int64_t rem) {
        const bool full = rem >= kChunk32;
        float X[kP32], Y[kP32], R2[kP32], AX[kP32], AY[kP32];
        uint64_t inm[kP32], unc[kP32];
#pragma unroll
        for (int j = 0; j < kP32; ++j) {
            X[j] = local_coord(p[j].x, fox);
            Y[j] = local_coord(p[j].y, foy);
            R2[j] = fmaf(X[j], X[j], Y[j] * Y[j]);
            AX[j] = fabsf(X[j]);
            AY[j] = fabsf(Y[j]);
            inm[j] = 0;
            unc[j] = 0;
        }
        for (int k = 0; k < K; ++k) {
            const int n4 = __builtin_amdgcn_readfirstlane(hs[k].n4);
            if (n4 == 0) continue;
            const float4* cf = rs + __builtin_amdgcn_readfirstlane(hs[k].row);
            float Mx[kP32];
            {
                const float4 q0 = cf[0], q1 = cf[1], q2 = cf[2], q3 = cf[3];
#pragma unroll
                for (int j = 0; j < kP32; ++j) {
                    const float m0 = fmaf(q0.x, X[j], fmaf(q0.y, Y[j], q0.z));
                    const float m1 = fmaf(q1.x, X[j], fmaf(q1.y, Y[j], q1.z));
                    const float m2 = fmaf(q2.x, X[j], fmaf(q2.y, Y[j], q2.z));
                    const float m3 = fmaf(q3.x, X[j], fmaf(q3.y, Y[j], q3.z));
                    Mx[j] = fmaxf(fmaxf(fmaxf(m0, m1), m2), m3);
                }
            }
            for (int e = 4; e < n4; e += 4) {
                const float4 q0 = cf[e + 0], q1 = cf[e + 1], q2 = cf[e + 2], q3 = cf[e + 3];
#pragma unroll
                for (int j = 0; j < kP32; ++j) {
                    const float m0 = fmaf(q0.x, X[j], fmaf(q0.y, Y[j], q0.z));
                    const float m1 = fmaf(q1.x, X[j], fmaf(q1.y, Y[j], q1.z));
                    const float m2 = fmaf(q2.x, X[j], fmaf(q2.y, Y[j], q2.z));
                    const float m3 = fmaf(q3.x, X[j], fmaf(q3.y, Y[j], q3.z));
                    Mx[j] = fmaxf(fmaxf(Mx[j], m0), m1);
                    Mx[j] = fmaxf(fmaxf(Mx[j], m2), m3);
                }
            }
            const float KQ = hs[k].KQ, KA = hs[k].KA, KB = hs[k].KB, KC = hs[k].KC;
#pragma unroll
            for (int j = 0; j < kP32; ++j) {
                const float E = fmaf(KQ, R2[j], fmaf(KA, AX[j], fmaf(KB, AY[j], KC)));
                const uint64_t in = __ballot(Mx[j] < -E), out = __ballot(Mx[j] > E);
                inm[j] |= in;
                unc[j] |= ~(in | out);
            }
        }
#pragma unroll
        for (int j = 0; j < kP32; ++j) unc[j] &= ~inm[j];  // one piece already says inside
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
                flush_pieces<PT>(hs, K, gens, queue_c[wv], queue_x[wv], queue_y[wv], qcount, labels,
                                 lane, c0, stride);
                qcount = 0;
            }
            const uint64_t lt = lanemask_lt();
#pragma unroll
            for (int j = 0; j < kP32; ++j) {
                if (unc[j] == 0) continue;  // wave-uniform: no undecided point in this slot
                if ((unc[j] >> lane) & 1ull) {
                    const int slot = qcount + __popcll(unc[j] & lt);
                    queue_c[wv][slot] = (kc << 9) | (uint32_t)(lane + kWave * j);
                    queue_x[wv][slot] = p[j].x;
                    queue_y[wv][slot] = p[j].y;
                }
                qcount += __popcll(unc[j]);
            }
        }
        ++kc;
    };

    for (;;) {
        if (chunk >= nfull) break;
        load(chunk + stride < nfull ? chunk + stride : chunk, pb);
        process(pa, chunk, kChunk32);
        chunk += stride;
        if (chunk >= nfull) break;
        load(chunk + stride < nfull ? chunk + stride : chunk, pa);
        process(pb, chunk, kChunk32);
        chunk += stride;
    }
    if (chunk == nfull && nfull * kChunk32 < m) {  // the partial chunk
        const int64_t base = nfull * kChunk32;
        const int rem = (int)(m - base);
        P2 pt[kP32];
#pragma unroll
        for (int j = 0; j < kP32; ++j) {
            const int r = lane + kWave * j;
            pt[j] = Q[base + (r < rem ? r : rem - 1)];
        }
        process(pt, chunk, rem);
    }
    if (qcount > 0)
        flush_pieces<PT>(hs, K, gens, queue_c[wv], queue_x[wv], queue_y[wv], qcount, labels, lane,
                         c0, stride);
}

constexpr size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

namespace pipdev {

size_t pieces_workspace_layout(int64_t K, int64_t idx_count, PiecesLayout* L) {
    size_t o = 0;
    L->hdr = o;
    o = up256(o + sizeof(PieceHdr) * (size_t)K);
    L->rows = o;
    o = up256(o + sizeof(float4) * (size_t)(idx_count + 3 * K));
    L->gens = o;
    o = up256(o + sizeof(double2) * (size_t)(idx_count + K));
    return o;
}

size_t pieces_lds_bytes(int64_t K, int64_t idx_count) {
    return sizeof(PieceHdr) * (size_t)K + sizeof(float4) * (size_t)(idx_count + 3 * K);
}

hipError_t pieces_max_blocks_per_cu(int qdt, size_t lds, int* out) {
    const void* f = qdt == 1 ? (const void*)k_pieces<double> : (const void*)k_pieces<float>;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, f, kBlock, lds);
}

hipError_t launch_pieces(const PiecesLaunch& A, hipStream_t stream) {
    PiecesLayout L;
    pieces_workspace_layout(A.K, A.idx_count, &L);
    char* ws = static_cast<char*>(A.ws);
    PieceHdr* hdr = reinterpret_cast<PieceHdr*>(ws + L.hdr);
    float4* rows = reinterpret_cast<float4*>(ws + L.rows);
    double2* gens = reinterpret_cast<double2*>(ws + L.gens);
    const int pblocks = (A.K + kWavesPerBlock - 1) / kWavesPerBlock;
    hipLaunchKernelGGL(k_prepare_pieces, dim3(pblocks), dim3(kBlock), 0, stream, A.V, A.n, A.K,
                       A.off, A.idx, A.idx_count, hdr, rows, gens, A.status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || A.m == 0) return e;
    const int nrows = (int)(A.idx_count + 3 * (int64_t)A.K);
    const size_t lds = pieces_lds_bytes(A.K, A.idx_count);
    const int64_t nchunks = (A.m + kChunk32 - 1) / kChunk32;
    const int64_t want = (nchunks + kWavesPerBlock - 1) / kWavesPerBlock;
    int grid = (int)(want < A.max_blocks ? want : A.max_blocks);
    if (grid < 1) grid = 1;
    if (A.qdt == 1)
        hipLaunchKernelGGL(k_pieces<double>, dim3(grid), dim3(kBlock), lds, stream, A.V, A.K, nrows,
                           hdr, rows, gens, A.Q, A.m, A.labels);
    else
        hipLaunchKernelGGL(k_pieces<float>, dim3(grid), dim3(kBlock), lds, stream, A.V, A.K, nrows,
                           hdr, rows, gens, A.Q, A.m, A.labels);
    return hipGetLastError();
}

}  // namespace pipdev
