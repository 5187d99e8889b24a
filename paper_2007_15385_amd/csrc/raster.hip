// Coverage raster: one convex polygon against every pixel point of a regular
// grid, the graphics use of point inclusion (Section 1: each screen pixel's
// membership decided by a point inclusion test).  Pixel (i, j) is the
// binary64 point (x0 + i dx, y0 + j dy) (one product and one sum per
// coordinate); bit i % 32 of label word j * ceil(width / 32) + i / 32 is its
// Voronoi label (Section 4, Eq. 1 and 9-11, Algorithm 5).
//
// Nothing is read from memory but the polygon, so the kernel is bound by the
// vector units.  A wave screens 512-pixel segments of one row: lane l holds
// pixels 512 s + l + 64 k (k < 8), the layout of the streaming kernels, so a
// segment's 16 label words come from the ballots as there.  Along a row Y is
// constant, so the inner fma(B_i, Y, -C_i) of every edge is formed once per
// segment (the float32 operation the streaming screen performs per point) and
// a pixel costs one fma and half a max3 per edge.
//
// X is formed as fl32(i dx_32 + (x0 - o_x)_32) by one fma, not by rounding
// the binary64 pixel point.  Its distance from px - o_x, beyond the fma's own
// rounding (the band's local-coordinate term), is at most
//     DX = 1.02 u T + 2 v (|x0| + (W - 1)|dx|),  T = (W - 1)|dx| + |x0 - o_x|
// (the float32 roundings of dx and x0 - o_x, the binary64 roundings of the
// pixel point), so the band gains alpha DX (alpha = max |A_i|) and
// 50 v (T + DX) DX for the binary64 quadratic term.  Y = fl32(py - o_y) is the
// band's own conversion, formed in binary64 once per segment.  Undecided
// pixels are re-decided in binary64 on the spot from their recomputed
// coordinates.
//
// With the radial pre-screen (radial.hpp, thresholds derived with the
// raster's band constant), a pixel closer to p_0 than its octant's inner
// radius is inside and one beyond the outer radius outside, from r2 alone;
// only the segments holding a pixel between the radii run the per-edge
// screen (rows cross the polygon's boundary at two places, so most segments
// need no margin at all).  A whole segment is decided first when it can be:
// X = fl32(i dx + b) is monotone in the pixel index i and r2 =
// fl32(X^2 + Y^2) in |X| (correctly rounded operations keep order), so the
// segment's largest r2 is at an end pixel and its smallest at the other end,
// or at least fl32(Y^2) if X changes sign.  Along a row the octant of a pixel
// (sign bits of X and Y, |Y| > |X|) runs through four octants in a fixed
// order as X grows (Y >= 0: 4, 5, 1, 0; Y < 0: 6, 7, 3, 2), so a segment's
// pixels lie in the octants between those of its end pixels.  Below the
// smallest T_in of those octants every pixel is inside; beyond their largest
// T_out (and short of T_far) every pixel is outside, with no per-pixel work.
#include "device.hpp"
#include "kernels.hpp"
#include "radial.hpp"
#include "stream32.hpp"

using namespace pipdev;

namespace {

// early: the paper's early break (Section 5) in wave form -- every 8 edges
// the per-edge screen stops once every pixel of the segment is already
// decided outside (its partial largest margin beyond its band; the margin
// only grows with more edges), leaving the same labels.
template <bool RADIAL>
__global__ __launch_bounds__(kBlock) void k_raster(const double* __restrict__ V, int n,
                                                 RasterGrid G, uint32_t* __restrict__ labels,
                                                 int32_t* __restrict__ status, int early) {
    __shared__ PolyLds S;
    __shared__ RadialTab R;
    __shared__ float KC_s;                                // band constant with the X term
    __shared__ float ax_s[kMaxEdges];                     // A_i
    __shared__ float cy_s[kWavesPerBlock][kMaxEdges];     // fma(B_i, Y, -C_i) of the segment's row
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);

    if (tid < n) S.vtx[tid] = make_double2(V[2 * tid], V[2 * tid + 1]);
    if (tid == 0) S.n = n;
    __syncthreads();
    if (wv == 0) {
        prepare_polygon(S, K_VORONOI, lane);
        __builtin_amdgcn_wave_barrier();
        const float a = S.coef[lane].x;  // rows past n copy edge 0
        ax_s[lane] = a;
        const double alpha = wave_max(fabs((double)a));
        if (lane == 0) {
            const double span = (double)(G.width > 0 ? G.width - 1 : 0) * fabs(G.dx);
            const double T = span + fabs(G.x0 - (double)S.ox);
            const double DX = 1.02 * kU32 * T + 2.0 * kU64 * (fabs(G.x0) + span);
            const double infl = 1.0 + 9.5367431640625e-07;  // 1 + 2^-20
            KC_s = round_up_f32(((double)S.KC + alpha * DX + 50.0 * kU64 * (T + DX) * DX) * infl);
        }
        if constexpr (RADIAL) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            prepare_radial(S, lane, R, KC_s);
        }
    }
    __syncthreads();
    if (status && blockIdx.x == 0 && tid == 0) *status = S.status;

    const int64_t row_words = (G.width + 31) / 32;
    const int64_t segs = (G.width + kChunk32 - 1) / kChunk32;  // per row
    if (segs == 0 || G.height == 0) return;                    // status only
    const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
    const int n4 = S.n4;
    const float oy = S.oy, KQ = S.KQ, KA = S.KA, KB = S.KB, KC = KC_s;
    const float dxf = (float)G.dx;
    const float bxf = (float)(G.x0 - (double)S.ox);

    // segment seg = row * segs + s, walked with a stride of whole rows plus a
    // remainder (no division in the loop)
    const int64_t seg0 = (int64_t)blockIdx.x * kWavesPerBlock + wv;
    const int64_t drow = stride / segs, ds = stride - drow * segs;
    int64_t row = seg0 / segs, s = seg0 - row * segs;
    for (; row < G.height; row += drow, s += ds) {
        if (s >= segs) {
            s -= segs;
            row += 1;
            if (row >= G.height) break;
        }
        const double py = G.y0 + (double)row * G.dy;
        const float Y = (float)(py - (double)oy);
        const int64_t left = row_words - s * kWords32;
        const int nw = left < kWords32 ? (int)left : kWords32;
        if constexpr (RADIAL) {  // the whole segment at once, from its end pixels
            const int i0 = (int)s * kChunk32;
            const int64_t rem = G.width - (int64_t)i0;
            const int last = i0 + (rem < kChunk32 ? (int)rem : kChunk32) - 1;
            const float yy = Y * Y;
            const float Xa = fmaf((float)i0, dxf, bxf), Xb = fmaf((float)last, dxf, bxf);
            const float ra = fmaf(Xa, Xa, yy), rb = fmaf(Xb, Xb, yy);
            const float rmax = fmaxf(ra, rb);
            const float rmin = (Xa < 0.0f) != (Xb < 0.0f) ? yy : fminf(ra, rb);
            // position along the row's octant sequence: 0 (X < 0, |Y| <= |X|),
            // 1 (X < 0, |Y| > |X|), 2 (X >= 0, |Y| > |X|), 3 (X >= 0, |Y| <= |X|);
            // "X < 0" is the sign bit, as in the per-pixel octant
            const auto seq = [&](float X) {
                const bool neg = (__float_as_uint(X) >> 31) != 0;
                const bool steep = fabsf(Y) > fabsf(X);
                return neg ? (steep ? 1 : 0) : (steep ? 2 : 3);
            };
            const int qa = seq(Xa), qb = seq(Xb);
            const uint32_t sy = __float_as_uint(Y) >> 31;
            float tin = __builtin_huge_valf(), tout = 0.0f;
            for (int q = min(qa, qb); q <= max(qa, qb); ++q) {
                const int o = (q < 2 ? 4 : 0) + 2 * (int)sy + ((q == 1 || q == 2) ? 1 : 0);
                tin = fminf(tin, R.t[o].x);
                tout = fmaxf(tout, R.t[o].y);
            }
            const bool all_in = rmax < tin;  // NaN: false
            const bool all_out = rmin > tout && rmax < R.tfar;
            if (all_in || all_out) {
                uint32_t w = 0;
                if (all_in) {  // bits of the segment's existing pixels
                    const int64_t b = rem - 32 * (int64_t)lane;
                    w = b >= 32 ? ~0u : (b > 0 ? (1u << b) - 1u : 0u);
                }
                if (lane < nw) labels[row * row_words + s * kWords32 + lane] = w;
                continue;
            }
        }
        // this row's inner products, one edge per lane (same wave reads them)
        if (lane < n4) {
            const float4 c = S.coef[lane];
            cy_s[wv][lane] = fmaf(c.y, Y, c.z);
        }
        __builtin_amdgcn_wave_barrier();
        const float eY = fmaf(KQ, Y * Y, fmaf(KB, fabsf(Y), KC));
        const int i0 = (int)s * kChunk32;  // pixels i < width <= 2^24 are exact in float32
        float X[kP32], M[kP32];
#pragma unroll
        for (int j = 0; j < kP32; ++j) X[j] = fmaf((float)(i0 + lane + kWave * j), dxf, bxf);
        // the band of every pixel, needed by the early break before the loop ends
        const auto band = [&](int j) { return fmaf(KQ, X[j] * X[j], fmaf(KA, fabsf(X[j]), eY)); };
        uint64_t rin[kP32], ramb[kP32];  // radial decisions: inside, between the radii
        uint64_t any_amb = ~0ull;
        if constexpr (RADIAL) {
            const char* tab = reinterpret_cast<const char*>(R.t);
            const float tfar = R.tfar;
            const uint32_t sy = (__float_as_uint(Y) >> 31) << 4;
            const float yy = Y * Y;
            any_amb = 0;
#pragma unroll
            for (int j = 0; j < kP32; ++j) {
                const float r2 = fmaf(X[j], X[j], yy);  // the r2 of the thresholds
                const uint32_t off = ((__float_as_uint(X[j]) >> 31) << 5) | sy |
                                     (fabsf(Y) > fabsf(X[j]) ? 8u : 0u);
                const float2 t = *reinterpret_cast<const float2*>(tab + off);
                rin[j] = __ballot(r2 < t.x);
                ramb[j] = ~(rin[j] | __ballot((r2 > t.y) & (r2 < tfar)));
                any_amb |= ramb[j];
            }
        }
        if (any_amb) {  // per-edge screen of the whole segment
        const float4* A4 = reinterpret_cast<const float4*>(ax_s);
        const float4* C4 = reinterpret_cast<const float4*>(cy_s[wv]);
        {  // edges 0-3 start the max (n4 >= 4)
            const float4 a = A4[0], c = C4[0];
#pragma unroll
            for (int j = 0; j < kP32; ++j)
                M[j] = fmaxf(fmaxf(fmaxf(fmaf(a.x, X[j], c.x), fmaf(a.y, X[j], c.y)),
                                   fmaf(a.z, X[j], c.z)),
                             fmaf(a.w, X[j], c.w));
        }
        for (int e = 4; e < n4; e += 4) {
            if (early && (e & 7) == 0) {  // wave-uniform: all pixels already outside?
                uint64_t open = 0;
#pragma unroll
                for (int j = 0; j < kP32; ++j) open |= __ballot(!(M[j] > band(j)));
                if (open == 0) break;
            }
            const float4 a = A4[e / 4], c = C4[e / 4];
#pragma unroll
            for (int j = 0; j < kP32; ++j) {
                M[j] = fmaxf(fmaxf(M[j], fmaf(a.x, X[j], c.x)), fmaf(a.y, X[j], c.y));
                M[j] = fmaxf(fmaxf(M[j], fmaf(a.z, X[j], c.z)), fmaf(a.w, X[j], c.w));
            }
        }
        }
        // inside: M < -E; undecided: !(|M| > E) (E >= 0; NaN undecided)
        uint64_t inm[kP32], unc[kP32];
        uint64_t any_unc = 0;
#pragma unroll
        for (int j = 0; j < kP32; ++j) {
            if (any_amb) {
                const float E = band(j);
                inm[j] = __ballot(M[j] < -E);
                unc[j] = __ballot(!(fabsf(M[j]) > E));
            } else {
                inm[j] = 0;
                unc[j] = 0;
            }
            if constexpr (RADIAL) {  // the radial decision wherever it has one
                inm[j] = (inm[j] & ramb[j]) | rin[j];
                unc[j] &= ramb[j];
            }
            any_unc |= unc[j];
        }
        const int64_t rem = G.width - (int64_t)i0;  // pixels of this segment in the row
        if (rem < kChunk32) {
            any_unc = 0;
#pragma unroll
            for (int j = 0; j < kP32; ++j) {
                const uint64_t vm = __ballot(lane + kWave * j < rem);
                inm[j] &= vm;
                unc[j] &= vm;
                any_unc |= unc[j];
            }
        }
        if (any_unc) {  // rare: binary64 replay of Algorithm 5 at the pixel point
#pragma unroll
            for (int j = 0; j < kP32; ++j) {
                if (unc[j]) {
                    bool r = false;
                    if ((unc[j] >> lane) & 1ull) {
                        const double px = G.x0 + (double)(i0 + lane + kWave * j) * G.dx;
                        r = voronoi64(px, py, S.gen, n);
                    }
                    inm[j] = (inm[j] & ~unc[j]) | (__ballot(r) & unc[j]);
                }
            }
        }
        const uint32_t w = chunk_word32(inm);
        if (lane < nw) labels[row * row_words + s * kWords32 + lane] = w;
    }
}

}  // namespace

namespace pipdev {

hipError_t launch_raster(const double* V, int n, const RasterGrid& G, uint32_t* labels,
                         int32_t* status, int radial, int early, int max_blocks,
                         hipStream_t stream) {
    const int64_t segs = (G.width + kChunk32 - 1) / kChunk32 * G.height;
    const int64_t want = (segs + kWavesPerBlock - 1) / kWavesPerBlock;
    int grid = (int)(want < max_blocks ? want : max_blocks);
    if (grid < 1) grid = 1;
    if (radial)
        hipLaunchKernelGGL(k_raster<true>, dim3(grid), dim3(kBlock), 0, stream, V, n, G, labels, status,
                           early);
    else
        hipLaunchKernelGGL(k_raster<false>, dim3(grid), dim3(kBlock), 0, stream, V, n, G, labels, status,
                           early);
    return hipGetLastError();
}

hipError_t raster_max_blocks_per_cu(int radial, int* out) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        out, radial ? (const void*)k_raster<true> : (const void*)k_raster<false>, kBlock, 0);
}

}  // namespace pipdev
