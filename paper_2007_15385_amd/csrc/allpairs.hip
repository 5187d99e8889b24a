// All pairs: every polygon of a set (typically one footprint placed at many
// poses, the collision check of Section 1) against every point of one cloud.
//
//   k_poses_to_polygons  world vertices w = R(theta) v + t in binary64,
//                        ((c vx - s vy) + tx, (s vx + c vy) + ty).
//   k_prepare_uniform    one wave per polygon: generators (Section 3,
//                        Algorithms 3-4, binary64), float32 coefficients of the
//                        global-frame margin and its band constants.
//   k_allpairs           workgroup = 2048-point tile (8 points per lane) x
//                        group of up to 16 polygons whose coefficients are
//                        staged in LDS; per (polygon, point): n margins (2 FMA
//                        each), max3, compare with the band bounded once per
//                        (polygon, wave) from the wave's coordinate maxima;
//                        undecided pairs are re-decided in binary64 on the spot
//                        (Algorithm 5); inside bits go straight from the
//                        compares into ballots, 16 label words per (polygon,
//                        wave) are assembled in one VGPR and stored at once,
//                        and the inside bits are counted per polygon.
//
// Antipodal pairing (optional, Section 5's remark that work per edge is what
// counts): for a centrally symmetric polygon with an even number of edges,
// edge j = i + n/2 is parallel to edge i on the other side of p_0, so
// p_j - p_0 = -(p_i - p_0) and, with t = a X + b Y + s, a = (A_i - A_j)/2,
// b = (B_i - B_j)/2, s = (C_j - C_i)/2, h = (C_i + C_j)/2,
//     max(m_i, m_j) = |t| - h + (delta_a X + delta_b Y),
// delta_a = (A_i + A_j)/2, delta_b likewise (zero for exact symmetry).  One
// pair costs two fma and one subtraction instead of four fma and two max.
// The binary64 placement of a footprint leaves delta of a few ulps; its bound
// goes into the band (KA, KB), so labels stay those of Algorithm 5.
#include "device.hpp"
#include "kernels.hpp"
#include "stream32.hpp"

using namespace pipdev;

namespace {

constexpr int kTilePoints = kWavesPerBlock * kChunk32;  // 2048 points per workgroup tile
constexpr int kLdsCoefBytes = 16384;                    // coefficient staging per workgroup
constexpr int kMaxGroup = 16;                           // polygons per workgroup

__global__ void k_poses_to_polygons(const double* __restrict__ F, int n,
                                    const float* __restrict__ pose, const double* __restrict__ cs,
                                    int64_t K, double* __restrict__ Wout) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K * n) return;
    const int64_t k = i / n;
    const int v = (int)(i - k * n);
    const double c = cs[2 * k], s = cs[2 * k + 1];
    const double tx = (double)pose[3 * k], ty = (double)pose[3 * k + 1];
    const double vx = F[2 * v], vy = F[2 * v + 1];
    Wout[2 * i] = (c * vx - s * vy) + tx;
    Wout[2 * i + 1] = (s * vx + c * vy) + ty;
}

// Table rows of polygon k: hdr[k], coef[k * n4 ...], gen[k * (n + 1) ...]
// for P polygons of n vertices each (V [P][n][2]); with vtx_off (CSR, polygon
// k = V[vtx_off[k] .. vtx_off[k+1]), 3..64 vertices) the rows start at
// vtx_off[k] + 3 k and the generators at vtx_off[k] + k, and a polygon with a
// bad vertex range or count gets a status, no rows, labels 0 and count 0.
__global__ __launch_bounds__(kBlock) void k_prepare_uniform(int64_t P, int n_uniform,
                                                          const int64_t* __restrict__ vtx_off,
                                                          int64_t total_vertices,
                                                          const double* __restrict__ V,
                                                          PolyHdr* __restrict__ hdr,
                                                          float4* __restrict__ coef,
                                                          double2* __restrict__ gen,
                                                          int32_t* __restrict__ status,
                                                          int32_t* __restrict__ counts, int pair) {
    __shared__ PolyLds S[kWavesPerBlock];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int64_t k = (int64_t)blockIdx.x * kWavesPerBlock + wv;
    if (k >= P) return;
    int64_t v0 = k * n_uniform, nk = n_uniform;
    int64_t row0 = k * ((n_uniform + 3) & ~3), gen0 = k * (n_uniform + 1);
    if (vtx_off) {
        v0 = vtx_off[k];
        nk = vtx_off[k + 1] - v0;
        row0 = v0 + 3 * k;
        gen0 = v0 + k;
        int bad = 0;
        if (v0 < 0 || nk < 0 || v0 + nk > total_vertices || nk < 3) bad = 1;  // PIP_EINVAL
        else if (nk > kMaxEdges) bad = 6;                                   // PIP_EUNSUPPORTED
        if (bad) {
            if (lane == 0) {
                PolyHdr H;
                H.ox = H.oy = 0.f;
                H.KQ = H.KA = H.KB = H.KC = __builtin_huge_valf();
                H.n = 0;
                H.n4 = 0;
                H.status = bad;
                H.cx = H.cy = 0.f;
                H.rad = __builtin_huge_valf();
                H.npair = 0;
                H.radial = 0;
                H.row = 0;
                H.RQ = 0.f;
                hdr[k] = H;
                if (status) status[k] = bad;
                if (counts) counts[k] = 0;
            }
            return;
        }
    }
    const int n = (int)nk;
    PolyLds& L = S[wv];
    if (lane < n) L.vtx[lane] = make_double2(V[2 * (v0 + lane)], V[2 * (v0 + lane) + 1]);
    if (lane == 0) L.n = n;
    __builtin_amdgcn_wave_barrier();
    prepare_polygon(L, K_VORONOI, lane, /*global_frame=*/true);
    __builtin_amdgcn_wave_barrier();
    // disk containing the polygon: centre p_0 rounded to float32, radius =
    // largest vertex distance from p_0 plus the centre's rounding, inflated
    // and rounded up (every point of a convex polygon is within it)
    const double g0x = L.gen[0].x, g0y = L.gen[0].y;
    double dv = 0.0;
    if (lane < n) {
        const double dx = L.vtx[lane].x - g0x, dy = L.vtx[lane].y - g0y;
        dv = sqrt(dx * dx + dy * dy);
    }
    const double rmax = wave_max(dv);
    const int n4 = L.n4;

    // Antipodal pairs (edge i, edge i + n/2), lane i < n/2; binary64 values
    // formed as prepare_polygon forms them in the global frame (o = 0).
    //   float32 part: t = fma(a, X, fma(b, Y, s)) and |t| - h carry
    //     5.1 u (|a||X| + |b||Y| + |s| + |h|) (coefficient roundings 1.01 u
    //     each, two fma, one subtraction), plus the binary64 roundings of
    //     a, b (2 v max|h_x|, |h_y| each) and of s, h (v max|C| each, and
    //     4.1 v (G2 + d2) each from C_i, C_j);
    //   asymmetry: |delta_a||X| + |delta_b||Y|, delta formed in binary64
    //     (error v (2 max|h_x| + |delta_a|));
    //   binary64 part of Algorithm 5: as for the unpaired table.
    // Pairing is used only when the asymmetry is below u of the pair
    // coefficients (at most doubles the X, Y terms of the band).
    int npair = 0;
    float pKQ = 0.f, pKA = 0.f, pKB = 0.f, pKC = 0.f;
    float4 prow = make_float4(0.f, 0.f, 0.f, 0.f);
    if (pair && (n & 1) == 0) {
        const int hn = n >> 1;
        const int i = lane < hn ? lane : 0;
        const double d2 = g0x * g0x + g0y * g0y;
        const double gix = L.gen[1 + i].x, giy = L.gen[1 + i].y;
        const double gjx = L.gen[1 + i + hn].x, gjy = L.gen[1 + i + hn].y;
        const double hxi = gix - g0x, hyi = giy - g0y, hxj = gjx - g0x, hyj = gjy - g0y;
        const double g2i = gix * gix + giy * giy, g2j = gjx * gjx + gjy * gjy;
        const double Ci = g2i - d2, Cj = g2j - d2;
        const float a = (float)(hxi - hxj), b = (float)(hyi - hyj);
        const float s = (float)(0.5 * (Cj - Ci)), h = (float)(0.5 * (Ci + Cj));
        prow = make_float4(a, b, s, h);
        const bool fin = isfinite(a) && isfinite(b) && isfinite(s) && isfinite(h) &&
                         fabs((double)a) < kCoefLimit && fabs((double)b) < kCoefLimit &&
                         fabs((double)s) < kCoefLimit && fabs((double)h) < kCoefLimit;
        const double ap = wave_max(fabs((double)a)), bp = wave_max(fabs((double)b));
        const double gp = wave_max(fabs((double)s) + fabs((double)h));
        const double DA = wave_max(fabs(hxi + hxj)), DB = wave_max(fabs(hyi + hyj));
        const double hmx = wave_max(fmax(fabs(hxi), fabs(hxj)));
        const double hmy = wave_max(fmax(fabs(hyi), fabs(hyj)));
        const double cm = wave_max(fmax(fabs(Ci), fabs(Cj)));
        const double G2 = wave_max(fmax(g2i, g2j));
        const double H2 = wave_max(fmax(hxi * hxi + hyi * hyi, hxj * hxj + hyj * hyj));
        const bool sym = __ballot(!fin) == 0 && L.status == 0 && DA <= kU32 * ap &&
                         DB <= kU32 * bp && ap > 0.0 && bp > 0.0;
        if (sym) {
            const double infl = 1.0 + 9.5367431640625e-07;  // 1 + 2^-20
            npair = hn;
            pKA = round_up_f32((5.1 * kU32 * ap + DA + 2.02 * kU64 * (2.0 * hmx + DA)) * infl);
            pKB = round_up_f32((5.1 * kU32 * bp + DB + 2.02 * kU64 * (2.0 * hmy + DB)) * infl);
            pKC = round_up_f32((5.1 * kU32 * gp + 2.02 * kU64 * cm + 8.2 * kU64 * (G2 + d2) +
                                4.0001 * kU64 * (6.0 * d2 + 2.0 * H2) +
                                kEpsAbs * (1.0 + ap + bp)) * infl);
            pKQ = round_up_f32(24.01 * kU64 * infl);
        }
    }
    const int np4 = (npair + 3) & ~3;
    if (npair > 0) {
        if (lane < np4) coef[row0 + lane] = prow;  // rows past n/2 repeat pair 0
    } else if (lane < n4) {
        coef[row0 + lane] = L.coef[lane];
    }
    for (int i = lane; i <= n; i += kWave) gen[gen0 + i] = L.gen[i];
    if (lane == 0) {
        PolyHdr H;
        H.ox = L.ox;
        H.oy = L.oy;
        H.KQ = npair ? pKQ : L.KQ;
        H.KA = npair ? pKA : L.KA;
        H.KB = npair ? pKB : L.KB;
        H.KC = npair ? pKC : L.KC;
        H.n = n;
        H.n4 = n4;
        H.status = L.status;
        H.cx = (float)g0x;
        H.cy = (float)g0y;
        const double ce = fabs((double)H.cx - g0x) + fabs((double)H.cy - g0y);
        H.rad = round_up_f32((rmax + ce) * (1.0 + 1.0 / 65536.0) + 1e-30);  // NaN -> +inf
        H.npair = npair;
        H.radial = 0;
        H.row = (int)row0;
        H.RQ = 0.f;
        hdr[k] = H;
        if (status) status[k] = L.status;
        if (counts) counts[k] = 0;  // k_allpairs accumulates into it
    }
}

__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
    return v;
}

// grid: x = point tiles of 2048, y = polygon groups of PG (<= 16).  CULL:
// skip (polygon, wave) pairs whose bounding disk misses the wave's points.
// PAIR: polygons whose table holds antipodal pairs take the paired loop.
// CSR: polygons of uneven vertex counts (n4, row and generator offset from
// each polygon's header; LDS rows at a fixed stride of kCsrStride per polygon).
constexpr int kCsrStride = kMaxEdges + 4;

template <bool CULL, bool PAIR, bool CSR>
__global__ __launch_bounds__(kBlock) void k_allpairs(const PolyHdr* __restrict__ hdr,
                                                   const float4* __restrict__ coef,
                                                   const double2* __restrict__ gen, int64_t P,
                                                   int n, int PG, const float2* __restrict__ Q,
                                                   int64_t m, uint32_t* __restrict__ labels,
                                                   int32_t* __restrict__ counts) {
    extern __shared__ float4 coef_s[];  // [PG][n4], CSR: [PG][kCsrStride]
    __shared__ int32_t cnt_s[kMaxGroup];
    __shared__ float band_s[kWavesPerBlock][kMaxGroup];  // per (wave, polygon)
    __shared__ int skip_s[kWavesPerBlock][kMaxGroup];    // polygon's disk misses the wave's points
    __shared__ int npair_s[kMaxGroup];                   // antipodal pair rows (0: edge rows)
    __shared__ int n_s[kMaxGroup], n4_s[kMaxGroup];      // CSR: edges and rows per polygon
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int n4u = (n + 3) & ~3;
    const int64_t k0 = (int64_t)blockIdx.y * PG;
    const int pg = (int)((P - k0) < PG ? (P - k0) : PG);
    const int64_t words = (m + 31) / 32;

    if constexpr (CSR) {
        for (int p = wv; p < pg; p += kWavesPerBlock) {  // one wave per polygon
            const PolyHdr& H = hdr[k0 + p];
            const int r4 = __builtin_amdgcn_readfirstlane(H.n4);
            const int row = __builtin_amdgcn_readfirstlane(H.row);
            if (lane < r4) coef_s[p * kCsrStride + lane] = coef[row + lane];
            if (lane == 0) {
                n_s[p] = H.n;
                n4_s[p] = r4;
            }
        }
    } else {
        for (int i = tid; i < pg * n4u; i += kBlock) coef_s[i] = coef[k0 * n4u + i];
    }
    for (int i = tid; i < pg; i += kBlock) cnt_s[i] = 0;

    // this wave's 512 points (lane l holds points l + 64 j); past the end and
    // non-finite points are outside for every polygon
    const int64_t base = (int64_t)blockIdx.x * kTilePoints + (int64_t)wv * kChunk32;
    const int64_t rem64 = m - base;
    const int rem = (int)(rem64 < kChunk32 ? (rem64 > 0 ? rem64 : 0) : kChunk32);
    float x[kP32], y[kP32];
    uint64_t live[kP32] = {};
    float xm = 0.f, ym = 0.f;
    // box and distance range (from the origin) of the wave's live points
    float xlo = __builtin_huge_valf(), xhi = -__builtin_huge_valf();
    float ylo = __builtin_huge_valf(), yhi = -__builtin_huge_valf();
    float r2lo = __builtin_huge_valf(), r2hi = 0.f;
    if (rem > 0) {
#pragma unroll
        for (int j = 0; j < kP32; ++j) {
            const int r = lane + kWave * j;
            const float2 p = Q[base + (r < rem ? r : rem - 1)];
            x[j] = p.x;
            y[j] = p.y;
            const bool ok = r < rem && isfinite(p.x) && isfinite(p.y);
            live[j] = __ballot(ok);
            if (ok) {
                xm = fmaxf(xm, fabsf(p.x));
                ym = fmaxf(ym, fabsf(p.y));
                if constexpr (CULL) {
                    xlo = fminf(xlo, p.x);
                    xhi = fmaxf(xhi, p.x);
                    ylo = fminf(ylo, p.y);
                    yhi = fmaxf(yhi, p.y);
                    const float r2 = fmaf(p.x, p.x, p.y * p.y);
                    r2lo = fminf(r2lo, r2);
                    r2hi = fmaxf(r2hi, r2);
                }
            }
        }
        xm = wave_max_f(xm);
        ym = wave_max_f(ym);
        if constexpr (CULL) {
            xlo = -wave_max_f(-xlo);
            xhi = wave_max_f(xhi);
            ylo = -wave_max_f(-ylo);
            yhi = wave_max_f(yhi);
            r2lo = -wave_max_f(-r2lo);
            r2hi = wave_max_f(r2hi);
        }
    }
    uint64_t live_all = ~0ull;
#pragma unroll
    for (int j = 0; j < kP32; ++j) live_all &= live[j];
    const bool all_live = rem == kChunk32 && live_all == ~0ull;
    const float r2m = fmaf(xm, xm, ym * ym);
    // band for every point of this wave and polygon p of the group (monotone
    // in |x|, |y|), one lane per polygon
    if (lane < pg) {
        const PolyHdr& H = hdr[k0 + lane];
        band_s[wv][lane] = fmaf(H.KQ, r2m, fmaf(H.KA, xm, fmaf(H.KB, ym, H.KC)));
        // Culling (optional): the polygon lies in the disk (c, R); when that
        // disk misses the wave's box or its distance range from the origin,
        // no point of the wave is inside.  The disk is widened by
        // 2^-16 (|c_x| + |c_y| + R) and the squared distances carry a relative
        // slack of 2^-16, far above the float32 rounding of every quantity
        // compared; such a point is then also far outside in binary64.
        bool skip = false;
        if constexpr (CULL) {
            const float R = H.rad, cx = H.cx, cy = H.cy;
            const float sl = 1.0f / 65536.0f;
            const float Rs = R + (fabsf(cx) + fabsf(cy) + R) * sl;
            skip = cx + Rs < xlo || cx - Rs > xhi || cy + Rs < ylo || cy - Rs > yhi;
            const float dc = sqrtf(fmaf(cx, cx, cy * cy));
            const float hi = dc + Rs, lo = dc - Rs;
            skip = skip || hi * hi * (1.0f + sl) < r2lo * (1.0f - sl);
            skip = skip || (lo > 0.f && lo * lo * (1.0f - sl) > r2hi * (1.0f + sl));
            // no culling for a polygon without a finite disk (bad input)
            skip = skip && R < __builtin_huge_valf() && cx == cx && cy == cy;
        }
        if constexpr (CULL) skip_s[wv][lane] = skip ? 1 : 0;
        if (PAIR && wv == 0) npair_s[lane] = H.npair;
    }
    __syncthreads();

    if (rem > 0) {
        const int nw = (rem + 31) / 32;
        for (int p = 0; p < pg; ++p) {
            const int64_t k = k0 + p;
            const int n4 = CSR ? __builtin_amdgcn_readfirstlane(n4_s[p]) : n4u;
            if ((CULL && __builtin_amdgcn_readfirstlane(skip_s[wv][p])) || n4 == 0) {
                // all outside (or a polygon that contains no point)
                if (lane < nw) labels[k * words + base / 32 + lane] = 0u;
                continue;
            }
            const float E = band_s[wv][p];
            const float4* cf = coef_s + p * (CSR ? kCsrStride : n4u);
            float M[kP32];
            const int np = PAIR ? __builtin_amdgcn_readfirstlane(npair_s[p]) : 0;
            if (PAIR && np > 0) {
                // max over pairs of |t| - h, four pairs at a time (rows past
                // the last pair repeat pair 0)
                const int np4 = (np + 3) & ~3;
                auto pm = [](float4 c, float xx, float yy) {
                    return fabsf(fmaf(c.x, xx, fmaf(c.y, yy, c.z))) - c.w;
                };
                {
                    const float4 c0 = cf[0], c1 = cf[1], c2 = cf[2], c3 = cf[3];
#pragma unroll
                    for (int j = 0; j < kP32; ++j)
                        M[j] = fmaxf(fmaxf(fmaxf(pm(c0, x[j], y[j]), pm(c1, x[j], y[j])),
                                           pm(c2, x[j], y[j])),
                                     pm(c3, x[j], y[j]));
                }
                for (int e = 4; e < np4; e += 4) {
                    const float4 c0 = cf[e + 0], c1 = cf[e + 1], c2 = cf[e + 2], c3 = cf[e + 3];
#pragma unroll
                    for (int j = 0; j < kP32; ++j) {
                        M[j] = fmaxf(fmaxf(M[j], pm(c0, x[j], y[j])), pm(c1, x[j], y[j]));
                        M[j] = fmaxf(fmaxf(M[j], pm(c2, x[j], y[j])), pm(c3, x[j], y[j]));
                    }
                }
            } else {
                {  // edges 0-3 start the max (n4 >= 4)
                    const float4 c0 = cf[0], c1 = cf[1], c2 = cf[2], c3 = cf[3];
#pragma unroll
                    for (int j = 0; j < kP32; ++j) {
                        const float m0 = fmaf(c0.x, x[j], fmaf(c0.y, y[j], c0.z));
                        const float m1 = fmaf(c1.x, x[j], fmaf(c1.y, y[j], c1.z));
                        const float m2 = fmaf(c2.x, x[j], fmaf(c2.y, y[j], c2.z));
                        const float m3 = fmaf(c3.x, x[j], fmaf(c3.y, y[j], c3.z));
                        M[j] = fmaxf(fmaxf(fmaxf(m0, m1), m2), m3);
                    }
                }
                for (int e = 4; e < n4; e += 4) {
                    const float4 c0 = cf[e + 0], c1 = cf[e + 1], c2 = cf[e + 2], c3 = cf[e + 3];
#pragma unroll
                    for (int j = 0; j < kP32; ++j) {
                        const float m0 = fmaf(c0.x, x[j], fmaf(c0.y, y[j], c0.z));
                        const float m1 = fmaf(c1.x, x[j], fmaf(c1.y, y[j], c1.z));
                        const float m2 = fmaf(c2.x, x[j], fmaf(c2.y, y[j], c2.z));
                        const float m3 = fmaf(c3.x, x[j], fmaf(c3.y, y[j], c3.z));
                        M[j] = fmaxf(fmaxf(M[j], m0), m1);
                        M[j] = fmaxf(fmaxf(M[j], m2), m3);
                    }
                }
            }
            // inside: M < -E; undecided: !(|M| > E) (E >= 0; a NaN margin
            // or band is undecided); lanes past the end or holding a
            // non-finite point are masked only in waves that have any
            uint64_t inm[kP32];
            uint64_t any_unc = 0;
#pragma unroll
            for (int j = 0; j < kP32; ++j) {
                inm[j] = __ballot(M[j] < -E);
                any_unc |= __ballot(!(fabsf(M[j]) > E));
            }
            if (!all_live) {
                any_unc = 0;
#pragma unroll
                for (int j = 0; j < kP32; ++j) {
                    inm[j] &= live[j];
                    any_unc |= __ballot(!(fabsf(M[j]) > E)) & live[j];
                }
            }
            if (any_unc) {  // rare: re-decide in binary64 (Algorithm 5)
                const int nk = CSR ? n_s[p] : n;
                const double2* G = gen + (CSR ? (int64_t)hdr[k].row - 2 * (int64_t)k : k * (n + 1));
#pragma unroll
                for (int j = 0; j < kP32; ++j) {
                    const uint64_t unc = ~(inm[j] | __ballot(M[j] > E)) & live[j];
                    if (unc) {
                        bool r = false;
                        if ((unc >> lane) & 1ull) {
                            // the empty asm keeps the conversions here: hoisted
                            // out of the polygon loop they would hold 16
                            // binary64 values in registers for this rare path
                            float px = x[j], py = y[j];
#if defined(__HIP_DEVICE_COMPILE__)
                            asm volatile("" : "+v"(px), "+v"(py));
#endif
                            r = voronoi64((double)px, (double)py, G, nk);
                        }
                        inm[j] = (inm[j] & ~unc) | (__ballot(r) & unc);
                    }
                }
            }
            int c = 0;
#pragma unroll
            for (int j = 0; j < kP32; ++j) c += __popcll(inm[j]);
            const uint32_t w = chunk_word32(inm);
            if (lane < nw) labels[k * words + base / 32 + lane] = w;
            if (lane == 0 && c) atomicAdd(&cnt_s[p], c);
        }
    }
    __syncthreads();
    if (counts)
        for (int i = tid; i < pg; i += kBlock)
            if (cnt_s[i]) atomicAdd(&counts[k0 + i], cnt_s[i]);
}

}  // namespace

namespace pipdev {

size_t allpairs_workspace_layout(int64_t P, int n, AllpairsLayout* L) {
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    const int n4 = (n + 3) & ~3;
    size_t off = 0;
    L->hdr = off;
    off = up(off + sizeof(PolyHdr) * (size_t)P);
    L->coef = off;
    off = up(off + 16 * (size_t)P * n4);
    L->gen = off;
    off = up(off + 16 * (size_t)P * (n + 1));
    return off;
}

int allpairs_group(int n) {
    const int n4 = (n + 3) & ~3;
    int pg = kLdsCoefBytes / (16 * n4);
    return pg > kMaxGroup ? kMaxGroup : pg;
}

hipError_t launch_poses_to_polygons(const double* F, int n, const float* pose, const double* cs,
                                    int64_t K, double* Wout, hipStream_t stream) {
    const int64_t total = K * n;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_poses_to_polygons, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                       stream, F, n, pose, cs, K, Wout);
    return hipGetLastError();
}

hipError_t launch_allpairs(int64_t P, int n, const double* V, const float* Q, int64_t m,
                           uint32_t* labels, int32_t* counts, int32_t* status, void* ws, int cull,
                           int pair, hipStream_t stream) {
    AllpairsLayout L;
    allpairs_workspace_layout(P, n, &L);
    char* b = static_cast<char*>(ws);
    PolyHdr* hdr = reinterpret_cast<PolyHdr*>(b + L.hdr);
    float4* coef = reinterpret_cast<float4*>(b + L.coef);
    double2* gen = reinterpret_cast<double2*>(b + L.gen);
    const unsigned pblocks = (unsigned)((P + kWavesPerBlock - 1) / kWavesPerBlock);
    hipLaunchKernelGGL(k_prepare_uniform, dim3(pblocks), dim3(kBlock), 0, stream, P, n,
                       (const int64_t*)nullptr, (int64_t)0, V, hdr, coef, gen, status, counts,
                       pair);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (m == 0) return hipSuccess;
    const int pg = allpairs_group(n);
    const int n4 = (n + 3) & ~3;
    dim3 grid((unsigned)((m + kTilePoints - 1) / kTilePoints), (unsigned)((P + pg - 1) / pg));
    const size_t lds = (size_t)pg * n4 * 16;
    const float2* Q2 = reinterpret_cast<const float2*>(Q);
    auto kern = cull ? (pair ? k_allpairs<true, true, false> : k_allpairs<true, false, false>)
                     : (pair ? k_allpairs<false, true, false> : k_allpairs<false, false, false>);
    hipLaunchKernelGGL(kern, grid, dim3(kBlock), lds, stream, hdr, coef, gen, P, n, pg, Q2, m,
                       labels, counts);
    return hipGetLastError();
}

size_t allpairs_csr_workspace_layout(int64_t P, int64_t total_vertices, AllpairsLayout* L) {
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t off = 0;
    L->hdr = off;
    off = up(off + sizeof(PolyHdr) * (size_t)P);
    L->coef = off;
    off = up(off + 16 * (size_t)(total_vertices + 3 * P));
    L->gen = off;
    off = up(off + 16 * (size_t)(total_vertices + P));
    return off;
}

hipError_t launch_allpairs_csr(int64_t P, const int64_t* vtx_off, const double* V,
                               int64_t total_vertices, const float* Q, int64_t m,
                               uint32_t* labels, int32_t* counts, int32_t* status, void* ws,
                               int cull, int pair, hipStream_t stream) {
    AllpairsLayout L;
    allpairs_csr_workspace_layout(P, total_vertices, &L);
    char* b = static_cast<char*>(ws);
    PolyHdr* hdr = reinterpret_cast<PolyHdr*>(b + L.hdr);
    float4* coef = reinterpret_cast<float4*>(b + L.coef);
    double2* gen = reinterpret_cast<double2*>(b + L.gen);
    const unsigned pblocks = (unsigned)((P + kWavesPerBlock - 1) / kWavesPerBlock);
    hipLaunchKernelGGL(k_prepare_uniform, dim3(pblocks), dim3(kBlock), 0, stream, P, 0, vtx_off,
                       total_vertices, V, hdr, coef, gen, status, counts, pair);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (m == 0) return hipSuccess;
    const int pg = kLdsCoefBytes / (16 * kCsrStride);  // 15 polygons of up to 64 edges
    dim3 grid((unsigned)((m + kTilePoints - 1) / kTilePoints), (unsigned)((P + pg - 1) / pg));
    const size_t lds = (size_t)pg * kCsrStride * 16;
    const float2* Q2 = reinterpret_cast<const float2*>(Q);
    auto kern = cull ? (pair ? k_allpairs<true, true, true> : k_allpairs<true, false, true>)
                     : (pair ? k_allpairs<false, true, true> : k_allpairs<false, false, true>);
    hipLaunchKernelGGL(kern, grid, dim3(kBlock), lds, stream, hdr, coef, gen, P, 0, pg, Q2, m,
                       labels, counts);
    return hipGetLastError();
}

}  // namespace pipdev
