// Point location in a stored set of convex polygons (the GIS use of
// Section 1: field measurements matched against a polygon database).  The
// generators of the constant polygons are derived once and kept beside the
// vertices (Section 7: about twice the storage), with the float32 screen
// table and the band constants of each polygon; a uniform grid over the
// polygons' bounding boxes lists, per cell, every polygon whose box meets
// the cell.  A query point looks up its cell and tests the listed polygons
// (float32 screen, binary64 replay of Algorithm 5 inside the band); its id
// is the smallest index of a polygon that contains it, or -1.
//
// Exactness of the index.  Binary64 rounding can put a point just outside a
// polygon inside it, so a polygon's box is its vertex bounds widened by a
// bound on that distance.  Two errors add up.  (1) The evaluation of
// Algorithm 5 with the stored generators differs from their exact margin
// by at most E64 = 24.01 v |p - o|^2 + 4.0001 v (6 d2 + 2 H2) (the band's
// binary64 part).  (2) The stored generator p_i differs from the exact
// mirror image R_i of the stored p_0 across edge line i by some delta_i
// (the rounding of Algorithm 4): a, b, c and the products of Eq. 8 are
// rounded relative to the coordinate scale S = max |coordinate| over the
// vertices and p_0, and a first-order count of those roundings gives
// |delta_i| <= 40 v S; the index uses 64 v S (exact rational reflections of
// random polygons measure at most 7 v S).  Against the exact edge line the
// margin changes by at most 2 |p - R_i| delta + delta^2.  With
// m_i = 2 |R_i - p_0| s_i (s_i the signed distance past edge line i), every
// point binary64 calls inside lies in the polygon with each edge moved out
// by t(rho) = (E64 + 2 (rho + sqrt(d2) + sqrt(H2) + delta) delta + delta^2)
// / (2 (min |h_i| - delta)), rho = |p - o|; such an offset moves a vertex of
// interior angle theta by t / sin(theta / 2).  The box is widened by twice
// t(2 r) / min sin(theta_i / 2) (r the largest vertex distance from o) and
// rounded outwards to float32.  For rho > 2 r the same offset polygon lies
// within r + t(rho) / smin of o, so binary64 calls no point inside for
// r + t(rho) / smin < rho: a quadratic in rho, negative between two roots;
// the polygon is cell-listed only if 2 r lies between them, and the larger
// root (rounded down) is its far radius.  The grid's near region is the
// box of the cell-listed boxes and local origins, widened by its diagonal
// on each side; a polygon whose far radius does not exceed four times
// that diagonal goes to the global list, so within the near region a point
// outside a cell-listed polygon's box is outside it in binary64 too.  A
// point beyond the near region tests every polygon in index order (such
// points are far from all of them; at distances beyond the far radii
// Algorithm 5's rounding can call them inside: at 1e30 from a unit polygon
// every squared distance rounds to the same value).  A polygon without a
// finite, small widening (degenerate or non-convex input, non-finite
// vertices, or a centroid that binary64 rounding put outside the polygon)
// goes to the global list, which every query tests as well
// (binary64 decides; normally empty).  A box corner and a query point are
// mapped to cells by the same float32 function, monotone in the coordinate,
// so a point inside a box is in a cell of the box's range.  The answer is
// the minimum containing index, so the order of a cell's list does not
// matter.
//
//   k_index_prepare   one wave per polygon: generators (Algorithms 3-4),
//                     float32 table in the polygon's local frame, band
//                     constants, outward-rounded box; n > 64 is flagged.
//   k_index_bounds    one block: near region, demotions, union box of the
//                     cell-listed polygons, grid
//                     shape (about the requested cell count, square cells).
//   k_index_count /   one thread per polygon: its cell range, counted, then
//   k_index_fill      written into the cell lists (after an exclusive scan).
//   k_locate          one query point per lane; its cell's entries carry the
//                     candidates' boxes, so only box hits read a record.
#include "device.hpp"
#include "kernels.hpp"

using namespace pipdev;

namespace {

__device__ __forceinline__ float round_out_hi(double d) {
    float f = (float)d;
    if ((double)f < d) f = nextafterf(f, __builtin_huge_valf());
    return f;
}
__device__ __forceinline__ float round_out_lo(double d) {
    float f = (float)d;
    if ((double)f > d) f = nextafterf(f, -__builtin_huge_valf());
    return f;
}

// grid cell of a coordinate (monotone non-decreasing in x)
__device__ __forceinline__ int cell_of(float x, float x0, float inv, int g) {
    const float t = fminf(fmaxf((x - x0) * inv, 0.0f), (float)(g - 1));
    return (int)t;
}

__global__ __launch_bounds__(kBlock) void k_index_prepare(int64_t P,
                                                        const int64_t* __restrict__ vtx_off,
                                                        const double* __restrict__ V,
                                                        LocRec* __restrict__ rec,
                                                        float4* __restrict__ qrec,
                                                        double2* __restrict__ gen,
                                                        int32_t* __restrict__ status,
                                                        int32_t* __restrict__ flags) {
    __shared__ PolyLds S[kWavesPerBlock];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int64_t k = (int64_t)blockIdx.x * kWavesPerBlock + wv;
    if (k >= P) return;
    PolyLds& L = S[wv];
    const int64_t v0 = vtx_off[k];
    const int64_t nn = vtx_off[k + 1] - v0;
    LocRec R;
    R.n = 0;
    R.usable = 0;
    if (nn < 3 || nn > kMaxEdges) {  // contains no point / not supported
        if (lane == 0) {
            R.status = nn > kMaxEdges ? 6 : 1;  // PIP_EUNSUPPORTED, PIP_EINVAL
            rec[k] = R;
            if (status) status[k] = R.status;
            if (nn > kMaxEdges) atomicOr(flags, 1);
        }
        return;
    }
    const int n = (int)nn;
    if (lane < n) L.vtx[lane] = make_double2(V[2 * (v0 + lane)], V[2 * (v0 + lane) + 1]);
    if (lane == 0) L.n = n;
    __builtin_amdgcn_wave_barrier();
    prepare_polygon(L, K_VORONOI, lane);
    __builtin_amdgcn_wave_barrier();
    // vertex bounds (NaN poisons them: such a polygon is not indexed)
    const int i = lane < n ? lane : 0;
    const double2 v = L.vtx[i];
    const double xlo = -wave_max(-v.x), xhi = wave_max(v.x);
    const double ylo = -wave_max(-v.y), yhi = wave_max(v.y);
    const bool all_fin = __ballot(!(isfinite(v.x) && isfinite(v.y))) == 0;
    // widening: binary64 misclassification distance (see the file comment)
    double widen = __builtin_huge_val(), rfar = 0.0;
    {
        const double g0x = L.gen[0].x, g0y = L.gen[0].y;
        const double hx = L.gen[1 + i].x - g0x, hy = L.gen[1 + i].y - g0y;
        const double hmin = -wave_max(-sqrt(hx * hx + hy * hy));
        const double H2 = wave_max(hx * hx + hy * hy);
        // interior angle at vertex i: incoming edge a = v_i - v_{i-1},
        // outgoing b = v_{i+1} - v_i; sin(theta / 2) = sqrt((1 + a.b) / 2)
        // for unit a, b of a convex polygon
        const double2 vp = L.vtx[i == 0 ? n - 1 : i - 1], vn = L.vtx[i + 1 == n ? 0 : i + 1];
        const double ax = v.x - vp.x, ay = v.y - vp.y, bx = vn.x - v.x, by = vn.y - v.y;
        const double cosab = (ax * bx + ay * by) / (sqrt(ax * ax + ay * ay) * sqrt(bx * bx + by * by));
        const double smin = -wave_max(-sqrt(fmax(0.5 * (1.0 + cosab), 0.0)));
        const double ox = (double)L.ox, oy = (double)L.oy;
        const double rv = wave_max(sqrt((v.x - ox) * (v.x - ox) + (v.y - oy) * (v.y - oy)));
        const double d2 = (g0x - ox) * (g0x - ox) + (g0y - oy) * (g0y - oy);
        const double S = fmax(wave_max(fmax(fabs(v.x), fabs(v.y))), fmax(fabs(g0x), fabs(g0y)));
        const double dl = 64.0 * kU64 * S;                 // generator error bound
        const double hs = (hmin - dl) * smin;              // > 0 for a usable polygon
        const double e0 = 4.0001 * kU64 * (6.0 * d2 + 2.0 * H2);
        const double lev = sqrt(d2) + sqrt(H2) + dl;       // |p - R_i| - rho
        // t(rho) and the far quadratic qa rho^2 - qb rho + qc < 0
        const double rho2 = 2.0 * rv;
        const double t2 = (24.01 * kU64 * rho2 * rho2 + e0 + 2.0 * (rho2 + lev) * dl + dl * dl) /
                          (2.0 * (hmin - dl));
        const double w = 2.0 * t2 / smin * 1.01;
        const double qa = 24.01 * kU64 * 1.01;
        const double qb = (2.0 * hs - 2.0 * dl) * 0.99;
        const double qc = (2.0 * hs * rv + e0 + 2.0 * lev * dl + dl * dl) * 1.01;
        const double disc = qb * qb - 4.0 * qa * qc;
        const bool near_ok = qa * rho2 * rho2 - qb * rho2 + qc < 0.0 && disc > 0.0;
        // p_0 strictly on the inner side of every edge line (its orientation
        // against edge i, with 8 v |e| |r| for the rounding of the cross
        // product): Algorithm 3 in the global frame can place the centroid
        // of a small polygon far from the origin outside it, and then the
        // set Algorithm 5 accepts is not the polygon
        const double ex = v.x - vp.x, ey = v.y - vp.y, rx = g0x - vp.x, ry = g0y - vp.y;
        const double cr = ex * ry - ey * rx;
        const double crb = 8.0 * kU64 * sqrt(ex * ex + ey * ey) * sqrt(rx * rx + ry * ry);
        const bool g0_in = -wave_max(-(cr - crb)) > 0.0 || wave_max(cr + crb) < 0.0;
        if (L.status == 0 && g0_in && hmin > 2.0 * dl && smin > 0.0 && w <= rv && w == w &&
            near_ok) {
            widen = w;
            rfar = (qb + sqrt(disc)) / (2.0 * qa) * 0.999;
        }
    }
    const double wx = widen + 4.0 * kU64 * fmax(fabs(xlo), fabs(xhi));
    const double wy = widen + 4.0 * kU64 * fmax(fabs(ylo), fabs(yhi));
    // query record at float4 offset v0 + 5k: header (2 float4), n4 rows
    const int64_t qbase = v0 + 5 * k, gbase = v0 + k;
    const int n4 = L.n4;
    if (lane < n4) qrec[qbase + 2 + lane] = L.coef[lane];
    if (lane == 0) {
        qrec[qbase] = make_float4(L.ox, L.oy, L.KQ, L.KA);
        qrec[qbase + 1] = make_float4(L.KB, L.KC, __int_as_float(n | (n4 << 16)),
                                      __int_as_float((int)gbase));
    }
    for (int r = lane; r <= n; r += kWave) gen[gbase + r] = L.gen[r];
    if (lane == 0) {
        R.ox = L.ox;
        R.oy = L.oy;
        R.KQ = L.KQ;
        R.KA = L.KA;
        R.KB = L.KB;
        R.KC = L.KC;
        R.n = n;
        R.n4 = n4;
        R.qoff = qbase;
        R.gen_off = gbase;
        R.status = L.status;
        R.usable = all_fin && widen < __builtin_huge_val() ? 1 : 2;  // 2: global list
        R.bx0 = round_out_lo(xlo - wx);
        R.by0 = round_out_lo(ylo - wy);
        R.bx1 = round_out_hi(xhi + wx);
        R.by1 = round_out_hi(yhi + wy);
        R.rfar = round_out_lo(rfar);
        rec[k] = R;
        if (status) status[k] = L.status;
    }
}

// One block: the near region (the box of the cell-listed boxes and local
// origins, widened by its diagonal on each side, rounded inwards), the
// demotion to the global list of polygons whose far radius does not cover
// it, then the union of the remaining cell-listed boxes and the grid shape.
__device__ __forceinline__ void block_min4(float (&v)[4], float (*red)[1024]) {
    const int t = threadIdx.x;
    for (int c = 0; c < 4; ++c) red[c][t] = v[c];
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s)
            for (int c = 0; c < 4; ++c) red[c][t] = fminf(red[c][t], red[c][t + s]);
        __syncthreads();
    }
    for (int c = 0; c < 4; ++c) v[c] = red[c][0];
    __syncthreads();
}

__global__ __launch_bounds__(1024) void k_index_bounds(int64_t P, LocRec* __restrict__ rec,
                                                     int64_t cells, LocGrid* __restrict__ grid) {
    __shared__ float red[4][1024];
    const int t = threadIdx.x;
    // near region from the cell-listed boxes and their local origins
    float u[4] = {__builtin_huge_valf(), __builtin_huge_valf(), __builtin_huge_valf(),
                  __builtin_huge_valf()};  // x0, y0, -x1, -y1
    for (int64_t k = t; k < P; k += blockDim.x) {
        const LocRec& R = rec[k];
        if (R.usable != 1) continue;
        u[0] = fminf(u[0], fminf(R.bx0, R.ox));
        u[1] = fminf(u[1], fminf(R.by0, R.oy));
        u[2] = fminf(u[2], -fmaxf(R.bx1, R.ox));
        u[3] = fminf(u[3], -fmaxf(R.by1, R.oy));
    }
    block_min4(u, red);
    const bool any_u = u[0] <= -u[2] && u[1] <= -u[3];
    // the region's diagonal (rounded up) and the near region U widened by it
    double diag = 0.0;
    if (any_u) {
        const double wx = (double)(-u[2]) - (double)u[0], wy = (double)(-u[3]) - (double)u[1];
        diag = sqrt(wx * wx + wy * wy) * (1.0 + 1e-12);
    }
    const float fx0 = round_out_hi((double)u[0] - diag), fy0 = round_out_hi((double)u[1] - diag);
    const float fx1 = round_out_lo((double)(-u[2]) + diag), fy1 = round_out_lo((double)(-u[3]) + diag);
    // a point of the near region is within (1 + 2 sqrt 2) diag < 4 diag of
    // every local origin
    const double need = 4.0 * diag * (1.0 + 1e-9);
    float x[4] = {__builtin_huge_valf(), __builtin_huge_valf(), __builtin_huge_valf(),
                  __builtin_huge_valf()};
    for (int64_t k = t; k < P; k += blockDim.x) {
        LocRec& R = rec[k];
        if (R.usable != 1) continue;
        if (!((double)R.rfar > need)) {
            R.usable = 2;
            continue;
        }
        x[0] = fminf(x[0], R.bx0);
        x[1] = fminf(x[1], R.by0);
        x[2] = fminf(x[2], -R.bx1);
        x[3] = fminf(x[3], -R.by1);
    }
    block_min4(x, red);
    if (t == 0) {
        LocGrid G;
        G.x0 = x[0];
        G.y0 = x[1];
        G.x1 = -x[2];
        G.y1 = -x[3];
        const bool any = G.x0 <= G.x1 && G.y0 <= G.y1;
        const double w = any ? (double)G.x1 - (double)G.x0 : 0.0;
        const double h = any ? (double)G.y1 - (double)G.y0 : 0.0;
        int gx = 1, gy = 1;
        if (w > 0.0 && h > 0.0) {
            gx = (int)fmin(fmax(rint(sqrt((double)cells * w / h)), 1.0), (double)cells);
            gy = (int)fmax((double)(cells / gx), 1.0);
        } else if (w > 0.0) {
            gx = (int)cells;
        } else if (h > 0.0) {
            gy = (int)cells;
        }
        G.gx = gx;
        G.gy = gy;
        G.inv_w = w > 0.0 ? (float)((double)gx / w) : 0.0f;
        G.inv_h = h > 0.0 ? (float)((double)gy / h) : 0.0f;
        G.any = any ? 1 : 0;
        // no cell-listed polygon: every point takes the global list only
        G.fx0 = any_u ? fx0 : -__builtin_huge_valf();
        G.fy0 = any_u ? fy0 : -__builtin_huge_valf();
        G.fx1 = any_u ? fx1 : __builtin_huge_valf();
        G.fy1 = any_u ? fy1 : __builtin_huge_valf();
        *grid = G;
    }
}

__global__ void k_index_zero(int32_t* __restrict__ p, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

// FILL = false: count entries per cell (and their total); true: write them.
template <bool FILL>
__global__ void k_index_cells(int64_t P, const LocRec* __restrict__ rec,
                              const LocGrid* __restrict__ grid, int32_t* __restrict__ cnt,
                              const int32_t* __restrict__ cell_off, LocEntry* __restrict__ list,
                              unsigned long long* __restrict__ total) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P) return;
    const LocRec R = rec[k];
    LocEntry en;
    en.bx0 = R.bx0;
    en.by0 = R.by0;
    en.bx1 = R.bx1;
    en.by1 = R.by1;
    en.k = (int)k;
    en.qoff = (int)R.qoff;
    en.nn = R.n | (R.n4 << 16);
    en.pad = 0;
    if (R.usable == 2) {  // global list: its count sits after the cells'
        const int64_t C = (int64_t)grid->gx * grid->gy;
        if (!FILL) atomicAdd(total, 1ull);
        const int slot = atomicAdd(&cnt[C], 1);
        if (FILL) list[cell_off[C] + slot] = en;
        return;
    }
    if (R.usable != 1) return;
    const LocGrid G = *grid;
    const int cx0 = cell_of(R.bx0, G.x0, G.inv_w, G.gx), cx1 = cell_of(R.bx1, G.x0, G.inv_w, G.gx);
    const int cy0 = cell_of(R.by0, G.y0, G.inv_h, G.gy), cy1 = cell_of(R.by1, G.y0, G.inv_h, G.gy);
    if (!FILL) atomicAdd(total, (unsigned long long)(cx1 - cx0 + 1) * (unsigned long long)(cy1 - cy0 + 1));
    for (int cy = cy0; cy <= cy1; ++cy)
        for (int cx = cx0; cx <= cx1; ++cx) {
            const int64_t c = (int64_t)cy * G.gx + cx;
            const int slot = atomicAdd(&cnt[c], 1);
            if (FILL) list[cell_off[c] + slot] = en;
        }
}

// Each list (the cells', then the global list) in ascending polygon index,
// so that a point's first containing candidate is its answer and its later
// box hits skip their records.  One thread per list, insertion sort; lists
// longer than kSortMax keep their order (the answer does not depend on it).
constexpr int kSortMax = 64;
__global__ void k_index_sort(int64_t nlists, const int32_t* __restrict__ cell_off,
                             LocEntry* __restrict__ list) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nlists) return;
    const int b = cell_off[i], e = cell_off[i + 1];
    if (e - b > kSortMax) return;
    for (int a = b + 1; a < e; ++a) {
        const LocEntry x = list[a];
        int j = a;
        while (j > b && list[j - 1].k > x.k) {
            list[j] = list[j - 1];
            --j;
        }
        list[j] = x;
    }
}

// Exclusive scan of count[0..C) into off[0..C] in one block.
__global__ __launch_bounds__(1024) void k_index_scan(int64_t C, const int32_t* __restrict__ count,
                                                   int32_t* __restrict__ off) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (C + blockDim.x - 1) / blockDim.x;
    const int64_t b = t * per, e = b + per < C ? b + per : C;
    int64_t s = 0;
    for (int64_t i = b; i < e; ++i) s += count[i];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t acc = 0;
        for (int i = 0; i < (int)blockDim.x; ++i) {
            const int64_t v = part[i];
            part[i] = acc;
            acc += v;
        }
    }
    __syncthreads();
    int64_t acc = part[t];
    for (int64_t i = b; i < e; ++i) {
        off[i] = (int32_t)acc;
        acc += count[i];
    }
    if (e == C && b < e) off[C] = (int32_t)acc;
    if (C == 0 && t == 0) off[0] = 0;
}

constexpr int kScanBatch = 8;  // cell entries per round trip (a cell holds ~5 on average)

// Smallest index of a polygon containing p, or -1: the candidates of p's
// cell (their boxes first: only box hits read a record), then the global
// list.  Each candidate: float32 screen, binary64 replay inside the band; a
// NaN box (non-finite vertices) never rejects.  A point beyond the near
// region tests every polygon in index order; a non-finite point is outside
// every polygon.
__device__ __forceinline__ int locate_point(float2 p, const LocGrid& G,
                                            const int32_t* __restrict__ cell_off,
                                            const LocEntry* __restrict__ list,
                                            const float4* __restrict__ qrec,
                                            const double2* __restrict__ gen, int gbeg, int gend,
                                            const LocRec* __restrict__ rec, int64_t P) {
    int id = -1;
    if (!(isfinite(p.x) && isfinite(p.y))) return -1;
    // polygon k (record at qoff) contains p: float32 screen, binary64 inside the band
    auto inside = [&](int qoff, int nn) -> bool {
        const float4* r = qrec + qoff;
        const int n = nn & 0xffff, n4 = nn >> 16;
        // the header and the first four rows in one round trip
        const float4 h0 = r[0], h1 = r[1];
        float4 c4[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) c4[e] = r[2 + (e < n4 ? e : 0)];
        const float X = p.x - h0.x, Y = p.y - h0.y;
        float M = -__builtin_huge_valf();
#pragma unroll
        for (int e = 0; e < 4; ++e) M = fmaxf(M, fmaf(c4[e].x, X, fmaf(c4[e].y, Y, c4[e].z)));
        for (int e = 4; e < n4; ++e) {
            const float4 c = r[2 + e];
            M = fmaxf(M, fmaf(c.x, X, fmaf(c.y, Y, c.z)));
        }
        const float E =
            fmaf(h0.z, fmaf(X, X, Y * Y), fmaf(h0.w, fabsf(X), fmaf(h1.x, fabsf(Y), h1.y)));
        bool in = M < -E;
        if (!(fabsf(M) > E)) in = voronoi64((double)p.x, (double)p.y, gen + __float_as_int(h1.w), n);
        return in;
    };
    // entries [beg, end): kScanBatch at a time, their boxes and indices
    // loaded together (one memory round trip); the box hits become a bit mask
    // and each lane walks its own hits, so the lanes' record loads overlap.
    // Lists are in ascending polygon index (up to kSortMax entries), so hits
    // after a lane's first containing polygon skip their records.
    auto scan = [&](int beg, int end) {
        for (int t = beg; t < end; t += kScanBatch) {
            float4 box[kScanBatch];
            int4 kq[kScanBatch];  // k, qoff, n | n4 << 16
            // entries past the list's end are not loaded: the kernel is bound by
            // its memory requests more than by their latency
#pragma unroll
            for (int u = 0; u < kScanBatch; ++u) {
                box[u] = make_float4(0.f, 0.f, 0.f, 0.f);
                kq[u] = make_int4(0, 0, 0, 0);
                if (t + u < end) {
                    box[u] = *reinterpret_cast<const float4*>(&list[t + u]);
                    kq[u] = *reinterpret_cast<const int4*>(&list[t + u].k);
                }
            }
            uint32_t hits = 0;
#pragma unroll
            for (int u = 0; u < kScanBatch; ++u) {
                // a NaN box (non-finite vertices) never rejects
                const bool miss =
                    p.x < box[u].x || p.y < box[u].y || p.x > box[u].z || p.y > box[u].w;
                if (t + u < end && !miss) hits |= 1u << u;
            }
            while (hits) {
                const int u = __builtin_ctz(hits);
                hits &= hits - 1;
                int4 e = kq[0];
#pragma unroll
                for (int v = 1; v < kScanBatch; ++v)
                    if (u == v) e = kq[v];
                if (id >= 0 && e.x > id) continue;  // cannot lower the answer
                if (inside(e.y, e.z)) id = e.x;
            }
        }
    };
    if (!(p.x >= G.fx0 && p.x <= G.fx1 && p.y >= G.fy0 && p.y <= G.fy1)) {
        // beyond the near region: every polygon, in index order
        for (int64_t k = 0; k < P; ++k) {
            const LocRec& R = rec[k];
            if (R.usable != 0 && inside((int)R.qoff, R.n | (R.n4 << 16))) return (int)k;
        }
        return -1;
    }
    // outside the union of the cell boxes: only the global list
    if (G.any && p.x >= G.x0 && p.x <= G.x1 && p.y >= G.y0 && p.y <= G.y1) {
        const int64_t c =
            (int64_t)cell_of(p.y, G.y0, G.inv_h, G.gy) * G.gx + cell_of(p.x, G.x0, G.inv_w, G.gx);
        scan(cell_off[c], cell_off[c + 1]);
    }
    scan(gbeg, gend);
    return id;
}

__global__ __launch_bounds__(kBlock) void k_locate(const LocRec* __restrict__ rec, int64_t P,
                                                 const float4* __restrict__ qrec,
                                                 const double2* __restrict__ gen,
                                                 const LocGrid* __restrict__ grid,
                                                 const int32_t* __restrict__ cell_off,
                                                 const LocEntry* __restrict__ list,
                                                 const float2* __restrict__ Q, int64_t m,
                                                 int32_t* __restrict__ ids) {
    const LocGrid G = *grid;
    const int64_t C = (int64_t)G.gx * G.gy;
    const int gbeg = cell_off[C], gend = cell_off[C + 1];  // the global list
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        const vfloat2 pv = __builtin_nontemporal_load(reinterpret_cast<const vfloat2*>(Q) + i);
        ids[i] = locate_point(make_float2(pv.x, pv.y), G, cell_off, list, qrec, gen, gbeg, gend,
                              rec, P);
    }
}

// ---------------------------------------------------------------------------
// Coherent queries: the points are first binned by super-cell (sf x sf grid
// cells; bin nbins = outside the grid's box or NaN), so that the lanes of a
// wave share a few cells and their candidate loads hit the caches.
//   k_bin_points<false>  per-block LDS histogram of the bins, added to the
//                        global counts once per block;
//   k_bin_points<true>   the same histogram per tile, a global reservation per
//                        (tile, bin), then each point written to its slot;
//   k_locate_binned      binned points in order, ids written back by index.
// ---------------------------------------------------------------------------
constexpr int kBinPer = 16;                  // points per thread per tile
constexpr int kBinTile = kBlock * kBinPer;   // 4096 points

struct BinnedPt {
    float x, y;
    int32_t idx, pad;
};

__device__ __forceinline__ int bin_of(float2 p, const LocGrid& G, int sf, int sgx, int nbins) {
    if (!(G.any && p.x >= G.x0 && p.x <= G.x1 && p.y >= G.y0 && p.y <= G.y1)) return nbins;
    const int cy = cell_of(p.y, G.y0, G.inv_h, G.gy), cx = cell_of(p.x, G.x0, G.inv_w, G.gx);
    return (cy / sf) * sgx + cx / sf;
}

template <bool SCATTER>
__global__ __launch_bounds__(kBlock) void k_bin_points(const float2* __restrict__ Q, int64_t m,
                                                     const LocGrid* __restrict__ grid, int sf,
                                                     int sgx, int nbins,
                                                     int32_t* __restrict__ bin_cnt,
                                                     const int32_t* __restrict__ bin_off,
                                                     int32_t* __restrict__ bin_fill,
                                                     BinnedPt* __restrict__ binned) {
    extern __shared__ int32_t hist[];  // [nbins + 1] (+ [nbins + 1] bases when scattering)
    int32_t* base = hist + (nbins + 1);
    const int tid = threadIdx.x;
    const LocGrid G = *grid;
    const int64_t ntiles = (m + kBinTile - 1) / kBinTile;
    if (!SCATTER) {
        for (int b = tid; b <= nbins; b += kBlock) hist[b] = 0;
        __syncthreads();
    }
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        if (SCATTER) {
            for (int b = tid; b <= nbins; b += kBlock) hist[b] = 0;
            __syncthreads();
        }
        const int64_t i0 = tile * kBinTile;
        int bin[kBinPer], slot[kBinPer];
        float2 pt[kBinPer];
#pragma unroll
        for (int j = 0; j < kBinPer; ++j) {
            const int64_t i = i0 + j * kBlock + tid;
            bin[j] = -1;
            if (i < m) {
                const vfloat2 pv =
                    __builtin_nontemporal_load(reinterpret_cast<const vfloat2*>(Q) + i);
                pt[j] = make_float2(pv.x, pv.y);
                bin[j] = bin_of(pt[j], G, sf, sgx, nbins);
                slot[j] = atomicAdd(&hist[bin[j]], 1);
            }
        }
        if (SCATTER) {
            __syncthreads();
            for (int b = tid; b <= nbins; b += kBlock)
                base[b] = hist[b] ? bin_off[b] + atomicAdd(&bin_fill[b], hist[b]) : 0;
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kBinPer; ++j) {
                if (bin[j] >= 0) {
                    BinnedPt e;
                    e.x = pt[j].x;
                    e.y = pt[j].y;
                    e.idx = (int32_t)(j * kBlock + tid);  // within the tile
                    e.pad = (int32_t)tile;
                    binned[base[bin[j]] + slot[j]] = e;
                }
            }
            __syncthreads();  // hist and base are reused by the next tile
        }
    }
    if (!SCATTER) {
        __syncthreads();
        for (int b = tid; b <= nbins; b += kBlock)
            if (hist[b]) atomicAdd(&bin_cnt[b], hist[b]);
    }
}

// Binned points, a tile of kLocTile at a time: the tile is counting-sorted
// in LDS by the point's cell within its super-cell (sf * sf keys, one more
// for points outside the grid's box), so consecutive lanes share a cell and
// its candidates' loads are broadcasts; ids are written back by index.
// 512-thread blocks: the 37 KB of LDS per tile then serve 8 waves, and at
// 4 waves per SIMD (<= 128 VGPRs) two blocks share a CU.
constexpr int kLocBlock = 512;
constexpr int kLocPer = 4;
constexpr int kLocTile = kLocBlock * kLocPer;  // 2048 points
constexpr int kMaxKeys = 1025;                 // sf <= 32
constexpr int kScanPer = (kMaxKeys + kLocBlock - 1) / kLocBlock;

__global__ __launch_bounds__(kLocBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_locate_binned(
    const LocRec* __restrict__ rec, int64_t P, const float4* __restrict__ qrec, const double2* __restrict__ gen,
    const LocGrid* __restrict__ grid, const int32_t* __restrict__ cell_off,
    const LocEntry* __restrict__ list, const BinnedPt* __restrict__ binned, int64_t m, int sf,
    int32_t* __restrict__ ids) {
    __shared__ BinnedPt sorted_s[kLocTile];
    __shared__ int32_t key_s[kMaxKeys];
    __shared__ int32_t part_s[kLocBlock / kWave];
    const int tid = threadIdx.x;
    const LocGrid G = *grid;
    const int64_t C = (int64_t)G.gx * G.gy;
    const int gbeg = cell_off[C], gend = cell_off[C + 1];
    const bool local = sf <= 32;
    const int nkeys = local ? sf * sf + 1 : 1;
    const int64_t ntiles = (m + kLocTile - 1) / kLocTile;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t i0 = tile * kLocTile;
        const int cnt = (int)(m - i0 < kLocTile ? m - i0 : kLocTile);
        for (int k = tid; k < nkeys; k += kLocBlock) key_s[k] = 0;
        __syncthreads();
        BinnedPt e[kLocPer];
        int key[kLocPer], slot[kLocPer];
#pragma unroll
        for (int j = 0; j < kLocPer; ++j) {
            const int q = j * kLocBlock + tid;
            key[j] = -1;
            if (q < cnt) {
                e[j] = binned[i0 + q];
                const float2 p = make_float2(e[j].x, e[j].y);
                int k = nkeys - 1;  // outside the box (or NaN)
                if (local && G.any && p.x >= G.x0 && p.x <= G.x1 && p.y >= G.y0 && p.y <= G.y1)
                    k = (cell_of(p.y, G.y0, G.inv_h, G.gy) % sf) * sf + cell_of(p.x, G.x0, G.inv_w, G.gx) % sf;
                key[j] = k;
                slot[j] = atomicAdd(&key_s[k], 1);
            }
        }
        __syncthreads();
        // exclusive scan of the key counts: kScanPer keys per thread
        int run = 0;
        for (int u = 0; u < kScanPer; ++u) {
            const int k = tid * kScanPer + u;
            if (k < nkeys) run += key_s[k];
        }
        // exclusive over the block: a scan within the wave, then the totals
        // of the waves before this one
        const int lane = tid & (kWave - 1);
        int incl = run;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int t = __shfl_up(incl, d);
            if (lane >= d) incl += t;
        }
        if (lane == kWave - 1) part_s[tid / kWave] = incl;
        __syncthreads();
        int acc = incl - run;
        for (int w = 0; w < tid / kWave; ++w) acc += part_s[w];
        for (int u = 0; u < kScanPer; ++u) {
            const int k = tid * kScanPer + u;
            if (k < nkeys) {
                const int v = key_s[k];
                key_s[k] = acc;
                acc += v;
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kLocPer; ++j)
            if (key[j] >= 0) sorted_s[key_s[key[j]] + slot[j]] = e[j];
        __syncthreads();
        for (int q = tid; q < cnt; q += kLocBlock) {
            const BinnedPt b = sorted_s[q];
            const int id =
                locate_point(make_float2(b.x, b.y), G, cell_off, list, qrec, gen, gbeg, gend, rec, P);
            ids[(int64_t)b.pad * kBinTile + b.idx] = id;
        }
        __syncthreads();  // the tile's LDS is reused
    }
}

}  // namespace

namespace pipdev {

hipError_t index_prepare(int64_t P, const int64_t* vtx_off, const double* V, LocRec* rec,
                         float4* qrec, double2* gen, int32_t* status, int32_t* flags,
                         hipStream_t stream) {
    hipLaunchKernelGGL(k_index_zero, dim3(1), dim3(64), 0, stream, flags, (int64_t)1);
    if (P == 0) return hipGetLastError();
    const unsigned blocks = (unsigned)((P + kWavesPerBlock - 1) / kWavesPerBlock);
    hipLaunchKernelGGL(k_index_prepare, dim3(blocks), dim3(kBlock), 0, stream, P, vtx_off, V, rec,
                       qrec, gen, status, flags);
    return hipGetLastError();
}

// cnt: cells + 1 counters (cell counts, then the global list at gx * gy);
// total: entries of all lists (unsigned long long).
hipError_t index_grid(int64_t P, LocRec* rec, int64_t cells, LocGrid* grid, int32_t* cnt,
                      unsigned long long* total, hipStream_t stream) {
    hipLaunchKernelGGL(k_index_bounds, dim3(1), dim3(1024), 0, stream, P, rec, cells, grid);
    hipLaunchKernelGGL(k_index_zero, dim3((unsigned)((cells + 1 + 255) / 256)), dim3(256), 0,
                       stream, cnt, cells + 1);
    hipLaunchKernelGGL(k_index_zero, dim3(1), dim3(64), 0, stream,
                       reinterpret_cast<int32_t*>(total), (int64_t)2);
    if (P > 0)
        hipLaunchKernelGGL(k_index_cells<false>, dim3((unsigned)((P + 255) / 256)), dim3(256), 0,
                           stream, P, rec, grid, cnt, nullptr, nullptr, total);
    return hipGetLastError();
}

// cell_off: cells + 2 offsets (exclusive scan of cnt); list: total entries.
hipError_t index_fill(int64_t P, const LocRec* rec, const LocGrid* grid, int64_t cells,
                      int32_t* cnt, int32_t* cell_off, LocEntry* list, hipStream_t stream) {
    hipLaunchKernelGGL(k_index_scan, dim3(1), dim3(1024), 0, stream, cells + 1, cnt, cell_off);
    hipLaunchKernelGGL(k_index_zero, dim3((unsigned)((cells + 1 + 255) / 256)), dim3(256), 0,
                       stream, cnt, cells + 1);
    if (P > 0)
        hipLaunchKernelGGL(k_index_cells<true>, dim3((unsigned)((P + 255) / 256)), dim3(256), 0,
                           stream, P, rec, grid, cnt, cell_off, list, nullptr);
    hipLaunchKernelGGL(k_index_sort, dim3((unsigned)((cells + 1 + 255) / 256)), dim3(256), 0,
                       stream, cells + 1, cell_off, list);
    return hipGetLastError();
}

hipError_t launch_locate(const LocRec* rec, int64_t P, const float4* qrec, const double2* gen,
                         const LocGrid* grid, const int32_t* cell_off, const LocEntry* list,
                         const float* Q, int64_t m, int32_t* ids, int max_blocks,
                         hipStream_t stream) {
    if (m == 0) return hipSuccess;
    const int64_t want = (m + kBlock - 1) / kBlock;
    const int grid_blocks = (int)(want < max_blocks ? want : max_blocks);
    hipLaunchKernelGGL(k_locate, dim3(grid_blocks), dim3(kBlock), 0, stream, rec, P, qrec, gen, grid,
                       cell_off, list, reinterpret_cast<const float2*>(Q), m, ids);
    return hipGetLastError();
}

// Workspace of a binned query of m points with nbins super-cells.
size_t locate_binned_workspace(int nbins, int64_t m, size_t* o_cnt, size_t* o_off, size_t* o_fill,
                               size_t* o_pts) {
    auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
    size_t off = 0;
    *o_cnt = off;
    off = up(off + 4 * (size_t)(nbins + 1));
    *o_off = off;
    off = up(off + 4 * (size_t)(nbins + 2));
    *o_fill = off;
    off = up(off + 4 * (size_t)(nbins + 1));
    *o_pts = off;
    off = up(off + sizeof(BinnedPt) * (size_t)(m > 0 ? m : 1));
    return off;
}

hipError_t launch_locate_binned(const LocRec* rec, int64_t P, const float4* qrec,
                                const double2* gen, const LocGrid* grid,
                                const int32_t* cell_off, const LocEntry* list, int sf, int sgx,
                                int nbins, const float* Q, int64_t m, int32_t* ids, void* ws,
                                int cus, hipStream_t stream) {
    if (m == 0) return hipSuccess;
    size_t o_cnt, o_off, o_fill, o_pts;
    locate_binned_workspace(nbins, m, &o_cnt, &o_off, &o_fill, &o_pts);
    char* b = static_cast<char*>(ws);
    int32_t* cnt = reinterpret_cast<int32_t*>(b + o_cnt);
    int32_t* boff = reinterpret_cast<int32_t*>(b + o_off);
    int32_t* fill = reinterpret_cast<int32_t*>(b + o_fill);
    BinnedPt* pts = reinterpret_cast<BinnedPt*>(b + o_pts);
    const float2* Q2 = reinterpret_cast<const float2*>(Q);
    const unsigned zb = (unsigned)((nbins + 1 + 255) / 256);
    hipLaunchKernelGGL(k_index_zero, dim3(zb), dim3(256), 0, stream, cnt, (int64_t)(nbins + 1));
    hipLaunchKernelGGL(k_index_zero, dim3(zb), dim3(256), 0, stream, fill, (int64_t)(nbins + 1));
    const int64_t ntiles = (m + kBinTile - 1) / kBinTile;
    const int64_t bmax = (int64_t)cus * 4;
    const unsigned bb = (unsigned)(ntiles < bmax ? ntiles : bmax);
    hipLaunchKernelGGL(k_bin_points<false>, dim3(bb), dim3(kBlock), 4 * (size_t)(nbins + 1), stream,
                       Q2, m, grid, sf, sgx, nbins, cnt, nullptr, nullptr, nullptr);
    hipLaunchKernelGGL(k_index_scan, dim3(1), dim3(1024), 0, stream, (int64_t)(nbins + 1), cnt, boff);
    hipLaunchKernelGGL(k_bin_points<true>, dim3(bb), dim3(kBlock), 8 * (size_t)(nbins + 1), stream,
                       Q2, m, grid, sf, sgx, nbins, nullptr, boff, fill, pts);
    // one block per tile (m < 2^31: fewer than 2^20 tiles): more blocks than
    // fit on the chip at once even out the end of the launch
    const int64_t tiles = (m + kLocTile - 1) / kLocTile;
    hipLaunchKernelGGL(k_locate_binned, dim3((unsigned)tiles), dim3(kLocBlock), 0, stream, rec, P,
                       qrec, gen,
                       grid, cell_off, list, pts, m, sf, ids);
    return hipGetLastError();
}

hipError_t locate_max_blocks_per_cu(int* out) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, (const void*)k_locate, kBlock, 0);
}

}  // namespace pipdev
