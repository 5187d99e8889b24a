// Device-side building blocks shared by the HIP kernels of the library.
//
// Polygon preparation follows Section 3 of Zengin & Sezer (arXiv:2007.15385):
// the centroid of Eq. 3-4 / Algorithm 3 is the inner generator p_0, and every
// edge contributes an outer generator, p_0 mirrored across the edge line
// (Eq. 5-8 / Algorithm 4).  The inclusion test of Section 4 (Eq. 1, 9-11 /
// Algorithm 5) compares squared distances; rearranged (Eq. 11) it is the sign
// of an affine margin per edge,
//     m_i(p) = |p - p_0|^2 - |p - p_i|^2 = 2 (p - o).h_i - (|p_i - o|^2 - |p_0 - o|^2),
// with h_i = p_i - p_0 and any origin o.  The streaming kernels evaluate m_i
// in float32 in a polygon-local frame (o = p_0 rounded to float32) and only
// decide a point when the float32 result is farther from zero than a proven
// bound on its distance from the binary64 evaluation of Algorithm 5; the
// rest are recomputed in binary64 with exactly the operation sequence of
// Algorithm 5, so every label equals the binary64 answer.
//
// All binary64 code is compiled with -ffp-contract=off: no multiply-add is
// fused and each expression is evaluated as written, so generator derivation
// and recheck reproduce the IEEE binary64 results of a plain sequential
// implementation bit for bit.  float32 multiply-adds are written explicitly
// with fmaf().
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace pipdev {

constexpr int kWave = 64;
constexpr int kMaxEdges = 64;
constexpr int kBlock = 256;                 // 4 waves per workgroup
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kPPL = 4;                     // points per lane per chunk
constexpr int kChunk = kWave * kPPL;        // 256 points per wave iteration
constexpr int kWordsPerChunk = kChunk / 32; // 8 label words
constexpr int kQueueCap = 256;              // per-wave queue of undecided points

// Device status codes (same numbering as the C-ABI's pip_status).
constexpr int ST_OK = 0;
constexpr int ST_INVAL = 1;       // non-finite vertex
constexpr int ST_DEGENERATE = 2;  // zero area or zero-length edge
constexpr int ST_NONCONVEX = 3;


typedef float vfloat2 __attribute__((ext_vector_type(2)));

// Unit roundoffs.
constexpr double kU32 = 5.9604644775390625e-08;   // 2^-24
constexpr double kU64 = 1.1102230246251565e-16;   // 2^-53
constexpr double kEpsAbs = 7.888609052210118e-31;  // 2^-100, covers float32 underflow
constexpr double kCoefLimit = 1.152921504606846976e18;  // 2^60

// Per-polygon data staged in LDS by the preparation step.
struct alignas(32) PolyLds {
    double2 vtx[kMaxEdges];          // vertices v_0..v_{n-1}
    double2 gen[kMaxEdges + 1];      // p_0, then p_i for edge i (v_{i-1} -> v_i)
    float4 coef[kMaxEdges];          // float32 filter coefficients, padded by copies of edge 0
    union {
        struct {
            double4 ray[kMaxEdges];  // ray crossing: (V'_y, V_y, dV_x, dV_y)
            double rhs[kMaxEdges];   // ray crossing: RHS of the line equation
        };
        uint32_t aux[kMaxEdges * 10];  // free for kernels that never take the ray-crossing test
    };
    float ox, oy;                    // float32 local origin
    float KQ, KA, KB, KC;            // band E = KQ (X^2 + Y^2) + KA |X| + KB |Y| + KC
    float RQ;                        // for |X|, |Y| <= RQ, E = KA |X| + KB |Y| + KC suffices
    float SO;                        // sign of offset: fl32(|X| + |Y|) < SO proves an inner edge (0: never)
    int n, n4, status;
};

// ----------------------------------------------------------------------------
// small helpers
// ----------------------------------------------------------------------------
__device__ __forceinline__ int prev_edge(int i, int n) { return i == 0 ? n - 1 : i - 1; }

__device__ __forceinline__ float round_up_f32(double d) {
    // smallest float32 >= d (d >= 0); +inf stays +inf, NaN becomes +inf
    if (!(d == d)) return __builtin_huge_valf();
    float f = (float)d;
    if ((double)f < d) f = __uint_as_float(__float_as_uint(f) + 1u);  // next float up (f >= 0)
    return f;
}

__device__ __forceinline__ float ceil_f32(double d) {
    // smallest float32 >= d (any sign); +-inf and NaN map to themselves
    float f = (float)d;
    if ((double)f < d) {
        const uint32_t b = __float_as_uint(f);
        f = f == 0.0f ? __uint_as_float(1u)             // smallest positive subnormal
          : f > 0.0f  ? __uint_as_float(b + 1u)         // away from zero
                      : __uint_as_float(b - 1u);        // towards zero
    }
    return f;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// largest float32 <= d for d >= 0 (at most FLT_MAX); 0 for NaN
__device__ __forceinline__ float round_down_f32(double d) {
    if (!(d > 0.0)) return 0.0f;
    if (d >= 3.4028234663852886e38) return 3.4028234663852886e38f;
    float f = (float)d;
    if ((double)f > d) f = __uint_as_float(__float_as_uint(f) - 1u);
    return f;
}

// Fold of the quadratic band term into the linear ones near the polygon: for
// |X|, |Y| <= RQ, KQ (X^2 + Y^2) <= KQ RQ (|X| + |Y|).  RQ is the largest
// power of two with KQ RQ <= 2^-8 min(KA, KB) (at most 2^60), so the linear
// constants grow by at most 2^-8 of themselves.  Returns RQ (0: no fold).
__device__ inline double fold_band(double KQ, double& KA, double& KB) {
    const double kmin = fmin(KA, KB);
    if (!(kmin > 0.0 && kmin < 1e300)) return 0.0;
    int e = 0;
    (void)frexp(kmin * 0.00390625 / KQ, &e);  // value in [2^(e-1), 2^e)
    const double RQ = ldexp(1.0, e - 1 < 60 ? e - 1 : 60);
    KA += KQ * RQ;
    KB += KQ * RQ;
    return RQ;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// ----------------------------------------------------------------------------
// Section 3: centroid (Eq. 3-4, Algorithm 3) and generators (Eq. 5-8,
// Algorithm 4), binary64.  Every lane of the calling wave evaluates the
// centroid (identical sequential sums, i = 0 upwards); lane i < n then
// derives the outer generator of edge i.  Returns the centroid; *gx, *gy get
// lane i's generator (unspecified for lanes >= n), *area the signed area.
// ----------------------------------------------------------------------------
__device__ inline void derive_generators(const double2* vtx, int n, int lane, double* g0x,
                                         double* g0y, double* area, double* gx, double* gy,
                                         double* den_out) {
    double S = 0.0, Sx = 0.0, Sy = 0.0;
    for (int i = 0; i < n; ++i) {
        const int j = prev_edge(i, n);
        const double vx = vtx[i].x, vy = vtx[i].y;
        const double wx = vtx[j].x, wy = vtx[j].y;
        const double Ai = wx * vy - vx * wy;
        S = S + Ai;
        Sx = Sx + (vx + wx) * Ai;
        Sy = Sy + (vy + wy) * Ai;
    }
    const double a = 0.5 * S;
    const double cx = Sx / (6.0 * a);
    const double cy = Sy / (6.0 * a);
    *g0x = cx;
    *g0y = cy;
    *area = a;
    const int i = lane < n ? lane : 0;
    const int j = prev_edge(i, n);
    const double vx = vtx[i].x, vy = vtx[i].y;
    const double wx = vtx[j].x, wy = vtx[j].y;
    const double ea = vy - wy;
    const double eb = wx - vx;
    const double ec = -(ea * vx + eb * vy);
    const double w11 = eb * eb - ea * ea;
    const double w12 = (-2.0 * ea) * eb;
    const double w22 = ea * ea - eb * eb;
    const double dx = w11 * cx + w12 * cy;
    const double dy = w12 * cx + w22 * cy;
    const double ex = (-2.0 * ec) * ea;
    const double ey = (-2.0 * ec) * eb;
    const double den = ea * ea + eb * eb;
    *gx = (dx + ex) / den;
    *gy = (dy + ey) / den;
    *den_out = den;
}

// Validation of one polygon by one wave (lane i looks at vertex/edge i):
// non-finite vertex -> ST_INVAL; zero area or zero-length edge ->
// ST_DEGENERATE; mixed turn directions -> ST_NONCONVEX (checked only when
// check_convex).  Collinear consecutive edges are allowed.
__device__ inline int validate_polygon(const double2* vtx, int n, int lane, double area, double den,
                                       bool check_convex) {
    const bool act = lane < n;
    const double2 v = vtx[act ? lane : 0];
    const bool nonfinite = act && !(isfinite(v.x) && isfinite(v.y));
    const bool zero_edge = act && !(den > 0.0);
    int turn = 0;
    if (act) {
        const double2 a = vtx[prev_edge(lane, n)];
        const double2 c = vtx[lane + 1 < n ? lane + 1 : 0];
        const double cr = (v.x - a.x) * (c.y - v.y) - (v.y - a.y) * (c.x - v.x);
        turn = cr > 0.0 ? 1 : (cr < 0.0 ? -1 : 0);
    }
    const uint64_t bad_v = __ballot(nonfinite);
    const uint64_t bad_e = __ballot(zero_edge);
    const uint64_t pos = __ballot(turn > 0);
    const uint64_t neg = __ballot(turn < 0);
    if (bad_v) return ST_INVAL;
    if (bad_e || !(area != 0.0) || !isfinite(area)) return ST_DEGENERATE;
    if (check_convex && pos && neg) return ST_NONCONVEX;
    return ST_OK;
}

// ----------------------------------------------------------------------------
// Preparation of one polygon into LDS by one wave.  The caller has written
// S.vtx[0..n) and S.n; all 64 lanes of the wave must call this.
//
// Band for the Voronoi margin (per point, X = fl32(p_x - o_x), Y likewise):
//   |m_hat_i - (fl64(M_0) - fl64(M_i))| <= E = KQ (X^2+Y^2) + KA|X| + KB|Y| + KC
// where m_hat_i = fma(A_i, X, fma(B_i, Y, -C_i)) with A_i, B_i, C_i the
// float32-rounded coefficients, M_0, M_i the binary64 squared distances of
// Algorithm 5.  Derivation (u = 2^-24, v = 2^-53, first order plus slack):
//   coefficient rounding + local coordinates + two fma roundings
//     <= 4.05 u (alpha|X| + beta|Y| + gamma) + 4.1 v (G2 + d2),
//   binary64 squared distances (relative error (1+v)^4 - 1 each)
//     <= 4.0001 v (M_0 + M_i) <= 24.01 v (X^2 + Y^2) + 4.0001 v (6 d2 + 2 H2),
// with alpha, beta, gamma the largest |A_i|, |B_i|, |C_i|, H2 = max |h_i|^2,
// d2 = |p_0 - o|^2, G2 = max |p_i - o|^2.  All constants are inflated by
// (1 + 2^-20) to cover the float32 evaluation of E and rounded upwards.
// A polygon whose coefficients are not finite or exceed 2^60 gets KC = +inf
// (every point goes to the binary64 path), and X^2 overflows to +inf for
// |X| >= 2^64, so no float32 margin can overflow undetected.
//
// Sign-of-offset band: the test of Algorithm 2 compares LHS = Q_y dV_x -
// Q_x dV_y with RHS = V'_y dV_x - V'_x dV_y; the filter evaluates
// s_hat_i = fma(-dV_y, X, fma(dV_x, Y, -R_i)) with R_i = RHS in the local
// frame, and the binary64 evaluation errs by at most
// 2.0001 v (|dV_x| (|Q_y| + |V'_y|) + |dV_y| (|Q_x| + |V'_x|)).
// ----------------------------------------------------------------------------
// f32_factor: multiple of u bounding the float32 evaluation of one margin
// relative to alpha|X| + beta|Y| + gamma: 4.05 for the two-fma screen; 6.05
// when the margin comes from a matrix-core multiply-add (exact products, up to
// two roundings of the sum, measured <= 1.96 u of the sum of |terms|, bounded
// here by 4 u, plus the same coefficient and coordinate rounding).
// given_frame: the local frame is (gox, goy) instead (one frame shared by
// several polygons); the band holds for any float32 origin.
__device__ inline void prepare_polygon(PolyLds& S, int kind, int lane, bool global_frame = false,
                                       double f32_factor = 4.05, bool given_frame = false,
                                       float gox = 0.0f, float goy = 0.0f) {
    const int n = S.n;
    double g0x, g0y, area, gx, gy, den;
    derive_generators(S.vtx, n, lane, &g0x, &g0y, &area, &gx, &gy, &den);
    const int status = validate_polygon(S.vtx, n, lane, area, den, kind == K_VORONOI || kind == K_SOO);
    if (lane < n) S.gen[1 + lane] = make_double2(gx, gy);
    if (lane == 0) S.gen[0] = make_double2(g0x, g0y);

    // Local frame o = fl32(p_0) (Voronoi), fl32 of the vertex mean (sign of
    // offset and ray crossing, whose offsets do not involve p_0: the binary64
    // centroid of a polygon that is tiny against its distance from the
    // origin can lie far from it, the vertex mean cannot), or the global
    // frame (o = 0, so X = p_x exactly); the bands below hold for any frame.
    double fx = g0x, fy = g0y;
    if (kind == K_SOO || kind == K_RAY32) {
        fx = wave_sum(lane < n ? S.vtx[lane].x : 0.0) / (double)n;
        fy = wave_sum(lane < n ? S.vtx[lane].y : 0.0) / (double)n;
    }
    const float ox = given_frame ? gox : global_frame ? 0.0f : (float)fx;
    const float oy = given_frame ? goy : global_frame ? 0.0f : (float)fy;
    const double dox = (double)ox, doy = (double)oy;
    const int i = lane < n ? lane : 0;
    const double d2x = g0x - dox, d2y = g0y - doy;
    const double d2 = d2x * d2x + d2y * d2y;
    double qa = 0.0, qb = 0.0, qc = 0.0, KA = 0.0, KB = 0.0, KC = 0.0, KQ = 0.0, RQ = 0.0;
    double soL = 0.0, soMx = 0.0, soMy = 0.0;  // sign of offset: the one-sided screen's sums
    bool finite_ok = true;
    if (kind == K_VORONOI || kind == K_MARGIN) {
        const double hx = gx - g0x, hy = gy - g0y;
        const double A = 2.0 * hx, B = 2.0 * hy;
        const double ux = gx - dox, uy = gy - doy;
        const double gi2 = ux * ux + uy * uy;
        const double C = gi2 - d2;
        const float a = (float)A, b = (float)B, c = (float)C;
        S.coef[lane] = make_float4(a, b, -c, 0.0f);
        finite_ok = isfinite(a) && isfinite(b) && isfinite(c) && fabs((double)a) < kCoefLimit &&
                    fabs((double)b) < kCoefLimit && fabs((double)c) < kCoefLimit;
        const double alpha = wave_max(fabs((double)a));
        const double beta = wave_max(fabs((double)b));
        const double gam = wave_max(fabs((double)c));
        const double H2 = wave_max(hx * hx + hy * hy);
        const double G2 = wave_max(gi2);
        const double infl = 1.0 + 9.5367431640625e-07;  // 1 + 2^-20
        KA = f32_factor * kU32 * alpha * infl;
        KB = f32_factor * kU32 * beta * infl;
        KC = (f32_factor * kU32 * gam + 4.1 * kU64 * (G2 + d2) +
              4.0001 * kU64 * (6.0 * d2 + 2.0 * H2) + kEpsAbs * (1.0 + alpha + beta)) * infl;
        KQ = 24.01 * kU64 * infl;
        RQ = fold_band(KQ, KA, KB);
        (void)qa; (void)qb; (void)qc;
    } else if (kind == K_SOO || kind == K_RAY32) {
        const int j = prev_edge(i, n);
        const double2 v = S.vtx[i], w = S.vtx[j];
        const double dVx = v.x - w.x, dVy = v.y - w.y;
        const double R = (w.y - doy) * dVx - (w.x - dox) * dVy;
        const float p = (float)(-dVy), q = (float)dVx, r = (float)R;
        // ray crossing: the row negated for an edge going down (V_y <= V'_y,
        // on the left when LHS < RHS), so that "on the left" is s > 0 for
        // every edge (negation is exact); and the height of the edge's end
        // vertex rounded up to float32, c: for a float32 Q_y, V_y > Q_y
        // exactly when c > Q_y
        // sign of offset: every row negated for a clockwise polygon, so that
        // the inner side of every edge is s > 0 (the labels do not change:
        // the test accepts either orientation).  The orientation is the sign
        // of C = -sum(V'_y dV_x - V'_x dV_y) (below), formed from the edge
        // vectors and so accurate where the shoelace sum of a tiny polygon
        // far from the origin (the centroid's area) is not.
        const bool act = lane < n;
        const double soC = kind == K_SOO ? -wave_sum(act ? w.y * dVx - w.x * dVy : 0.0) : 0.0;
        if (kind == K_RAY32) {
            const float sg = v.y > w.y ? 1.0f : -1.0f;
            S.coef[lane] = make_float4(sg * p, sg * q, -(sg * r), ceil_f32(v.y));
        } else {
            const float sg = soC < 0.0 ? -1.0f : 1.0f;
            S.coef[lane] = make_float4(sg * p, sg * q, -(sg * r), 0.0f);
        }
        finite_ok = isfinite(p) && isfinite(q) && isfinite(r) && fabs((double)p) < kCoefLimit &&
                    fabs((double)q) < kCoefLimit && fabs((double)r) < kCoefLimit;
        const double pm = wave_max(fabs((double)p));
        const double qm = wave_max(fabs((double)q));
        const double rm = wave_max(fabs((double)r));
        const double dxm = wave_max(fabs(dVx));
        const double dym = wave_max(fabs(dVy));
        // binary64 LHS/RHS error terms that do not scale with |X|, |Y|, and
        // the binary64 error of R itself
        const double k64 = wave_max(fabs(dVx) * (fabs(doy) + fabs(w.y)) +
                                    fabs(dVy) * (fabs(dox) + fabs(w.x)));
        const double kR = wave_max(fabs(w.y - doy) * fabs(dVx) + fabs(w.x - dox) * fabs(dVy));
        const double infl = 1.0 + 9.5367431640625e-07;
        KA = (f32_factor * kU32 * pm + 2.0001 * kU64 * dym) * infl;
        KB = (f32_factor * kU32 * qm + 2.0001 * kU64 * dxm) * infl;
        KC = (f32_factor * kU32 * rm + 3.1 * kU64 * kR + 2.0001 * kU64 * k64 +
              kEpsAbs * (1.0 + pm + qm)) * infl;
        KQ = kEpsAbs;  // no quadratic term; keeps X^2 overflow -> E = +inf
        if (kind == K_SOO) {
            RQ = fold_band(KQ, KA, KB);
            // One-sided screen.  With the rounded edge vectors (dV_x, dV_y)
            // of Algorithm 2, the exact offsets s_i = LHS_i - RHS_i of a point
            // Q sum to C + Q_y sum(dV_x) - Q_x sum(dV_y), C = -sum(V'_y dV_x -
            // V'_x dV_y) (twice the signed area when the edge vectors close
            // up exactly).  With the rows oriented by sg, some edge has
            // sg s_i >= (sg C - |sum dV_x| |Q_y| - |sum dV_y| |Q_x|) / n; when
            // that exceeds the band, that edge's binary64 comparison falls on
            // the inner side, and a point certified on the outer side of one
            // edge is certified outside.  The sums are bounded for any
            // summation order by 80 v of the sums of absolute values
            // (>= gamma_{n+2} for n <= 64); SO below turns the condition into
            // one float32 comparison per point.
            const double sg = soC < 0.0 ? -1.0 : 1.0;
            const double g = 80.0 * kU64;
            const double Ca = wave_sum(act ? fabs(w.y * dVx) + fabs(w.x * dVy) : 0.0);
            soL = sg * soC - g * Ca;  // <= sg C
            soMx = fabs(wave_sum(act ? dVx : 0.0)) + g * wave_sum(act ? fabs(dVx) : 0.0);
            soMy = fabs(wave_sum(act ? dVy : 0.0)) + g * wave_sum(act ? fabs(dVy) : 0.0);
        }
    }
    if (kind == K_RAY || kind == K_RAY32) {
        const int j = prev_edge(i, n);
        const double2 v = S.vtx[i], w = S.vtx[j];
        const double dVx = v.x - w.x, dVy = v.y - w.y;
        if (lane < n) {
            S.ray[lane] = make_double4(w.y, v.y, dVx, dVy);
            S.rhs[lane] = w.y * dVx - w.x * dVy;
        }
    }
    const uint64_t bad = __ballot(!finite_ok);
    // Sign of offset: |Q_x| <= |o_x| + |X| / (1 - u) (X = fl32(Q_x - o_x)),
    // |X| + |Y| <= fl32(|X| + |Y|) / (1 - u), and the folded band
    // E <= KS (|X| + |Y|) + KC with KS = max(KA, KB) for |X|, |Y| <= RQ
    // (stored, rounded-up constants).  The one-sided condition above then
    // holds whenever fl32(|X| + |Y|) < SO with
    //   SO <= (1 - u) T / (n KS + max(Mx, My) / (1 - u)),
    //   T = L - Mx |o_y| - My |o_x| - n KC,
    // L <= sg C, Mx >= |sum dV_x|, My >= |sum dV_y|; the factors 1 +- 2^-40
    // and 1 - 2^-20 cover the binary64 evaluation here, and SO <= RQ / 2
    // keeps |X|, |Y| <= RQ.  Unusable polygons get SO = 0 (never).
    float SO = 0.0f;
    if (kind == K_SOO) {
        const double KSs = fmax((double)round_up_f32(KA), (double)round_up_f32(KB));
        const double KCs = (double)round_up_f32(KC);
        const double T = soL - (soMx * fabs(doy) + soMy * fabs(dox) + (double)n * KCs) * (1.0 + 0x1p-40);
        const double den = (double)n * KSs * (1.0 + 0x1p-40) + fmax(soMx, soMy) * (1.0 + 0x1p-20);
        SO = fminf(round_down_f32(T * (1.0 - 0x1p-20) / den), (float)(0.5 * RQ));
        if (status != ST_OK || bad) SO = 0.0f;
    }
    if (lane == 0) {
        S.ox = ox;
        S.oy = oy;
        S.KQ = round_up_f32(KQ);
        S.KA = round_up_f32(KA);
        S.KB = round_up_f32(KB);
        S.KC = bad ? __builtin_huge_valf() : round_up_f32(KC);
        S.RQ = (float)RQ;  // a power of two (or 0), exact in float32
        S.SO = SO;
        S.n4 = (n + 3) & ~3;
        S.status = status;
    }
}

// ----------------------------------------------------------------------------
// binary64 decisions, replaying the plain algorithms operation by operation
// ----------------------------------------------------------------------------
// Algorithm 5 (Eq. 1, 10-11): inside iff M_0 <= M_i for every i; a point
// with a non-finite coordinate is outside.
__device__ inline bool voronoi64(double px, double py, const double2* gen, int n) {
    bool in = isfinite(px) && isfinite(py);
    const double dx0 = px - gen[0].x;
    const double dy0 = py - gen[0].y;
    const double M0 = dx0 * dx0 + dy0 * dy0;
    for (int i = 0; i < n; ++i) {
        const double dx = px - gen[1 + i].x;
        const double dy = py - gen[1 + i].y;
        const double Mi = dx * dx + dy * dy;
        if (!(M0 <= Mi)) in = false;
    }
    return in;
}

// Algorithm 2: D_i = LHS < RHS, inside iff (sum D_i) mod n == 0.
__device__ inline bool sign_of_offset64(double px, double py, const double2* vtx, int n) {
    int count = 0;
    for (int i = 0; i < n; ++i) {
        const int j = prev_edge(i, n);
        const double dVx = vtx[i].x - vtx[j].x;
        const double dVy = vtx[i].y - vtx[j].y;
        const double LHS = py * dVx - px * dVy;
        const double RHS = vtx[j].y * dVx - vtx[j].x * dVy;
        if (LHS < RHS) count += 1;
    }
    return ((count % n) == 0) && isfinite(px) && isfinite(py);
}

// Ray crossing of one point in binary64 (Section 2.1, Algorithm 1) from the
// ray table (V'_y, V_y, dV_x, dV_y) and RHS of each edge V' -> V.
__device__ inline bool ray_crossing64(double px, double py, const double4* ray, const double* rhs,
                                      int n) {
    bool cross = false;
    for (int e = 0; e < n; ++e) {
        const double4 r = ray[e];
        const bool inr = (r.y > py) != (r.x > py);
        const double L = py * r.z - px * r.w;
        const bool left = r.y > r.x ? (L > rhs[e]) : (L < rhs[e]);
        cross = cross != (inr && left);
    }
    return cross && isfinite(px) && isfinite(py);
}

// ----------------------------------------------------------------------------
// Per-polygon table in global memory (batched and all-pairs work): written by
// a preparation kernel, read by the screening kernels.
// ----------------------------------------------------------------------------
static_assert(sizeof(PolyHdr) == 64, "PolyHdr is 64 bytes");

// Offsets of polygon k's rows in the coefficient and generator arrays,
// derived from the vertex offsets alone (no scan): n_k + 3 padded float4
// coefficients and n_k + 1 generators per polygon.
__device__ __forceinline__ int64_t coef_base(const int64_t* vtx_off, int64_t k) {
    return vtx_off[k] + 3 * k;
}
__device__ __forceinline__ int64_t gen_base(const int64_t* vtx_off, int64_t k) {
    return vtx_off[k] + k;
}

// ----------------------------------------------------------------------------
// The float32 screen of one chunk (kPPL points per lane) against n4 padded
// edges whose coefficients are in LDS (binary64 points).  Voronoi: Mx = max
// margin.  Sign of offset: Mx, Mn = max and min offsets (both extremes, so
// the orientation of the rows does not matter).  Classification against the band E:
// see prepare_polygon.  valid[j] false -> neither inside nor undecided.
// ----------------------------------------------------------------------------
template <int KIND>
__device__ __forceinline__ void screen_chunk(const float4* coef, int n4, float KQ, float KA, float KB,
                                             float KC, const float (&X)[kPPL],
                                             const float (&Y)[kPPL], const bool (&valid)[kPPL],
                                             uint64_t (&inm)[kPPL], uint64_t (&unc)[kPPL]) {
    float Mx[kPPL], Mn[kPPL];
#pragma unroll
    for (int j = 0; j < kPPL; ++j) {
        Mx[j] = -__builtin_huge_valf();
        Mn[j] = __builtin_huge_valf();
    }
    for (int e = 0; e < n4; e += 4) {
        const float4 c0 = coef[e + 0], c1 = coef[e + 1];
        const float4 c2 = coef[e + 2], c3 = coef[e + 3];
#pragma unroll
        for (int j = 0; j < kPPL; ++j) {
            const float m0 = fmaf(c0.x, X[j], fmaf(c0.y, Y[j], c0.z));
            const float m1 = fmaf(c1.x, X[j], fmaf(c1.y, Y[j], c1.z));
            const float m2 = fmaf(c2.x, X[j], fmaf(c2.y, Y[j], c2.z));
            const float m3 = fmaf(c3.x, X[j], fmaf(c3.y, Y[j], c3.z));
            Mx[j] = fmaxf(fmaxf(Mx[j], m0), m1);  // v_max3_f32
            Mx[j] = fmaxf(fmaxf(Mx[j], m2), m3);
            if constexpr (KIND == K_SOO) {
                Mn[j] = fminf(fminf(Mn[j], m0), m1);  // v_min3_f32
                Mn[j] = fminf(fminf(Mn[j], m2), m3);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kPPL; ++j) {
        const float ax = fabsf(X[j]), ay = fabsf(Y[j]);
        const float r2 = fmaf(X[j], X[j], Y[j] * Y[j]);
        const float E = fmaf(KQ, r2, fmaf(KA, ax, fmaf(KB, ay, KC)));
        bool ins, outs;
        if constexpr (KIND == K_SOO) {
            ins = (Mx[j] < -E) || (Mn[j] > E);
            outs = (Mx[j] > E) && (Mn[j] < -E);
        } else {
            ins = Mx[j] < -E;
            outs = Mx[j] > E;
        }
        inm[j] = __ballot(valid[j] && ins);
        unc[j] = __ballot(valid[j] && !ins && !outs);
    }
}

// Lane k (k < 8) stores label word k of a chunk whose first word is `wbase`
// (nwords words exist from wbase on).  The masks are wave-uniform; a select
// tree on the lane's bits picks the word (no per-lane array indexing).
__device__ __forceinline__ void store_chunk_words(uint32_t* labels, int64_t wbase, int64_t nwords,
                                                  int lane, const uint64_t (&mask)[kPPL]) {
    const uint32_t lo0 = (uint32_t)mask[0], hi0 = (uint32_t)(mask[0] >> 32);
    const uint32_t lo1 = (uint32_t)mask[1], hi1 = (uint32_t)(mask[1] >> 32);
    const uint32_t lo2 = (uint32_t)mask[2], hi2 = (uint32_t)(mask[2] >> 32);
    const uint32_t lo3 = (uint32_t)mask[3], hi3 = (uint32_t)(mask[3] >> 32);
    const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4;
    const uint32_t w0 = b0 ? hi0 : lo0, w1 = b0 ? hi1 : lo1;
    const uint32_t w2 = b0 ? hi2 : lo2, w3 = b0 ? hi3 : lo3;
    const uint32_t w01 = b1 ? w1 : w0, w23 = b1 ? w3 : w2;
    const uint32_t w = b2 ? w23 : w01;
    if (lane < kWordsPerChunk && lane < nwords) labels[wbase + lane] = w;
}

// Wait for every outstanding memory operation of this wave (its label
// stores are then acknowledged by the L2 of its XCD, where the
// workgroup-scope atomics that patch them are performed).  Cheaper than an
// agent-scope fence, which writes back and invalidates the XCD's whole L2.
__device__ __forceinline__ void wave_drain() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void or_label_bit(uint32_t* labels, int64_t word, uint32_t bit) {
    __hip_atomic_fetch_or(&labels[word], 1u << bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

}  // namespace pipdev
