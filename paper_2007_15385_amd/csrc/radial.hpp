// Radial pre-screen of the single-polygon Voronoi kernel.
//
// In the Voronoi view of Section 4 (Eq. 1, 9-11) a point is inside when p_0
// is its nearest generator, and the affine margin m_i of edge i (the
// difference of squared distances to p_0 and p_i, rearranged as in Eq. 11)
// grows along the edge's outward normal.  So the label of a point close
// enough to p_0 is "inside" and that of a point far enough away in any
// direction is "outside", whatever the other edges do: the polygon lies
// between two radii around p_0.  This file turns that into thresholds on
// r2 = fl32(X^2 + Y^2) (local coordinates X, Y as in the float32 screen),
// one pair per octant of directions (the polygon's extent differs by
// direction), such that
//   r2 < T_in[o]              =>  every binary64 difference of Algorithm 5
//                                 is negative (label inside),
//   T_out[o] < r2 < T_far     =>  some binary64 difference is positive
//                                 (label outside).
// Only the points between the radii take the per-edge float32 screen (and,
// inside its band, the binary64 recheck), so every label still equals the
// binary64 result of Algorithm 5.
//
// Derivation.  Let D_i = fl64(M_0) - fl64(M_i) (Algorithm 5 decides inside
// iff every D_i <= 0), m_i = A_i X + B_i Y - C_i evaluated exactly with the
// float32 coefficients and m_hat_i = fma(A_i, X, fma(B_i, Y, -C_i)).  The
// band of the screen gives |m_hat_i - D_i| <= E(X, Y) = KQ (X^2 + Y^2) +
// KA |X| + KB |Y| + KC, and the two fma roundings give |m_hat_i - m_i| <=
// g (|A_i X| + |B_i Y| + |C_i|), g = 2 u (1 + u), u = 2^-24.  With rho =
// |(X, Y)|, a_i = |(A_i, B_i)| and KAB = |(KA, KB)| (Cauchy-Schwarz bounds
// |A_i X| + |B_i Y| <= a_i rho and KA |X| + KB |Y| <= KAB rho):
//   D_i <= a_i rho k_i + g (a_i rho + |C_i|) - C_i + KQ rho^2 + KAB rho + KC,
// where k_i is the largest cosine between edge i's normal (A_i, B_i) and a
// direction of the octant.  The right side is a convex quadratic in rho that
// is negative at 0 for a valid polygon, so it is negative on [0, rho_i); the
// inner radius of the octant is min_i rho_i.
// Outward: the normals of a convex polygon wind once around the circle, so
// a direction w lies in the arc between two consecutive normals n_i, n_j
// (angle d < pi) and is within d/2 of one of them, say n_k:
//   D_k >= a_k rho cos(d/2) - C_k - g (a_k rho + |C_k|) - KQ rho^2 - KAB rho - KC,
// a concave quadratic in rho, positive on (r1, r2).  The octant's outer
// interval is (max r1, min r2) over the arcs that meet the octant and both
// of their normals.
// The octant of a point comes from the sign bits of X and Y and |Y| > |X|:
// exact predicates on the float32 values, and the octants are closed arcs, so
// a point on a boundary is covered by either side's bound.  r2 lies within
// (1 +- u)^2 of X^2 + Y^2, so T_in is rho_in^2 (1 - 2^-20) rounded down,
// T_out is rho_out^2 (1 + 2^-20) rounded up and T_far the smallest
// rho_far^2 (1 - 2^-20) rounded down; the 2^-20 also covers the binary64
// rounding of this computation.  A polygon that is not valid and convex, or
// whose coefficients are out of range (KC = +inf), gets T_in = 0 and
// T_out = +inf: every point takes the per-edge screen.  A NaN or infinite
// coordinate gives r2 = NaN or +inf, which no threshold accepts.
#pragma once
#include "device.hpp"

namespace pipdev {

struct RadialTab {
    float2 t[8];        // octant o = 4 sign(X) + 2 sign(Y) + (|Y| > |X|): (T_in, T_out)
    uint64_t cand[8];   // edges a point of octant o with r2 <= T_out[o] can violate
    uint64_t all;       // every edge
    float tfar;
    int len4[9];        // list lengths rounded up to a multiple of 4
    uint8_t list[9][kMaxEdges];  // cand[o] (class o < 8) and every edge (class 8) as edge
                                 // indices, padded to 64 entries by repeating the first
};

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
    return v;
}

// Octant o as the closed arc from e0 to e1 (counter-clockwise, pi/4 wide).
__device__ __forceinline__ void octant_arc(int o, double2* e0, double2* e1) {
    const double s = 0.70710678118654752440;
    const int sx = o >> 2, sy = (o >> 1) & 1, sw = o & 1;
    // first quadrant image: sw = 0 -> [0, pi/4], sw = 1 -> [pi/4, pi/2]
    double2 a = sw ? make_double2(s, s) : make_double2(1.0, 0.0);
    double2 b = sw ? make_double2(0.0, 1.0) : make_double2(s, s);
    // mirror into the quadrant of (sx, sy); a mirror reverses orientation
    if (sx) { a.x = -a.x; b.x = -b.x; }
    if (sy) { a.y = -a.y; b.y = -b.y; }
    if (sx != sy) { const double2 t = a; a = b; b = t; }
    *e0 = a;
    *e1 = b;
}

__device__ __forceinline__ double cross2(double2 a, double2 b) { return a.x * b.y - a.y * b.x; }
__device__ __forceinline__ double dot2(double2 a, double2 b) { return a.x * b.x + a.y * b.y; }

// v in the closed arc from s to e (counter-clockwise, narrower than pi), with
// a tolerance that only ever widens the arc.
__device__ __forceinline__ bool in_arc(double2 v, double2 s, double2 e) {
    return cross2(s, v) >= -1e-12 && cross2(v, e) >= -1e-12;
}

// Candidate edges.  For a point of octant o with r2 <= T_out[o], |(X, Y)| <
// sqrt(T_out[o]) (1 + 2^-20) =: lim, so every edge whose inner radius rho_i
// over the octant exceeds lim has a negative binary64 difference (the bound
// above): only the others can decide the point.  The per-edge screen of such
// a point (and its binary64 recheck) runs over cand[o]; every other point
// (beyond T_out, NaN) over all edges.  A polygon with the screen off, or an
// octant without an outer bound, lists every edge.
//
// Called by one whole wave after prepare_polygon (S.coef, S.K*, S.status set).
// KC_band replaces the band's constant term where a kernel widens it (the
// raster, whose pixel coordinates carry one more rounding); negative: S.KC.
__device__ inline void prepare_radial(const PolyLds& S, int lane, RadialTab& R,
                                      float KC_band = -1.0f) {
    const int n = S.n;
    const bool act = lane < n;
    const int i = act ? lane : 0;
    const int j = i + 1 < n ? i + 1 : 0;
    const float4 ci = S.coef[i], cj = S.coef[j];  // (A, B, -C)
    const double KQ = S.KQ, KC = KC_band >= 0.0f ? KC_band : S.KC;
    const double KAB = sqrt((double)S.KA * (double)S.KA + (double)S.KB * (double)S.KB);
    const double g = 2.0 * kU32 * (1.0 + kU32);
    const double ai = sqrt((double)ci.x * ci.x + (double)ci.y * ci.y);
    const double aj = sqrt((double)cj.x * cj.x + (double)cj.y * cj.y);
    const double Ci = -(double)ci.z, Cj = -(double)cj.z;
    const double2 ni = make_double2(ci.x / ai, ci.y / ai);
    const double2 nj = make_double2(cj.x / aj, cj.y / aj);
    bool usable = S.status == ST_OK && isfinite(KC) && n >= 3;

    // winding of the normals: arcs from s to e (counter-clockwise) narrower
    // than pi, chained once around the circle.  A turn backwards by less than
    // 1e-6 (float32 rounding of the coefficients of nearly collinear edges)
    // counts as an empty arc: its neighbours overlap by that much, so the
    // circle stays covered.  The half-open arcs [s, e) that hold
    // the direction (1, 0) are counted with exact sign tests on the unit
    // normals' components (the normalisation keeps every sign and zero).
    const double cr = cross2(ni, nj), dt = dot2(ni, nj);
    const bool ccw = wave_sum(act ? cr : 0.0) > 0.0;
    const double2 s = ccw ? ni : nj, e = ccw ? nj : ni;
    const double cse = ccw ? cr : -cr;
    const bool arc_ok = !act || cse > 0.0 || (cse >= -1e-6 && dt > 0.0);
    const bool holds_x = act && (s.y < 0.0 || (s.y == 0.0 && s.x > 0.0)) && e.y > 0.0;
    const bool wind_ok = __popcll(__ballot(holds_x)) == 1;
    usable = usable && wind_ok && !__ballot(!arc_ok) && (ai > 0.0) && (aj > 0.0);
    usable = !__ballot(!usable);
    const double chalf = sqrt(fmax(0.0, 0.5 * (1.0 + dt))) - 1e-12;  // cos of half the arc

    // outward quadratics of the arc's two normals: KQ r^2 - b r + c1 < 0 on (r1, r2)
    double r1a = __builtin_inf(), r2a = 0.0;
    {
        const double a2[2] = {ai, aj}, C2[2] = {Ci, Cj};
        double lo = 0.0, hi = __builtin_inf();
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const double b = a2[k] * (chalf - g) - KAB;
            const double c1 = C2[k] + g * fabs(C2[k]) + KC + 1e-30;
            const double disc = b * b - 4.0 * KQ * c1;
            if (b > 0.0 && disc > 0.0) {
                const double D = sqrt(disc);
                lo = fmax(lo, 2.0 * c1 / (b + D));
                hi = fmin(hi, (b + D) / (2.0 * KQ));
            } else {
                lo = __builtin_inf();
                hi = 0.0;
            }
        }
        r1a = lo;
        r2a = hi;
    }

    const uint64_t all = __ballot(act);  // taken by the whole wave, not inside a lane-0 branch
    double far_all = __builtin_inf();
#pragma unroll 1
    for (int o = 0; o < 8; ++o) {
        double2 e0, e1;
        octant_arc(o, &e0, &e1);
        // inner radius of edge i over the octant
        const double k = (in_arc(ni, e0, e1) ? 1.0 : fmax(dot2(ni, e0), dot2(ni, e1))) + 1e-12;
        const double b = ai * (k + g) + KAB;
        const double c0 = KC - Ci + g * fabs(Ci) + 1e-30;
        double rho = 0.0;
        if (c0 < 0.0) {
            const double D = sqrt(b * b - 4.0 * KQ * c0);
            rho = b >= 0.0 ? -2.0 * c0 / (b + D) : (D - b) / (2.0 * KQ);
        }
        const double rin = wave_min(act ? rho : __builtin_inf());
        // outer interval over the arcs that meet the octant
        const bool meets = act && (in_arc(s, e0, e1) || in_arc(e, e0, e1) || in_arc(e0, s, e) ||
                                   in_arc(e1, s, e));
        const double rout = wave_max(meets ? r1a : 0.0);
        const double rfar = wave_min(meets ? r2a : __builtin_inf());
        far_all = fmin(far_all, rfar);
        const bool any_meet = __ballot(meets) != 0;  // always, when the arcs cover the circle
        const bool out_ok = usable && any_meet && rout < rfar;
        const float t_out = out_ok ? round_up_f32(rout * rout * (1.0 + 9.5367431640625e-07))
                                   : __builtin_huge_valf();
        const double lim = out_ok ? sqrt((double)t_out) * (1.0 + 9.5367431640625e-07)
                                  : __builtin_inf();
        const uint64_t cand = __ballot(act && !(rho > lim));
        if (lane == 0) {
            R.t[o] = make_float2(usable ? round_down_f32(rin * rin * (1.0 - 9.5367431640625e-07)) : 0.0f,
                                 t_out);
            R.cand[o] = usable ? cand : all;
        }
    }
    if (lane == 0) R.all = all;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // index lists: lane l writes its own position in each class's list; the
    // padding repeats the class's first edge (a repeated edge leaves both the
    // float32 maximum and the binary64 conjunction unchanged)
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
#pragma unroll 1
    for (int c = 0; c < 9; ++c) {
        const uint64_t mk = c < 8 ? R.cand[c] : all;
        const int cnt = __popcll(mk);
        const int first = mk ? __builtin_ctzll(mk) : 0;
        if ((mk >> lane) & 1ull) R.list[c][__popcll(mk & below)] = (uint8_t)lane;
        if (lane >= cnt) R.list[c][lane] = (uint8_t)first;
        if (lane == 0) R.len4[c] = cnt == 0 ? 4 : (cnt + 3) & ~3;
    }
    if (lane == 0)
        R.tfar = usable ? round_down_f32(far_all * far_all * (1.0 - 9.5367431640625e-07)) : 0.0f;
}

// Candidate class of a point from its local coordinates: its octant if
// r2 <= T_out there, else 8 (every edge).
__device__ __forceinline__ int radial_class(const RadialTab& R, float X, float Y) {
    const float r2 = fmaf(X, X, Y * Y);
    const int o = (int)(((__float_as_uint(X) >> 31) << 2) | ((__float_as_uint(Y) >> 31) << 1) |
                        (fabsf(Y) > fabsf(X) ? 1u : 0u));
    return r2 <= R.t[o].y ? o : 8;
}

// Algorithm 5 in binary64 over the first `len` entries of an index list
// (repeats allowed; the other edges are known to compare M_0 < M_i).  Same
// operations and order per edge as the full replay.
__device__ inline bool voronoi64_list(double px, double py, const double2* gen,
                                      const uint8_t* list, int len) {
    bool in = isfinite(px) && isfinite(py);
    const double dx0 = px - gen[0].x;
    const double dy0 = py - gen[0].y;
    const double M0 = dx0 * dx0 + dy0 * dy0;
    for (int t = 0; t < len; ++t) {
        const int i = list[t];
        const double dx = px - gen[1 + i].x;
        const double dy = py - gen[1 + i].y;
        const double Mi = dx * dx + dy * dy;
        if (!(M0 <= Mi)) in = false;
    }
    return in;
}

}  // namespace pipdev
