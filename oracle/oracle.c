/*
 * FP64 CPU oracle for the Voronoi point-inclusion test for convex polygons
 * (R. S. Zengin, V. Sezer, "A Novel Point Inclusion Test for Convex Polygons
 * Based on Voronoi Tessellations", arXiv:2007.15385).
 *
 * TEST INFRASTRUCTURE ONLY.  The test-suite, the package smoke check and the
 * CPU-baseline leg of the benchmark are the only callers.  The GPU library
 * never links, loads or calls this file, and this file includes nothing of
 * the GPU library: the two share no code, header, table or constant.
 *
 * Every routine is a plain loop over points in IEEE binary64, evaluated
 * exactly in the order written (build with -O2 -ffp-contract=off and without
 * -ffast-math, so no multiply-add is fused and nothing is reassociated).
 * OpenMP splits the loop over points (or poses); each result depends on one
 * point only, so the thread count never changes a result.
 *
 * Naming follows the paper's algorithms: V are the polygon vertices
 * v_1..v_n (here 0-based, row-major [n][2] = x,y), V' is V rolled by one
 * (V'_i = v_{i-1}, so edge i runs from v_{i-1} to v_i), Q are the query
 * points ([m][2]) and P the generators: P[0] = p_0 (the centroid), P[1+i] =
 * the outer generator of edge i.
 *
 * Readings taken where the paper is silent or garbled:
 *  - ray crossing: an odd number of crossings means inside (the prose of
 *    Section 2.1); the printed final line of Algorithm 1 compares the parity
 *    with zero, which would invert every label;
 *  - each test keeps its own boundary convention: Voronoi is closed (<= in
 *    Eq. 1), sign of offset uses the strict < of Algorithm 2, ray crossing is
 *    half-open through its strict > comparisons;
 *  - the inner generator is the centroid of Eq. 4 (Section 3), never another
 *    interior point;
 *  - the weight contraction of Algorithm 4 is W_k p_0 per edge (the printed
 *    index 0 of p is the centroid column);
 *  - a query point with an infinite or NaN coordinate is outside in all
 *    three tests (the paper's arithmetic is not defined there: inf <= inf
 *    would otherwise admit a point at infinity).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

static int64_t prev_index(int64_t i, int64_t n) { return i == 0 ? n - 1 : i - 1; }

/*
 * Centroid and signed area, Section 3, Eq. 3-4 and Algorithm 3.
 * Partial areas A_i = V'_x,i * V_y,i - V_x,i * V'_y,i; a = (1/2) sum A_i;
 * mu = ((V + V') A) / (6 a).  Sums run from i = 0 upwards.
 * Returns 0, or -1 when the area is zero or not finite.
 */
int oracle_centroid(const double *V, int64_t n, double *g0, double *area)
{
    double S = 0.0, Sx = 0.0, Sy = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t j = prev_index(i, n);
        double vx = V[2 * i], vy = V[2 * i + 1];
        double wx = V[2 * j], wy = V[2 * j + 1]; /* V'_i = v_{i-1} */
        double Ai = wx * vy - vx * wy;
        S = S + Ai;
        Sx = Sx + (vx + wx) * Ai;
        Sy = Sy + (vy + wy) * Ai;
    }
    double a = 0.5 * S;
    if (area) *area = a;
    g0[0] = Sx / (6.0 * a);
    g0[1] = Sy / (6.0 * a);
    if (!(a != 0.0) || !isfinite(a) || !isfinite(g0[0]) || !isfinite(g0[1])) return -1;
    return 0;
}

/*
 * Generators, Section 3, Eq. 5-8 and Algorithm 4.
 * For edge i (from v_{i-1} to v_i): a = V_y - V'_y, b = V'_x - V_x,
 * c = -(a V_x + b V_y); W = [[b^2 - a^2, -2ab], [-2ab, a^2 - b^2]];
 * d = W p_0; e = -2c [a; b]; p_i = (d + e) / (a^2 + b^2), which is p_0
 * reflected across the line through the edge (Eq. 6 gives the foot of the
 * perpendicular x, Eq. 7 sets p_i = 2x - p_0).
 * P receives (n+1) points: P[0] = p_0, P[1+i] = p_i.
 * Returns 0, -1 for a zero or non-finite area, -2 for a zero-length edge.
 */
int oracle_generators(const double *V, int64_t n, double *P)
{
    double g0[2];
    int rc = oracle_centroid(V, n, g0, NULL);
    P[0] = g0[0];
    P[1] = g0[1];
    for (int64_t i = 0; i < n; ++i) {
        int64_t j = prev_index(i, n);
        double vx = V[2 * i], vy = V[2 * i + 1];
        double wx = V[2 * j], wy = V[2 * j + 1];
        double a = vy - wy;
        double b = wx - vx;
        double c = -(a * vx + b * vy);
        double w11 = b * b - a * a;
        double w12 = (-2.0 * a) * b;
        double w22 = a * a - b * b;
        double dx = w11 * g0[0] + w12 * g0[1];
        double dy = w12 * g0[0] + w22 * g0[1];
        double ex = (-2.0 * c) * a;
        double ey = (-2.0 * c) * b;
        double den = a * a + b * b;
        P[2 * (i + 1)] = (dx + ex) / den;
        P[2 * (i + 1) + 1] = (dy + ey) / den;
        if (rc == 0 && den == 0.0) rc = -2;
    }
    return rc;
}

/* Squared Euclidean distance as Algorithm 5 forms it: Delta, then sum of
 * squares (Eq. 10-11: the square root of Eq. 9 is dropped). */
static double sqdist(double px, double py, double gx, double gy)
{
    double dx = px - gx;
    double dy = py - gy;
    return dx * dx + dy * dy;
}

/*
 * Voronoi inclusion, Section 4, Eq. 1 and Algorithm 5:
 * inside iff M_0 <= M_i for every outer generator i (closed polygon).
 * A NaN anywhere makes a comparison false, so the point is outside.
 * isin[k] = 1 inside, 0 outside.  Returns the generator status.
 */
int oracle_voronoi(const double *V, int64_t n, const double *Q, int64_t m, uint8_t *isin)
{
    double *P = (double *)malloc(sizeof(double) * 2 * (size_t)(n + 1));
    if (!P) return -100;
    int rc = oracle_generators(V, n, P);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < m; ++k) {
        double px = Q[2 * k], py = Q[2 * k + 1];
        double M0 = sqdist(px, py, P[0], P[1]);
        int in = isfinite(px) && isfinite(py);
        for (int64_t i = 0; i < n; ++i) {
            double Mi = sqdist(px, py, P[2 * (i + 1)], P[2 * (i + 1) + 1]);
            if (!(M0 <= Mi)) in = 0;
        }
        isin[k] = (uint8_t)in;
    }
    free(P);
    return rc;
}

/*
 * Non-convex polygons as a union of convex pieces (Section 7 names the
 * extension; the test itself, Section 4, needs a convex polygon).  The
 * polygon's vertices V ([n][2]) are split into K convex pieces whose
 * vertices are vertices of V: piece k is V[idx[j]] for j in
 * [off[k], off[k+1]), in cyclic order.  Every piece gets its own generators
 * (Algorithms 3-4) and isin[q] = 1 iff the closed Voronoi test (Algorithm 5)
 * of at least one piece puts point q inside.  A piece of fewer than 3
 * vertices contains no point.  Returns 0, the first nonzero generator status
 * of a piece, or -3 when a vertex index lies outside [0, n).
 */
int oracle_voronoi_pieces(const double *V, int64_t n, const int64_t *off, int64_t K,
                          const int64_t *idx, const double *Q, int64_t m, uint8_t *isin)
{
    int64_t total = off[K];
    for (int64_t j = 0; j < total; ++j)
        if (idx[j] < 0 || idx[j] >= n) return -3;
    double *G = (double *)malloc(sizeof(double) * 2 * (size_t)(total + K + 1));
    double *W = (double *)malloc(sizeof(double) * 2 * (size_t)(total + 1));
    if (!G || !W) {
        free(G);
        free(W);
        return -100;
    }
    int rc = 0;
    for (int64_t k = 0; k < K; ++k) {
        int64_t nk = off[k + 1] - off[k];
        if (nk < 3) continue;
        for (int64_t j = 0; j < nk; ++j) {
            W[2 * j] = V[2 * idx[off[k] + j]];
            W[2 * j + 1] = V[2 * idx[off[k] + j] + 1];
        }
        int r = oracle_generators(W, nk, G + 2 * (off[k] + k));
        if (rc == 0) rc = r;
    }
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < m; ++q) {
        double px = Q[2 * q], py = Q[2 * q + 1];
        int in = 0;
        if (isfinite(px) && isfinite(py)) {
            for (int64_t k = 0; k < K && !in; ++k) {
                int64_t nk = off[k + 1] - off[k];
                if (nk < 3) continue;
                const double *Pk = G + 2 * (off[k] + k);
                double M0 = sqdist(px, py, Pk[0], Pk[1]);
                int all = 1;
                for (int64_t i = 0; i < nk; ++i) {
                    double Mi = sqdist(px, py, Pk[2 * (i + 1)], Pk[2 * (i + 1) + 1]);
                    if (!(M0 <= Mi)) all = 0;
                }
                if (all) in = 1;
            }
        }
        isin[q] = (uint8_t)in;
    }
    free(G);
    free(W);
    return rc;
}

/*
 * Coverage raster (the graphics use of Section 1: every pixel's membership
 * decided by a point inclusion test).  Pixel (i, j) of a width x height grid
 * stands for the point (x0 + i*dx, y0 + j*dy), each coordinate one binary64
 * product and one binary64 sum; isin[j*width + i] is that point's Voronoi
 * label (Algorithm 5), row by row.
 */
int oracle_voronoi_raster(const double *V, int64_t n, double x0, double y0, double dx, double dy,
                          int64_t width, int64_t height, uint8_t *isin)
{
    double *P = (double *)malloc(sizeof(double) * 2 * (size_t)(n + 1));
    if (!P) return -100;
    int rc = oracle_generators(V, n, P);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < height; ++j) {
        double py = y0 + (double)j * dy;
        for (int64_t i = 0; i < width; ++i) {
            double px = x0 + (double)i * dx;
            double M0 = sqdist(px, py, P[0], P[1]);
            int in = isfinite(px) && isfinite(py);
            for (int64_t e = 0; e < n; ++e) {
                double Me = sqdist(px, py, P[2 * (e + 1)], P[2 * (e + 1) + 1]);
                if (!(M0 <= Me)) in = 0;
            }
            isin[j * width + i] = (uint8_t)in;
        }
    }
    free(P);
    return rc;
}

/*
 * Point location in a stored set of polygons (the GIS use of Section 1, with
 * the generators of constant polygons derived once and kept beside the
 * vertices, Section 7).  Polygon k has vertices V[vtx_off[k] .. vtx_off[k+1]);
 * ids[j] is the smallest k whose Voronoi test (Algorithm 5) puts point j
 * inside, or -1.  Polygons with fewer than 3 vertices contain no point.
 */
int oracle_locate(const int64_t *vtx_off, int64_t P, const double *V, const double *Q, int64_t m,
                  int32_t *ids)
{
    int64_t total = vtx_off[P];
    double *G = (double *)malloc(sizeof(double) * 2 * (size_t)(total + P + 1));
    if (!G) return -100;
    for (int64_t k = 0; k < P; ++k) {
        int64_t n = vtx_off[k + 1] - vtx_off[k];
        if (n >= 3) oracle_generators(V + 2 * vtx_off[k], n, G + 2 * (vtx_off[k] + k));
    }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < m; ++j) {
        double px = Q[2 * j], py = Q[2 * j + 1];
        int32_t id = -1;
        for (int64_t k = 0; k < P && id < 0; ++k) {
            int64_t n = vtx_off[k + 1] - vtx_off[k];
            if (n < 3) continue;
            const double *Pk = G + 2 * (vtx_off[k] + k);
            double M0 = sqdist(px, py, Pk[0], Pk[1]);
            int in = isfinite(px) && isfinite(py);
            for (int64_t i = 0; i < n; ++i) {
                double Mi = sqdist(px, py, Pk[2 * (i + 1)], Pk[2 * (i + 1) + 1]);
                if (!(M0 <= Mi)) in = 0;
            }
            if (in) id = (int32_t)k;
        }
        ids[j] = id;
    }
    free(G);
    return 0;
}

/*
 * Largest Voronoi margin per point: max_i (|p - p_0|^2 - |p - p_i|^2), the
 * quantity whose sign Algorithm 5 tests (Eq. 11 rearranged); <= 0 inside.
 * Each difference is formed from the two squared distances of Algorithm 5.
 */
void oracle_voronoi_max_margin(const double *V, int64_t n, const double *Q, int64_t m,
                               double *out)
{
    double *P = (double *)malloc(sizeof(double) * 2 * (size_t)(n + 1));
    if (!P) return;
    oracle_generators(V, n, P);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < m; ++k) {
        double px = Q[2 * k], py = Q[2 * k + 1];
        double M0 = sqdist(px, py, P[0], P[1]);
        double best = -INFINITY;
        for (int64_t i = 0; i < n; ++i) {
            double Mi = sqdist(px, py, P[2 * (i + 1)], P[2 * (i + 1) + 1]);
            double mi = M0 - Mi;
            if (mi > best || i == 0) best = mi;
        }
        out[k] = best;
    }
    free(P);
}

/*
 * Sign of offset, Section 2.2 and Algorithm 2.
 * Delta V = V - V'; LHS = Q_y dV_x - Q_x dV_y; RHS = V'_y dV_x - V'_x dV_y;
 * D_i = LHS < RHS; inside iff (sum_i D_i) mod n == 0, i.e. every edge gives
 * the same answer (so either orientation is accepted).
 */
void oracle_sign_of_offset(const double *V, int64_t n, const double *Q, int64_t m, uint8_t *isin)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < m; ++k) {
        double px = Q[2 * k], py = Q[2 * k + 1];
        int64_t count = 0;
        for (int64_t i = 0; i < n; ++i) {
            int64_t j = prev_index(i, n);
            double dVx = V[2 * i] - V[2 * j];
            double dVy = V[2 * i + 1] - V[2 * j + 1];
            double LHS = py * dVx - px * dVy;
            double RHS = V[2 * j + 1] * dVx - V[2 * j] * dVy;
            if (LHS < RHS) count += 1;
        }
        isin[k] = (uint8_t)(((count % n) == 0) && isfinite(px) && isfinite(py));
    }
}

/*
 * Ray crossing, Section 2.1 and Algorithm 1, with a ray towards +x.
 * InRange = (V_y > Q_y) xor (V'_y > Q_y); GoingUp = V_y > V'_y;
 * LHS, RHS as in the sign-of-offset test; OnLeft = GoingUp ? LHS > RHS :
 * LHS < RHS; an edge is crossed when InRange and OnLeft; inside iff the
 * number of crossings is odd (the prose reading).
 */
void oracle_ray_crossing(const double *V, int64_t n, const double *Q, int64_t m, uint8_t *isin)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < m; ++k) {
        double px = Q[2 * k], py = Q[2 * k + 1];
        int64_t crossings = 0;
        for (int64_t i = 0; i < n; ++i) {
            int64_t j = prev_index(i, n);
            int in_range = (V[2 * i + 1] > py) != (V[2 * j + 1] > py);
            int going_up = V[2 * i + 1] > V[2 * j + 1];
            double dVx = V[2 * i] - V[2 * j];
            double dVy = V[2 * i + 1] - V[2 * j + 1];
            double LHS = py * dVx - px * dVy;
            double RHS = V[2 * j + 1] * dVx - V[2 * j] * dVy;
            int on_left = going_up ? (LHS > RHS) : (LHS < RHS);
            if (in_range && on_left) crossings += 1;
        }
        isin[k] = (uint8_t)(((crossings % 2) == 1) && isfinite(px) && isfinite(py));
    }
}

/*
 * World-frame vertices of a footprint F (body frame, [n][2]) placed at pose
 * (tx, ty) with heading given by (c, s) = (cos theta, sin theta):
 * w = R(theta) v + t, evaluated as ((c vx - s vy) + tx, (s vx + c vy) + ty).
 * This is the rigid placement of the car polygon of Section 1.
 */
void oracle_pose_polygon(const double *F, int64_t n, double tx, double ty, double c, double s,
                         double *W)
{
    for (int64_t i = 0; i < n; ++i) {
        double vx = F[2 * i], vy = F[2 * i + 1];
        W[2 * i] = (c * vx - s * vy) + tx;
        W[2 * i + 1] = (s * vx + c * vy) + ty;
    }
}

/*
 * All poses against one point cloud (the collision check of Section 1).
 * poses are (tx, ty) pairs [K][2] with (cos, sin) pairs cs [K][2]; for each
 * pose the footprint is placed, converted to generators (Algorithms 3-4) and
 * every point is tested with Algorithm 5.  bits receives K rows of
 * ceil(m/32) little-endian 32-bit words (bit k%32 of word k/32 = point k),
 * counts the number of inside points per pose.
 */
void oracle_allpairs(const double *F, int64_t n, const double *poses, const double *cs, int64_t K,
                     const double *Q, int64_t m, uint32_t *bits, int64_t *counts)
{
    int64_t words = (m + 31) / 32;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < K; ++k) {
        double *W = (double *)malloc(sizeof(double) * 2 * (size_t)n);
        double *P = (double *)malloc(sizeof(double) * 2 * (size_t)(n + 1));
        oracle_pose_polygon(F, n, poses[2 * k], poses[2 * k + 1], cs[2 * k], cs[2 * k + 1], W);
        oracle_generators(W, n, P);
        uint32_t *row = bits + k * words;
        memset(row, 0, sizeof(uint32_t) * (size_t)words);
        int64_t cnt = 0;
        for (int64_t j = 0; j < m; ++j) {
            double px = Q[2 * j], py = Q[2 * j + 1];
            double M0 = sqdist(px, py, P[0], P[1]);
            int in = isfinite(px) && isfinite(py);
            for (int64_t i = 0; i < n; ++i) {
                double Mi = sqdist(px, py, P[2 * (i + 1)], P[2 * (i + 1) + 1]);
                if (!(M0 <= Mi)) in = 0;
            }
            if (in) {
                row[j >> 5] |= (uint32_t)1u << (j & 31);
                cnt += 1;
            }
        }
        counts[k] = cnt;
        free(W);
        free(P);
    }
}

/*
 * Normalized Voronoi margin of point p for edge i: the margin
 * m_i = |p - p_0|^2 - |p - p_i|^2 (Eq. 11) divided by -2|p_i - p_0|.  Since
 * p_i is p_0 mirrored across edge line i, |p_i - p_0| is twice the distance
 * from p_0 to that line and this is the signed distance from p to line i,
 * positive on the side of p_0.
 */
static double normalized_margin(double px, double py, const double *P, int64_t i)
{
    double M0 = sqdist(px, py, P[0], P[1]);
    double Mi = sqdist(px, py, P[2 * (i + 1)], P[2 * (i + 1) + 1]);
    double hx = P[2 * (i + 1)] - P[0];
    double hy = P[2 * (i + 1) + 1] - P[1];
    double len = sqrt(hx * hx + hy * hy);
    return -(M0 - Mi) / (2.0 * len);
}

/*
 * Collision cost of one pose: the point cloud is moved into the body frame,
 * p_b = R(theta)^T (p - t) evaluated as dx = px - tx, dy = py - ty,
 * (c dx + s dy, (-s) dx + c dy); the cost is the sum over points of
 * relu(min_i d_i(p_b)), the penetration depth of each point into the
 * footprint.  P are the generators of the body-frame footprint.
 * state (optional, [m]) receives -1 for a point that contributes nothing and
 * otherwise the index of the edge attaining the minimum (lowest index on a
 * tie).
 */
static double cost_one_pose(const double *P, int64_t n, double tx, double ty, double c, double s,
                            const double *Q, int64_t m, int32_t *state)
{
    double total = 0.0;
    for (int64_t j = 0; j < m; ++j) {
        double dx = Q[2 * j] - tx;
        double dy = Q[2 * j + 1] - ty;
        double bx = c * dx + s * dy;
        double by = (-s) * dx + c * dy;
        double best = 0.0;
        int64_t arg = 0;
        for (int64_t i = 0; i < n; ++i) {
            double d = normalized_margin(bx, by, P, i);
            if (i == 0 || d < best) {
                best = d;
                arg = i;
            }
        }
        if (best > 0.0) {
            total += best;
            if (state) state[j] = (int32_t)arg;
        } else if (state) {
            state[j] = -1;
        }
    }
    return total;
}

/*
 * Costs of K poses (x, y, theta) [K][3] of footprint F [n][2] (body frame)
 * against points Q [m][2].  cos/sin of theta come from libm.
 */
int oracle_cost(const double *F, int64_t n, const double *poses, int64_t K, const double *Q,
                int64_t m, double *cost)
{
    double *P = (double *)malloc(sizeof(double) * 2 * (size_t)(n + 1));
    if (!P) return -100;
    int rc = oracle_generators(F, n, P);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < K; ++k) {
        double th = poses[3 * k + 2];
        cost[k] = cost_one_pose(P, n, poses[3 * k], poses[3 * k + 1], cos(th), sin(th), Q, m, NULL);
    }
    free(P);
    return rc;
}

/* Per-point (active?, argmin) state of one pose, for finite-difference kink
 * detection. */
int oracle_cost_state(const double *F, int64_t n, const double *pose, const double *Q, int64_t m,
                      int32_t *state)
{
    double *P = (double *)malloc(sizeof(double) * 2 * (size_t)(n + 1));
    if (!P) return -100;
    int rc = oracle_generators(F, n, P);
    double th = pose[2];
    cost_one_pose(P, n, pose[0], pose[1], cos(th), sin(th), Q, m, state);
    free(P);
    return rc;
}

/*
 * Reference gradient of sum_k w_k C_k, by closed form rather than through
 * the generator construction.  For a contributing point with minimising edge
 * i (segment a = v_{i-1} -> b = v_i, e = b - a, L = |e|, sigma = sign of the
 * polygon's area), the signed distance is d = sigma cross(e, p_b - a) / L.
 * Its gradients are
 *   dd/dp_b = sigma (-e_y, e_x) / L,
 *   dd/db   = sigma ((r_y, -r_x) / L - f e / L^3),
 *   dd/da   = sigma ((e_y - r_y, r_x - e_x) / L + f e / L^3),
 * with r = p_b - a and f = cross(e, r).  Through p_b = R^T (p - t):
 *   dC/dt = -R dd/dp_b,   dC/dtheta = dd/dp_b . (p_b,y, -p_b,x).
 * grad_pose [K][3] and grad_F [n][2] are overwritten.  abs_pose and abs_F
 * (optional, same shapes) receive the sums of the magnitudes of the
 * per-point contributions, the scale against which a float result is judged.
 */
int oracle_cost_grad(const double *F, int64_t n, const double *poses, int64_t K, const double *Q,
                     int64_t m, const double *w, double *grad_pose, double *grad_F,
                     double *abs_pose, double *abs_F)
{
    double *P = (double *)malloc(sizeof(double) * 2 * (size_t)(n + 1));
    if (!P) return -100;
    int rc = oracle_generators(F, n, P);
    double area = 0.0, g0[2];
    oracle_centroid(F, n, g0, &area);
    double sigma = area > 0.0 ? 1.0 : -1.0;
    /* per-pose footprint gradients, summed over poses in index order so
     * that the result does not depend on the thread count */
    double *gF_pose = (double *)calloc((size_t)K * 2 * (size_t)n, sizeof(double));
    double *aF_pose = (double *)calloc((size_t)K * 2 * (size_t)n, sizeof(double));
    if (!gF_pose || !aF_pose) {
        free(gF_pose);
        free(aF_pose);
        free(P);
        return -100;
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < K; ++k) {
        double *gF = gF_pose + (size_t)k * 2 * (size_t)n;
        double *aF = aF_pose + (size_t)k * 2 * (size_t)n;
        double tx = poses[3 * k], ty = poses[3 * k + 1], th = poses[3 * k + 2];
        double c = cos(th), s = sin(th);
        double gtx = 0.0, gty = 0.0, gth = 0.0;
        double atx = 0.0, aty = 0.0, ath = 0.0;
        for (int64_t j = 0; j < m; ++j) {
            double dx = Q[2 * j] - tx;
            double dy = Q[2 * j + 1] - ty;
            double bx = c * dx + s * dy;
            double by = (-s) * dx + c * dy;
            double best = 0.0;
            int64_t arg = 0;
            for (int64_t i = 0; i < n; ++i) {
                double d = normalized_margin(bx, by, P, i);
                if (i == 0 || d < best) {
                    best = d;
                    arg = i;
                }
            }
            if (!(best > 0.0)) continue;
            int64_t ib = arg, ia = prev_index(arg, n);
            double ax = F[2 * ia], ay = F[2 * ia + 1];
            double ex = F[2 * ib] - ax, ey = F[2 * ib + 1] - ay;
            double L = sqrt(ex * ex + ey * ey);
            double rx = bx - ax, ry = by - ay;
            double f = ex * ry - ey * rx;
            double gpx = sigma * (-ey) / L, gpy = sigma * ex / L;
            double ctx_ = -(c * gpx - s * gpy);
            double cty = -(s * gpx + c * gpy);
            double cth = gpx * by + gpy * (-bx);
            gtx += ctx_;
            gty += cty;
            gth += cth;
            atx += fabs(ctx_);
            aty += fabs(cty);
            ath += fabs(cth);
            double L3 = L * L * L;
            double cbx = sigma * (ry / L - f * ex / L3);
            double cby = sigma * (-rx / L - f * ey / L3);
            double cax = sigma * ((ey - ry) / L + f * ex / L3);
            double cay = sigma * ((rx - ex) / L + f * ey / L3);
            gF[2 * ib] += cbx;
            gF[2 * ib + 1] += cby;
            gF[2 * ia] += cax;
            gF[2 * ia + 1] += cay;
            aF[2 * ib] += fabs(cbx);
            aF[2 * ib + 1] += fabs(cby);
            aF[2 * ia] += fabs(cax);
            aF[2 * ia + 1] += fabs(cay);
        }
        grad_pose[3 * k] = w[k] * gtx;
        grad_pose[3 * k + 1] = w[k] * gty;
        grad_pose[3 * k + 2] = w[k] * gth;
        if (abs_pose) {
            abs_pose[3 * k] = fabs(w[k]) * atx;
            abs_pose[3 * k + 1] = fabs(w[k]) * aty;
            abs_pose[3 * k + 2] = fabs(w[k]) * ath;
        }
    }
    for (int64_t i = 0; i < 2 * n; ++i) {
        grad_F[i] = 0.0;
        if (abs_F) abs_F[i] = 0.0;
    }
    for (int64_t k = 0; k < K; ++k)
        for (int64_t i = 0; i < 2 * n; ++i) {
            grad_F[i] += w[k] * gF_pose[(size_t)k * 2 * (size_t)n + (size_t)i];
            if (abs_F) abs_F[i] += fabs(w[k]) * aF_pose[(size_t)k * 2 * (size_t)n + (size_t)i];
        }
    free(gF_pose);
    free(aF_pose);
    free(P);
    return rc;
}

/*
 * Costs of K poses plus, per pose, a 64-bit hash of every point's
 * (contributes?, minimising edge) state, so that finite differences can tell
 * whether a perturbation crossed a relu or min kink for any point.
 */
int oracle_cost_with_hash(const double *F, int64_t n, const double *poses, int64_t K,
                          const double *Q, int64_t m, double *cost, uint64_t *hash)
{
    double *P = (double *)malloc(sizeof(double) * 2 * (size_t)(n + 1));
    if (!P) return -100;
    int rc = oracle_generators(F, n, P);
#pragma omp parallel
    {
        int32_t *st = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
#pragma omp for schedule(dynamic, 1)
        for (int64_t k = 0; k < K; ++k) {
            double th = poses[3 * k + 2];
            cost[k] = cost_one_pose(P, n, poses[3 * k], poses[3 * k + 1], cos(th), sin(th), Q, m, st);
            uint64_t h = 1469598103934665603ull;
            for (int64_t j = 0; j < m; ++j) {
                h ^= (uint64_t)(uint32_t)(st[j] + 2) * 0x9E3779B97F4A7C15ull + (uint64_t)j;
                h *= 1099511628211ull;
            }
            hash[k] = h;
        }
        free(st);
    }
    free(P);
    return rc;
}
