/*
 * pip_voronoi.h -- C ABI of the MI355X (gfx950) point-inclusion library.
 *
 * The library implements the point-in-convex-polygon test of R. S. Zengin and
 * V. Sezer, "A Novel Point Inclusion Test for Convex Polygons Based on
 * Voronoi Tessellations" (arXiv:2007.15385), and the two reference tests the
 * paper compares it with:
 *   - Voronoi inclusion (Section 4, Eq. 1 and 9-11, Algorithm 5): the polygon
 *     is converted once into an inner generator p_0 (its centroid, Section 3,
 *     Eq. 3-4, Algorithm 3) and one outer generator per edge (p_0 mirrored
 *     across the edge line, Section 3, Eq. 5-8, Algorithm 4); a point is
 *     inside iff it is no farther from p_0 than from every outer generator;
 *   - sign of offset (Section 2.2, Algorithm 2), convex polygons;
 *   - ray crossing (Section 2.1, Algorithm 1), any simple polygon.
 *
 * Entry points, by use:
 *   - one polygon against a point array: pip_voronoi, pip_sign_of_offset,
 *     pip_ray_crossing, pip_voronoi_fp32_plain (speed reference),
 *     pip_voronoi_max_margin, polygon_to_generators; against a pixel grid
 *     (Section 1's rasterisation): pip_voronoi_raster;
 *   - many polygons: pip_voronoi_batched and its plans (pip_plan_*), each
 *     polygon against its own points; pip_poses_to_polygons and
 *     pip_voronoi_allpairs, one footprint at many poses against one cloud;
 *     pip_index_* (Section 1's GIS use), the polygon containing each point;
 *   - the differentiable collision cost: pip_cost_fwd, pip_cost_bwd.
 *
 * Conventions shared by every entry point
 *   - Polygons: binary64 vertices v_0..v_{n-1}, interleaved x,y ([n][2]), in
 *     cyclic order, either orientation.  Edge i runs from v_{i-1} to v_i
 *     (v_{-1} = v_{n-1}), the paper's rolled vertex matrix.  3 <= n <= 64.
 *   - Query points: interleaved x,y ([m][2]) as float32 (PIP_F32, 8-byte
 *     aligned) or binary64 (PIP_F64, 16-byte aligned).
 *   - Labels: ceil(m/32) little-endian 32-bit words, 4-byte aligned; bit
 *     (k mod 32) of word floor(k/32) is point k, 1 = inside.  Bits past m are
 *     written as 0.  A point with a non-finite coordinate is outside.
 *   - Exactness: every label equals the result of the paper's algorithm
 *     evaluated in IEEE binary64 in the order written (no fused
 *     multiply-add), with float32 query points widened exactly.  The
 *     Voronoi test keeps the closed boundary of Eq. 1, sign of offset the
 *     strict comparison of Algorithm 2, ray crossing the half-open rule of
 *     Algorithm 1 with odd parity meaning inside.
 *   - Memory: every pointer argument is a DEVICE pointer unless stated; the
 *     caller allocates and owns all buffers; the library frees nothing it did
 *     not allocate.
 *   - Streams: every compute call only enqueues work on `stream` (a
 *     hipStream_t; NULL is the default stream) and returns; results are ready
 *     when the stream has reached that point.  Plan and index creation
 *     (pip_plan_create_batched, pip_plan_autotune, pip_index_create)
 *     allocate and synchronize.
 *   - Errors: argument errors are detected on the host before anything is
 *     enqueued and returned as a pip_status; pip_last_error() then holds a
 *     sentence naming the argument.  Data-dependent problems of a polygon
 *     (non-finite vertex, zero area, zero-length edge, non-convex input) are
 *     written as a pip_status value to the optional device `status` word; the
 *     labels are still those of the binary64 algorithm for that input.
 *   - Threads: a pip_ctx may be used from several host threads; calls that
 *     share no output buffer may run concurrently on different streams.
 */
#ifndef PIP_VORONOI_H
#define PIP_VORONOI_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PIP_OK = 0,
    PIP_EINVAL = 1,        /* bad argument (host check) or non-finite vertex (device) */
    PIP_EDEGENERATE = 2,   /* zero area or zero-length edge (device) */
    PIP_ENONCONVEX = 3,    /* turn directions of the vertices are mixed (device) */
    PIP_EHIP = 4,          /* a HIP runtime call failed; see pip_last_error() */
    PIP_ENOMEM = 5,        /* device allocation failed */
    PIP_EUNSUPPORTED = 6   /* valid request outside the compiled limits (n > 64) */
} pip_status;

typedef enum { PIP_F32 = 0, PIP_F64 = 1 } pip_dtype;

#define PIP_MAX_EDGES 64

typedef struct pip_ctx_s *pip_ctx;

/* Create a context bound to HIP device `hip_device` (made current for the
 * call).  *out receives the handle.  Returns PIP_EINVAL for a bad device
 * index, PIP_EHIP if the device cannot be queried. */
pip_status pip_create(int hip_device, pip_ctx *out);

/* Destroy a context created by pip_create (NULL is ignored).  Work already
 * enqueued is not waited for; callers synchronise their streams first. */
void pip_destroy(pip_ctx ctx);

/* Static English name of a status code. */
const char *pip_status_str(pip_status s);

/* Detail of the last error returned on this host thread (never NULL). */
const char *pip_last_error(pip_ctx ctx);

/* Library version as major*10000 + minor*100 + patch. */
int pip_version(void);

/* Point-location index over a stored set of convex polygons (Section 1's
 * GIS use; Section 7: the generators of constant polygons are derived once
 * and kept beside the vertices, about twice the storage).  Owns device
 * memory until pip_index_destroy. */
typedef struct pip_index_s *pip_index;

/* Tuning options of a context.  Labels never depend on them.
 *   PIP_OPT_MFMA_MIN_EDGES: pip_voronoi / pip_sign_of_offset on float32 points
 *     evaluate the margins of polygons with at least this many edges as dense
 *     products on the matrix cores (v_mfma_f32_32x32x2f32) and those with fewer
 *     with two vector fma per edge; 0 disables the matrix-core path.
 *     Default 25 (measured crossover of the two screens).
 *   PIP_OPT_ALLPAIRS_CULL: 1 lets pip_voronoi_allpairs skip every (polygon,
 *     64 x 8-point wave) pair whose bounding disk (centre p_0, radius the
 *     largest vertex distance, rounded up) misses the bounding box or the range of
 *     distances from the origin of the wave's points; their labels are 0 and
 *     add 0 to the counts, exactly the dense result (a convex polygon lies in
 *     that disk).  Default 0 (dense: every pair evaluated).  Not from the
 *     paper: a culling layer in front of its test.
 *   PIP_OPT_COST_CULL: 1 lets pip_cost_fwd / pip_cost_bwd skip (pose, wave of
 *     256 points) pairs whose footprint disk, widened by 2^-12 of the
 *     coordinate scale, misses the wave's points: every such term is exactly
 *     zero, so costs and gradients are bit-identical to the dense ones.
 *     Default 0.
 *   PIP_OPT_ALLPAIRS_PAIR: 1 lets pip_voronoi_allpairs evaluate a polygon
 *     with an even edge count that is centrally symmetric (up to u = 2^-24 of
 *     its coefficients) as n/2 antipodal edge pairs: edges i and i + n/2 have
 *     opposite generator offsets (Section 3, Eq. 8), so the larger of their two
 *     margins (Eq. 11) is |t| - h of one affine form t; the remaining
 *     asymmetry is bounded in the float32 band, so labels and counts are those
 *     of the dense evaluation.  Other polygons keep the per-edge table.
 *     Default 0.
 *   PIP_OPT_COST_PAIR: 1 lets pip_cost_fwd / pip_cost_bwd evaluate a
 *     centrally symmetric footprint (edge normals of i and i + n/2 cancel to
 *     2^-20) as n/2 pairs: the smaller of the two signed distances is
 *     h - |t| of one affine form, at edge i when t >= 0.  Costs and gradients
 *     change by float32 rounding only (they are tolerance-graded); other
 *     footprints keep the per-edge loop.  Default 0.
 *   PIP_OPT_RADIAL_MIN_EDGES: pip_voronoi on float32 points first compares
 *     each point's squared distance from p_0 (in the float32 local frame)
 *     with two thresholds per octant of directions, derived in binary64 from
 *     the generators and the screen's error band (pip_voronoi_radial_bounds):
 *     below the inner one every binary64 comparison of Algorithm 5 says
 *     inside, beyond the outer one (and short of a far limit) one of them says
 *     outside.  Only the points in between take the per-edge screen (and, in
 *     its band, the binary64 recheck), so labels are unchanged.  Used for
 *     polygons with at least this many edges (before the matrix-core path),
 *     likewise by pip_voronoi_raster (with its own band, and the per-edge
 *     screen for every 512-pixel segment that holds a pixel between the
 *     radii) and by pip_voronoi_batched and batched plans for every polygon
 *     of the batch that has this many edges (a plan or workspace takes the
 *     setting when it is created or launched); 0 disables it.  Default 0 (off:
 *     every point meets every edge, as in the paper's own comparison of the
 *     tests, Section 6.2).  Measured: from about 20 edges it is faster than
 *     the per-edge screen (fewer edges leave more points between the radii).
 *     Not from the paper: a screen in front of its test, from the
 *     nearest-generator reading of Section 4. */
/*   PIP_OPT_EARLY_EXIT: 1 lets the per-edge screen of pip_voronoi_raster stop
 *     a 512-pixel segment after every 8 edges once each of its pixels has a
 *     partial largest margin beyond its band (the paper's early break of
 *     Section 5, taken by a whole wave; a margin maximum only grows with more
 *     edges, so such a pixel is outside).  Labels are unchanged.  Default 0
 *     (every edge evaluated, as in the paper's comparison of Section 6.2).
 *     Streaming and batched launches do not take it: their 512-point chunks
 *     are spatially random, so all of a chunk's points are almost never
 *     outside. */
typedef enum {
    PIP_OPT_MFMA_MIN_EDGES = 1,
    PIP_OPT_ALLPAIRS_CULL = 2,
    PIP_OPT_COST_CULL = 3,
    PIP_OPT_ALLPAIRS_PAIR = 4,
    PIP_OPT_COST_PAIR = 5,
    PIP_OPT_RADIAL_MIN_EDGES = 6,
    PIP_OPT_EARLY_EXIT = 7
} pip_option;
pip_status pip_set_option(pip_ctx ctx, pip_option opt, int64_t value);
pip_status pip_get_option(pip_ctx ctx, pip_option opt, int64_t *value);

/*
 * Generators of one convex polygon (Section 3, Eq. 3-8, Algorithms 3-4).
 *   V       [n][2] binary64 vertices.
 *   P       [n+1][2] binary64 output: P[0] = p_0 (centroid, Eq. 4), P[1+i] =
 *           outer generator of edge i (p_0 mirrored across the line through
 *           v_{i-1} and v_i, Eq. 8).
 *   status  optional [1] int32: PIP_OK / PIP_EINVAL / PIP_EDEGENERATE /
 *           PIP_ENONCONVEX for this polygon.
 * Bit-identical to the plain binary64 evaluation of Algorithms 3-4.
 */
pip_status polygon_to_generators(pip_ctx ctx, const double *V, int32_t n, double *P,
                                 int32_t *status, hipStream_t stream);

/*
 * Thresholds of the radial pre-screen of pip_voronoi (Section 4, Eq. 1 and
 * 9-11 read as a nearest-generator test), for tests and diagnostics.
 *   V    [n][2] binary64 vertices, 3 <= n <= PIP_MAX_EDGES.
 *   out  [17] float32 (device): out[o] = T_in and out[8 + o] = T_out of octant
 *        o = 4 s(X) + 2 s(Y) + (|Y| > |X|) (s = sign bit), out[16] = T_far,
 *        where X, Y are a point's float32 local coordinates (point minus
 *        fl32(p_0)) and r2 = fl32(X^2 + Y^2): r2 < T_in means the label is
 *        inside, T_out < r2 < T_far that it is outside.  A polygon that is not
 *        valid and convex gets T_in = 0, T_out = +inf.
 * Asynchronous on `stream`; allocates nothing.
 */
pip_status pip_voronoi_radial_bounds(pip_ctx ctx, const double *V, int32_t n, float *out,
                                     hipStream_t stream);

/*
 * The float32 screen table of one polygon, as pip_voronoi (test 0) or
 * pip_sign_of_offset (test 1) derive it for the vector screen (matrix 0) or
 * the matrix-core screen (matrix 1), for tests and diagnostics (the error
 * band is not in the paper; it keeps Algorithm 5's binary64 answer while
 * the margins of Eq. 11 are computed in float32).
 *   V    [n][2] binary64 vertices, 3 <= n <= PIP_MAX_EDGES.
 *   out  [12 + 4 n4] float32 (device), n4 = n rounded up to a multiple of 4:
 *        out[0..12) = o_x, o_y (the local origin, fl32(p_0)), KQ, KA, KB, KC
 *        (the band E = KQ (X^2 + Y^2) + KA |X| + KB |Y| + KC, X, Y the
 *        point's float32 local coordinates), n4, the polygon's pip_status,
 *        RQ (where |X| + |Y| <= RQ for every point of a screened chunk, the
 *        vector screens use E = max(KA, KB) (|X| + |Y|) + KC), SO (sign of
 *        offset: for fl32(|X| + |Y|) < SO some edge's offset is known to
 *        clear the band on the inner side, so one edge cleared on the outer
 *        side decides "outside"; 0 for Voronoi and for unusable polygons),
 *        then two zeros; then n4 rows (A_i, B_i, -C_i, 0) with margin
 *        m_i = A_i X + B_i Y - C_i (Voronoi; rows past n repeat edge 0) or
 *        sg (-dV_y, dV_x, -R_i, 0) (sign of offset, Algorithm 2's offset
 *        LHS - RHS in the local frame, sg = -1 for a clockwise polygon so
 *        that the inner side is positive).  A point is decided in float32
 *        only when its largest margin (sign of offset: its smallest
 *        offset) clears the band.
 * Asynchronous on `stream`; allocates nothing.  Errors: PIP_EINVAL for a bad
 * argument, PIP_EUNSUPPORTED for n > PIP_MAX_EDGES.
 */
pip_status pip_screen_table(pip_ctx ctx, int32_t test, int32_t matrix, const double* V, int32_t n,
                            float* out, hipStream_t stream);

/*
 * Diagnostic for tests: the float32 matrix-core multiply-add that the
 * matrix-core screen of pip_voronoi / pip_sign_of_offset evaluates (the margin
 * of Eq. 11 as A X + B Y + c, Section 4), on caller-chosen operands, so that
 * its rounding can be checked against the error bound the screen's band
 * assumes (within 4 u of |A X| + |B Y| + |c|, u = 2^-24).
 *   in   [count][5] float32 (device): A, B, c, X, Y per entry.
 *   out  [count] float32 (device): the sum as v_mfma_f32_32x32x2f32 forms it
 *        (entry e is row and column e % 32 of its group's product).
 * Asynchronous on `stream`; allocates nothing.
 */
pip_status pip_mfma_margin_probe(pip_ctx ctx, const float *in, int64_t count, float *out,
                                 hipStream_t stream);

/*
 * Voronoi point-inclusion test (Section 4, Algorithm 5) of m points against
 * one convex polygon.  Q is [m][2] of type qdt; labels [ceil(m/32)] words;
 * status optional [1].  The polygon's generators are derived on the device
 * in binary64; margins are screened in float32 with a proven error band and
 * the undecided points are re-decided in binary64.  For float32 points one
 * launch handles fewer than 2^23 chunks of 512 points per wave of the grid
 * (about 2^44 points on a full device); beyond that the call returns
 * PIP_EUNSUPPORTED and the points must be split over several calls.
 */
pip_status pip_voronoi(pip_ctx ctx, const double *V, int32_t n, const void *Q, pip_dtype qdt,
                       int64_t m, uint32_t *labels, int32_t *status, hipStream_t stream);

/* Sign-of-offset test (Section 2.2, Algorithm 2): inside iff every edge gives
 * the same answer to LHS < RHS.  Same arguments and guarantees as
 * pip_voronoi; status reports non-convex input. */
pip_status pip_sign_of_offset(pip_ctx ctx, const double *V, int32_t n, const void *Q,
                              pip_dtype qdt, int64_t m, uint32_t *labels, int32_t *status,
                              hipStream_t stream);

/* Ray-crossing test (Section 2.1, Algorithm 1) with a ray towards +x; the
 * polygon may be any simple polygon (convexity is not required or checked).
 * Labels equal Algorithm 1 in binary64.  Float64 points are evaluated in
 * binary64 directly; for float32 points the in-range test compares Q_y with
 * each vertex height rounded up to float32 (exact for float32 Q_y), the
 * line test is screened in float32 against the sign-of-offset band, and the
 * points with an undecided line test are re-decided in binary64. */
pip_status pip_ray_crossing(pip_ctx ctx, const double *V, int32_t n, const void *Q,
                            pip_dtype qdt, int64_t m, uint32_t *labels, int32_t *status,
                            hipStream_t stream);

/* The same Voronoi test evaluated entirely in float32 (generators derived in
 * float32 in the global frame, label = largest margin <= 0), with no error
 * band and no binary64 recheck.  A speed reference: its labels are NOT
 * guaranteed to equal the binary64 algorithm near the boundary. */
pip_status pip_voronoi_fp32_plain(pip_ctx ctx, const double *V, int32_t n, const void *Q,
                                  pip_dtype qdt, int64_t m, uint32_t *labels, int32_t *status,
                                  hipStream_t stream);

/* Largest Voronoi margin per point, max_i (|p - p_0|^2 - |p - p_i|^2)
 * (Eq. 11 rearranged; <= 0 inside), evaluated in float32 from the binary64
 * generators in the polygon-local frame.  max_margin is [m] float32. */
pip_status pip_voronoi_max_margin(pip_ctx ctx, const double *V, int32_t n, const void *Q,
                                  pip_dtype qdt, int64_t m, float *max_margin, int32_t *status,
                                  hipStream_t stream);

/* Coverage raster (Section 1's graphics use: every pixel's membership by a
 * point inclusion test; Section 4, Algorithm 5 per pixel).  Pixel (i, j),
 * 0 <= i < width, 0 <= j < height, is the binary64 point
 * (x0 + i*dx, y0 + j*dy), each coordinate one product and one sum, rounded to
 * nearest; no point array is read.  labels (device, caller-owned) holds
 * height rows of ceil(width / 32) uint32 words: bit i % 32 of word
 * j * ceil(width / 32) + i / 32 is 1 iff pixel (i, j) is inside, equal to the
 * plain binary64 algorithm; bits past width are 0.  status as in
 * pip_voronoi.  Errors: PIP_EINVAL for a bad polygon argument, a non-finite
 * x0, y0, dx or dy, a negative size, a NULL or misaligned labels;
 * PIP_EUNSUPPORTED for width > 2^24 or height > 2^31.  width or height 0
 * writes no label (status is still written when given). */
pip_status pip_voronoi_raster(pip_ctx ctx, const double *V, int32_t n, double x0, double y0,
                              double dx, double dy, int64_t width, int64_t height,
                              uint32_t *labels, int32_t *status, hipStream_t stream);

/* Builds the index of P polygons (device CSR: vtx_off [P+1] int64 with
 * vtx_off[P] == total_vertices, V [total_vertices][2] float64).  Per polygon:
 * generators (Algorithms 3-4), the float32 screen table and band, and a box
 * widened by the distance within which binary64 rounding can put an outside
 * point inside; a uniform grid of about `cells` square cells (0: one per
 * polygon; at most 2^24) lists every polygon whose box meets a cell.  A
 * polygon with fewer than 3 vertices contains no point; degenerate,
 * non-convex or non-finite polygons are kept in a list every query tests.
 * status (device [P] int32, optional) receives each polygon's pip_status.
 * Synchronizes `stream` (the list sizes are read back) and allocates.
 * Errors: PIP_EINVAL for bad arguments or vtx_off[P] != total_vertices,
 * PIP_EUNSUPPORTED for a polygon with more than 64 vertices or 2^31 or more
 * list entries, PIP_ENOMEM. */
pip_status pip_index_create(pip_ctx ctx, int32_t P, const int64_t *vtx_off, const double *V,
                            int64_t total_vertices, int64_t cells, int32_t *status,
                            hipStream_t stream, pip_index *out);

/* Locates m float32 points (Q [m][2], device): ids[j] (device [m] int32) is
 * the smallest k whose polygon contains point j under the Voronoi test
 * (Section 4, Algorithm 5; closed, equal to the plain binary64 algorithm),
 * or -1; non-finite points get -1.  Asynchronous on `stream`. */
pip_status pip_index_locate(pip_index index, const float *Q, int64_t m, int32_t *ids,
                            hipStream_t stream);

/* The same query with the points first binned by super-cell (at most 1024
 * blocks of grid cells, then sorted by cell within each 2048-point tile) so
 * that neighbouring lanes test the same candidates:
 * same ids as pip_index_locate.  workspace (device, caller-owned, 256-byte
 * aligned) holds the bin counts and a 16-byte copy of every point:
 * pip_index_locate_workspace_bytes(index, m) bytes (0 for a NULL index or
 * negative m).  Allocates nothing; asynchronous on `stream`.  Errors:
 * PIP_EINVAL for bad arguments or a short workspace, PIP_EUNSUPPORTED for
 * m >= 2^31 (the copy is indexed with 32-bit offsets). */
size_t pip_index_locate_workspace_bytes(pip_index index, int64_t m);
pip_status pip_index_locate_binned(pip_index index, const float *Q, int64_t m, int32_t *ids,
                                   void *workspace, size_t ws_bytes, hipStream_t stream);

/* Grid cells requested and list entries (cells and the global list). */
pip_status pip_index_info(pip_index index, int64_t *cells, int64_t *entries);

void pip_index_destroy(pip_index index);

/* ------------------------------------------------------------------------
 * Batched Voronoi inclusion: P convex polygons, each against its own point
 * set, in one persistent launch (Section 4, Algorithm 5 per polygon; the
 * generators of every polygon are derived once and stored beside it, the
 * precomputation Section 7 suggests for static polygons).
 *
 *   vtx_off       [P+1] int64, non-decreasing; polygon k has vertices
 *                 V[vtx_off[k] .. vtx_off[k+1]) of V ([total_vertices][2]
 *                 binary64).
 *   pt_off        [P+1] int64, non-decreasing; polygon k is tested against
 *                 points Q[pt_off[k] .. pt_off[k+1]) of Q ([total_points][2]
 *                 float32, 8-byte aligned).
 *   lbl_word_off  [P+1] int64; the labels of polygon k start at word
 *                 lbl_word_off[k] of `labels` (every set starts on a fresh
 *                 32-bit word; bit j of the set's words is its point j;
 *                 words must not overlap: lbl_word_off[k+1] - lbl_word_off[k]
 *                 >= ceil(set size / 32)).  Bits past a set's last point in its
 *                 last word are written as 0.
 *   status        optional [P] int32 device status per polygon; a polygon
 *                 with n < 3 gets PIP_EINVAL, n > 64 or a point set of 2^32 or
 *                 more points PIP_EUNSUPPORTED, and its points are all
 *                 labelled 0; offsets outside
 *                 [0, total_vertices] / [0, total_points] give PIP_EINVAL and
 *                 leave that polygon's labels untouched.
 *   workspace     device buffer of pip_voronoi_batched_workspace_bytes(P,
 *                 total_vertices, total_points) bytes, 256-byte aligned, owned
 *                 by the caller, not shared by calls that may overlap.
 *   config        tile shape; NULL for the default.  Labels do not depend on it.
 */
typedef struct {
    int32_t chunks_per_tile; /* a wave walks tiles of this many 256-point chunks */
    int32_t blocks_per_cu;   /* persistent workgroups (256 threads) per CU */
} pip_batched_config;

size_t pip_voronoi_batched_workspace_bytes(int32_t P, int64_t total_vertices,
                                           int64_t total_points);

pip_status pip_voronoi_batched(pip_ctx ctx, int32_t P, const int64_t *vtx_off, const double *V,
                               int64_t total_vertices, const int64_t *pt_off, const float *Q,
                               int64_t total_points, const int64_t *lbl_word_off,
                               uint32_t *labels, int32_t *status, void *workspace,
                               size_t workspace_bytes, const pip_batched_config *config,
                               hipStream_t stream);

/*
 * pip_voronoi_batched for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, labels and status without the workspace.
 * The polygon tables and chunk descriptors go to a static device array of
 * the library, PIP_BATCHED_SCRATCH_BYTES bytes on every GPU the library
 * runs on, held until the process ends; the call allocates nothing.
 *   Limit: a request whose pip_voronoi_batched_workspace_bytes(P,
 *   total_vertices, total_points) exceeds PIP_BATCHED_SCRATCH_BYTES returns
 *   PIP_EUNSUPPORTED (32 MiB holds about 9e8 points over 4096 polygons of
 *   up to 32 edges); such a batch needs pip_voronoi_batched with a workspace.
 *   Sharing: every call on one GPU uses that GPU's one array, whose contents
 *   are those of the last call (every word a launch reads is written earlier
 *   in the same launch).  Calls that overlap on one GPU -- on different
 *   streams, or from several host threads without ordering -- race on the
 *   array and give wrong labels; serialise them (one stream, or events).
 *   Errors: as pip_voronoi_batched; PIP_EHIP if the array's device address
 *   could not be obtained when the context was created.
 */
#define PIP_BATCHED_SCRATCH_BYTES ((size_t)32 << 20)
pip_status pip_voronoi_batched_noalloc(pip_ctx ctx, int32_t P, const int64_t *vtx_off,
                                       const double *V, int64_t total_vertices,
                                       const int64_t *pt_off, const float *Q,
                                       int64_t total_points, const int64_t *lbl_word_off,
                                       uint32_t *labels, int32_t *status,
                                       const pip_batched_config *config, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Non-convex polygons (the extension Section 7 names; the test of Section 4
 * needs a convex polygon): a simple polygon split into convex pieces whose
 * vertices are vertices of the polygon.  Each piece gets its own generators
 * (Section 3, Algorithms 3-4) and a point is inside iff the closed Voronoi
 * test (Algorithm 5, binary64) of at least one piece puts it inside.  In
 * exact arithmetic the union of the closed pieces is the closed polygon; in
 * binary64 the label can depend on the decomposition within rounding reach
 * of the pieces' boundaries, so it is always "the union of these pieces".
 *
 * pip_convex_decompose: one decomposition, on the host (no device work):
 *   ear clipping with exact orientation signs, then removal of every
 *   diagonal whose two sides merge into a piece that is strictly convex at
 *   both ends of the diagonal and has at most max_piece_vertices vertices
 *   (Hertel-Mehlhorn: at most four times the fewest convex pieces).  Vertices
 *   collinear with both neighbours may be left out of every piece (they lie
 *   on an edge of a piece).
 *   V            [n][2] HOST binary64, a simple polygon, either orientation,
 *                3 <= n <= 2^20 (self-intersection is not detected in
 *                general; an input with no ear left returns PIP_EINVAL).
 *   max_piece_vertices  3..PIP_MAX_EDGES.
 *   piece_off    HOST int32 [n - 1]: receives K + 1 offsets.
 *   piece_idx    HOST int32 [3 (n - 2)]: receives the pieces' vertex
 *                indices, each piece in the polygon's cyclic order.
 *   num_pieces   receives K; idx_count receives piece_off[K].
 *   Errors: PIP_EINVAL (NULL pointer, n out of range, non-finite vertex,
 *   zero area, not simple).  Runs on the calling thread; thread-safe.
 *
 * pip_voronoi_pieces: labels of m points against the union of K pieces.
 *   V            [n][2] binary64 vertices (device).
 *   piece_off    [K + 1] int32 (device), non-decreasing, piece_off[K] =
 *                idx_count; piece_idx [idx_count] int32 (device), values in
 *                [0, n).  A piece of 3..PIP_MAX_EDGES vertices, in cyclic
 *                order (either orientation).
 *   Q, qdt, m, labels  as pip_voronoi.
 *   status       optional [K] int32 (device): per piece, PIP_OK or the
 *                generator status of pip_voronoi (a non-convex piece gives
 *                PIP_ENONCONVEX and still takes part with Algorithm 5's
 *                answer for it); PIP_EINVAL for a piece with fewer than 3
 *                vertices or an index / offset out of range, PIP_EUNSUPPORTED
 *                for more than PIP_MAX_EDGES vertices: such a piece contains
 *                no point.
 *   workspace    device, 256-byte aligned, pip_voronoi_pieces_workspace_bytes
 *                (K, idx_count) bytes, caller-owned, not shared by
 *                overlapping calls.
 *   The piece tables (32 bytes per piece plus 16 per row, rows = idx_count
 *   + 3 K) live in each workgroup's LDS: at most PIP_PIECES_MAX_TABLE_BYTES,
 *   else PIP_EUNSUPPORTED.  Margins are screened in float32 in one frame
 *   shared by the pieces (origin fl32(v_0)) with the proven band of
 *   pip_voronoi; undecided points are re-decided in binary64 against every
 *   piece.
 */
#define PIP_PIECES_MAX_TABLE_BYTES 65536
pip_status pip_convex_decompose(const double *V, int32_t n, int32_t max_piece_vertices,
                                int32_t *piece_off, int32_t *piece_idx, int32_t *num_pieces,
                                int64_t *idx_count);
size_t pip_voronoi_pieces_workspace_bytes(int32_t K, int64_t idx_count);
pip_status pip_voronoi_pieces(pip_ctx ctx, const double *V, int64_t n, int32_t K,
                              const int32_t *piece_off, const int32_t *piece_idx,
                              int64_t idx_count, const void *Q, pip_dtype qdt, int64_t m,
                              uint32_t *labels, int32_t *status, void *workspace,
                              size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Plans: a batched request bound to its buffers, with a workspace the plan
 * allocates (pip_plan_create_batched is the only call that allocates device
 * memory, besides pip_plan_autotune's comparison buffers), a tile shape
 * chosen by timing candidates on the real data, and the whole launch
 * sequence captured in a hipGraph.
 *
 *   pip_plan_create_batched  arguments as pip_voronoi_batched; reads
 *                            lbl_word_off[P] from the device (synchronous).
 *   pip_plan_autotune        runs every candidate tile shape (chunks per tile
 *                            1, 4, 16, 64, whole range; three grid sizes) `reps`
 *                            times on `stream`, requires bitwise-identical
 *                            labels from all of them (PIP_EHIP otherwise),
 *                            keeps the fastest and captures the hipGraph.
 *                            Synchronises `stream`.
 *   pip_plan_launch          replays the graph on `stream` (captures the
 *                            default shape first if the plan was never tuned).
 *   pip_plan_config          the chosen shape and its measured time (ms, -1 if
 *                            not tuned).
 *   pip_plan_set_config      force a shape (recaptures the graph).
 *   pip_plan_destroy         frees the plan; destroy plans before their ctx.
 * The buffers bound at creation must stay valid while the plan is used.
 */
typedef struct pip_plan_s *pip_plan;

pip_status pip_plan_create_batched(pip_ctx ctx, int32_t P, const int64_t *vtx_off,
                                   const double *V, int64_t total_vertices,
                                   const int64_t *pt_off, const float *Q, int64_t total_points,
                                   const int64_t *lbl_word_off, uint32_t *labels,
                                   int32_t *status, pip_plan *out);
pip_status pip_plan_autotune(pip_plan plan, int32_t reps, hipStream_t stream);
pip_status pip_plan_launch(pip_plan plan, hipStream_t stream);
pip_status pip_plan_config(pip_plan plan, pip_batched_config *config, float *best_ms);
pip_status pip_plan_set_config(pip_plan plan, const pip_batched_config *config);
void pip_plan_destroy(pip_plan plan);

/* All-pairs plans (Section 1's collision check: one footprint at many poses
 * against one cloud): pip_voronoi_allpairs bound to its buffers (V
 * [P][n][2], Q [m][2], labels [P][ceil(m/32)], counts [P], optional status
 * [P]; the plan allocates its workspace).  The variants are the dense
 * screen, the bounding-disk cull, antipodal pairs and both; all give the
 * same labels and counts.  pip_plan_autotune runs each on the bound data,
 * requires labels and counts equal word for word to the dense run's
 * (PIP_EHIP otherwise), keeps the fastest and captures the hipGraph;
 * pip_plan_launch replays it (capturing the context's options first if the
 * plan was never tuned).  pip_plan_config / pip_plan_set_config reject
 * these plans (and collision-cost plans, below); pip_plan_variant and
 * pip_plan_set_variant read and force their variant (recapturing the
 * graph).  The buffers must stay valid while the plan is used. */
typedef struct {
    int32_t cull;  /* 1: skip (polygon, wave) pairs whose bounding disk misses */
    int32_t pair;  /* 1: antipodal edge pairs for centrally symmetric polygons */
} pip_variant_config;
pip_status pip_plan_create_allpairs(pip_ctx ctx, int32_t P, int32_t n, const double *V,
                                    const float *Q, int64_t m, uint32_t *labels, int32_t *counts,
                                    int32_t *status, pip_plan *out);
pip_status pip_plan_variant(pip_plan plan, pip_variant_config *config, float *best_ms);
pip_status pip_plan_set_variant(pip_plan plan, const pip_variant_config *config);

/* ------------------------------------------------------------------------
 * Poses and all pairs (the collision check of Section 1: a convex car
 * footprint placed at many poses, tested against a lidar point cloud).
 *
 * pip_poses_to_polygons: world vertices of footprint F ([n][2] binary64,
 *   body frame) at K poses.  pose [K][3] float32 (x, y, theta), cs [K][2]
 *   binary64 (cos theta, sin theta, supplied by the caller so that nobody
 *   recomputes them); V_out [K][n][2] binary64 receives
 *   ((c vx - s vy) + x, (s vx + c vy) + y) per vertex, evaluated in binary64
 *   in that order.
 *
 * pip_voronoi_allpairs: P convex polygons of n vertices each (V [P][n][2]
 *   binary64), every one against all m points of Q ([m][2] float32).
 *   labels [P][ceil(m/32)] words, row k = polygon k, same bit layout as
 *   pip_voronoi; counts optional [P] int32 = inside points per polygon
 *   (overwritten); status optional [P].  Labels are bit-identical to the
 *   binary64 Voronoi algorithm for each polygon.  workspace: device buffer of
 *   pip_voronoi_allpairs_workspace_bytes(P, n) bytes, 256-byte aligned.
 */
pip_status pip_poses_to_polygons(pip_ctx ctx, const double *footprint, int32_t n, const float *pose,
                                 const double *cs, int64_t K, double *V_out, hipStream_t stream);

size_t pip_voronoi_allpairs_workspace_bytes(int32_t P, int32_t n);

pip_status pip_voronoi_allpairs(pip_ctx ctx, int32_t P, int32_t n, const double *V, const float *Q,
                                int64_t m, uint32_t *labels, int32_t *counts, int32_t *status,
                                void *workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * pip_voronoi_allpairs_csr: the same all-pairs test for P convex polygons of
 * uneven vertex counts (Section 4, Algorithm 5 per polygon; Section 1's
 * collision check against many different shapes).
 *   vtx_off  [P+1] int64 (device), non-decreasing: polygon k has vertices
 *            V[vtx_off[k] .. vtx_off[k+1]) of V ([total_vertices][2]
 *            binary64).  total_vertices + 3 P < 2^31.
 *   Q, m, labels [P][ceil(m/32)], counts, status: as pip_voronoi_allpairs.
 *            A polygon with fewer than 3 vertices or a range outside
 *            [0, total_vertices] gets PIP_EINVAL, one with more than
 *            PIP_MAX_EDGES PIP_EUNSUPPORTED; its labels and count are 0.
 *   workspace  pip_voronoi_allpairs_csr_workspace_bytes(P, total_vertices)
 *            bytes (device, 256-byte aligned, caller-owned).
 * The options PIP_OPT_ALLPAIRS_CULL and PIP_OPT_ALLPAIRS_PAIR apply as for
 * pip_voronoi_allpairs; labels and counts never depend on them.
 */
size_t pip_voronoi_allpairs_csr_workspace_bytes(int32_t P, int64_t total_vertices);
pip_status pip_voronoi_allpairs_csr(pip_ctx ctx, int32_t P, const int64_t *vtx_off,
                                    const double *V, int64_t total_vertices, const float *Q,
                                    int64_t m, uint32_t *labels, int32_t *counts,
                                    int32_t *status, void *workspace, size_t workspace_bytes,
                                    hipStream_t stream);

/* ------------------------------------------------------------------------
 * Differentiable collision cost.  For edge i of a convex footprint the
 * Voronoi margin (Eq. 11) divided by -2|p_i - p_0| is the signed distance of
 * a point to edge line i, positive inside; the cost of a pose is the sum over
 * the cloud of relu(min_i of it) -- the total penetration depth -- evaluated
 * with every point moved into the body frame, p_b = R(theta)^T (p - t).
 *
 *   footprint  [n][2] float32 body-frame vertices, 3 <= n <= PIP_MAX_EDGES.
 *   pose       [K][3] float32 (x, y, theta); cos/sin of theta are taken in
 *              binary64 and rounded to float32.
 *   Q          [m][2] float32 points (non-finite points contribute nothing).
 *   cost       [K] float32 (forward output).
 *   grad_cost  [K] float32 upstream gradient (backward input).
 *   grad_pose  [K][3] float32, overwritten: d(sum_k grad_cost_k C_k)/d pose_k.
 *   grad_footprint [n][2] float32, overwritten: gradient to the footprint
 *              vertices, chained by hand through the generator construction
 *              (reflection, Eq. 8; centroid, Algorithm 3) in binary64.
 *   residual   optional [2] float32: |total gradient reaching p_0| and the
 *              sum of the magnitudes it cancels (exactly 0 in exact
 *              arithmetic, because every distance depends on its edge line
 *              only).
 *   workspace  pip_cost_workspace_bytes(n, K, m) bytes, 256-byte aligned.
 * Conventions: relu'(0) = 0; on a tie in the min, the lowest edge index.
 * Results are deterministic (fixed-order reductions, no float atomics).
 */
size_t pip_cost_workspace_bytes(int32_t n, int64_t K, int64_t m);

pip_status pip_cost_fwd(pip_ctx ctx, const float *footprint, int32_t n, const float *pose, int64_t K,
                        const float *Q, int64_t m, float *cost, void *workspace,
                        size_t workspace_bytes, hipStream_t stream);

pip_status pip_cost_bwd(pip_ctx ctx, const float *footprint, int32_t n, const float *pose, int64_t K,
                        const float *Q, int64_t m, const float *grad_cost, float *grad_pose,
                        float *grad_footprint, float *residual, void *workspace,
                        size_t workspace_bytes, hipStream_t stream);

/* Collision-cost plans: pip_cost_fwd (backward = 0; cost) or pip_cost_bwd
 * (backward = 1; grad_cost, grad_pose, grad_footprint, optional residual)
 * bound to its buffers, with a workspace the plan allocates.
 * pip_plan_autotune times the cost with and without the bounding-disk cull
 * (antipodal pairs as the context's PIP_OPT_COST_PAIR at creation), requires
 * the outputs of both equal word for word (PIP_EHIP otherwise), keeps the
 * faster and captures the hipGraph; pip_plan_launch replays it;
 * pip_plan_variant / pip_plan_set_variant read and force (cull, pair).
 * Errors as pip_cost_fwd / pip_cost_bwd, PIP_EINVAL for K < 1,
 * PIP_ENOMEM. */
pip_status pip_plan_create_cost(pip_ctx ctx, int32_t backward, const float *footprint, int32_t n,
                                const float *pose, int64_t K, const float *Q, int64_t m,
                                float *cost, const float *grad_cost, float *grad_pose,
                                float *grad_footprint, float *residual, pip_plan *out);

/* One creator for every plan kind (the plan interface of the boundary as a
 * single call): `desc` points to the descriptor of `kind` and holds exactly
 * the arguments of the typed creator, which it calls:
 *   PIP_PLAN_BATCHED   pip_batched_desc   -> pip_plan_create_batched
 *   PIP_PLAN_ALLPAIRS  pip_allpairs_desc  -> pip_plan_create_allpairs
 *   PIP_PLAN_COST_FWD  pip_cost_desc      -> pip_plan_create_cost (backward 0)
 *   PIP_PLAN_COST_BWD  pip_cost_desc      -> pip_plan_create_cost (backward 1)
 * The descriptor is read during the call only; the buffers it names are
 * bound to the plan as by the typed creator.  Errors: PIP_EINVAL for a
 * NULL ctx, desc or out or an unknown kind, else the typed creator's. */
typedef enum {
    PIP_PLAN_BATCHED = 0,
    PIP_PLAN_ALLPAIRS = 1,
    PIP_PLAN_COST_FWD = 2,
    PIP_PLAN_COST_BWD = 3
} pip_plan_kind;
typedef struct {
    int32_t P;
    const int64_t *vtx_off;       /* [P+1] */
    const double *V;              /* [total_vertices][2] */
    int64_t total_vertices;
    const int64_t *pt_off;        /* [P+1] */
    const float *Q;               /* [total_points][2] */
    int64_t total_points;
    const int64_t *lbl_word_off;  /* [P+1] */
    uint32_t *labels;
    int32_t *status;              /* [P], optional */
} pip_batched_desc;
typedef struct {
    int32_t P, n;
    const double *V;              /* [P][n][2] */
    const float *Q;               /* [m][2] */
    int64_t m;
    uint32_t *labels;             /* [P][ceil(m/32)] */
    int32_t *counts;              /* [P] */
    int32_t *status;              /* [P], optional */
} pip_allpairs_desc;
typedef struct {
    const float *footprint;       /* [n][2] */
    int32_t n;
    const float *pose;            /* [K][3] */
    int64_t K;
    const float *Q;               /* [m][2] */
    int64_t m;
    float *cost;                  /* forward: [K] */
    const float *grad_cost;       /* backward: [K] */
    float *grad_pose;             /* backward: [K][3] */
    float *grad_footprint;        /* backward: [n][2] */
    float *residual;              /* backward: optional */
} pip_cost_desc;
pip_status pip_plan_create(pip_ctx ctx, pip_plan_kind kind, const void *desc, pip_plan *out);

#ifdef __cplusplus
}
#endif

#endif /* PIP_VORONOI_H */
