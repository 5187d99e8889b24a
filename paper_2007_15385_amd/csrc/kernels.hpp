// Host-side launchers of the HIP kernels (private to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pipdev {

// K_RAY32: ray crossing with the float32 pre-screen (prepared like K_SOO, plus
// the binary64 ray table and the rounded-up vertex heights).
enum TestKind : int { K_VORONOI = 0, K_SOO = 1, K_RAY = 2, K_PLAIN = 3, K_MARGIN = 4, K_RAY32 = 5 };

struct StreamLaunch {
    int kind;             // TestKind
    const double* V;      // device [n][2]
    int n;
    const void* Q;        // device [m][2], float32 or binary64
    int qdt;              // 0 float32, 1 binary64
    int64_t m;
    uint32_t* labels;     // device [ceil(m/32)]
    float* margin;        // device [m] (margin kernel only)
    int32_t* status;      // device [1] or null
    int max_blocks;       // upper bound on the persistent grid
    int mfma;             // 1: matrix-core margins (float32 points, Voronoi / sign of offset)
    int radial;           // 1: radial pre-screen (float32 points, Voronoi); wins over mfma
    hipStream_t stream;
};

hipError_t launch_stream_mfma(const StreamLaunch& L);
hipError_t stream_mfma_max_blocks_per_cu(int kind, int n, int* out);
hipError_t launch_mfma_probe(const float* in, int64_t count, float* out, hipStream_t stream);

hipError_t launch_stream(const StreamLaunch& L);
hipError_t radial_max_blocks_per_cu(int* out);
hipError_t launch_radial_bounds(const double* V, int n, float* out, hipStream_t stream);

// Per-polygon table row of the batched and all-pairs paths.
struct alignas(16) PolyHdr {
    float ox, oy;          // float32 local origin (p_0 rounded)
    float KQ, KA, KB, KC;  // band constants
    int n, n4;             // edges (0 for an invalid polygon), padded to 4
    int status;            // pip_status of this polygon
    float cx, cy, rad;     // disk (float32 centre, radius rounded up) containing the polygon
    int npair;             // > 0: coefficient rows are npair antipodal edge pairs (all pairs)
    int radial;            // 1: the batched screen takes the radial pre-screen (table usable)
    int row;               // all pairs over CSR polygons: first coefficient row (the
                           // polygon's generators start at row - 2k for polygon k)
    float RQ;              // band fold radius (batched): for |X| + |Y| <= RQ the band is
                           // max(KA, KB) (|X| + |Y|) + KC
};

// Device view of a batched request plus its workspace.
struct BatchedDev {
    int64_t P;
    const int64_t* vtx_off;
    const double* V;
    int64_t total_vertices;
    const int64_t* pt_off;
    const void* Q;
    int64_t total_points;
    const int64_t* lbl_word_off;
    uint32_t* labels;
    int32_t* status;
    PolyHdr* hdr;
    float4* coef;
    double2* gen;
    int64_t* chunk_cnt;
    int64_t* chunk_off;
    void* desc;
    int64_t* misc;
    int64_t max_chunks;
    float* radial;   // [P][kRadialRow]: (T_in, T_out) of octants 0..7, then T_far
    int radial_min;  // polygons with at least this many edges use it; 0: none
};

constexpr int kRadialRow = 20;  // floats per polygon in the batched radial table

struct BatchedLayout {
    size_t hdr, coef, gen, chunk_cnt, chunk_off, desc, misc, radial;
    int64_t max_chunks;
};

size_t batched_workspace_layout(int64_t P, int64_t total_vertices, int64_t total_points,
                                BatchedLayout* L);
hipError_t launch_batched(const BatchedDev& D, int chunks_per_tile, int blocks, hipStream_t stream);
hipError_t batched_max_blocks_per_cu(int* out);
struct AllpairsLayout {
    size_t hdr, coef, gen;
};
size_t allpairs_workspace_layout(int64_t P, int n, AllpairsLayout* L);
int allpairs_group(int n);
hipError_t launch_poses_to_polygons(const double* F, int n, const float* pose, const double* cs,
                                    int64_t K, double* Wout, hipStream_t stream);
hipError_t launch_allpairs(int64_t P, int n, const double* V, const float* Q, int64_t m,
                           uint32_t* labels, int32_t* counts, int32_t* status, void* ws, int cull,
                           int pair, hipStream_t stream);
// All pairs over CSR polygons of uneven vertex counts (vtx_off [P+1]).
size_t allpairs_csr_workspace_layout(int64_t P, int64_t total_vertices, AllpairsLayout* L);
hipError_t launch_allpairs_csr(int64_t P, const int64_t* vtx_off, const double* V,
                               int64_t total_vertices, const float* Q, int64_t m,
                               uint32_t* labels, int32_t* counts, int32_t* status, void* ws,
                               int cull, int pair, hipStream_t stream);
// Non-convex polygon as a union of convex pieces (pieces.hip).
struct PiecesLayout {
    size_t hdr, rows, gens;
};
struct PiecesLaunch {
    const double* V;      // device [n][2]
    int64_t n;
    int K;                // pieces
    const int32_t* off;   // device [K+1]
    const int32_t* idx;   // device [idx_count]
    int64_t idx_count;
    const void* Q;        // device [m][2] float32 or binary64
    int qdt;
    int64_t m;
    uint32_t* labels;
    int32_t* status;      // device [K] or null
    void* ws;
    int max_blocks;
};
size_t pieces_workspace_layout(int64_t K, int64_t idx_count, PiecesLayout* L);
size_t pieces_lds_bytes(int64_t K, int64_t idx_count);
hipError_t pieces_max_blocks_per_cu(int qdt, size_t lds, int* out);
hipError_t launch_pieces(const PiecesLaunch& A, hipStream_t stream);
}  // namespace pipdev
#include <vector>
namespace pipdev {
int convex_decompose_host(const double* V, int n, int max_piece, std::vector<int32_t>& off,
                          std::vector<int32_t>& idx);
// Point-location index: one record per polygon (64 bytes), the grid.
struct alignas(16) LocRec {
    float ox, oy;          // float32 local origin
    float KQ, KA, KB, KC;  // band constants
    int n, n4;             // edges, padded to 4
    int64_t qoff;          // query record (float4 units)
    int64_t gen_off;       // first generator (double2): p_0, then p_i
    float bx0, by0, bx1, by1;  // widened, outward-rounded box
    int status;            // pip_status of the polygon
    int usable;            // 0: contains no point; 1: in the grid cells; 2: global list
    float rfar;            // binary64 calls no point inside beyond the box within this
                           // distance of (ox, oy) (rounded down)
};
// Cell-list entry: the polygon's box, index, query-record offset (float4
// units) and edge counts: record = {ox, oy, KQ, KA}, {KB, KC, n | n4 << 16,
// generator offset}, then n4 coefficient rows.
struct alignas(32) LocEntry {
    float bx0, by0, bx1, by1;
    int k, qoff, nn, pad;  // nn = n | n4 << 16
};
struct LocGrid {
    float x0, y0, x1, y1;  // union of the cell-listed boxes
    float inv_w, inv_h;    // cells per unit length
    int gx, gy;            // grid shape (gx * gy <= requested cells)
    int any;               // some polygon is cell-listed
    float fx0, fy0, fx1, fy1;  // near region: beyond it a point tests every polygon
};
hipError_t index_prepare(int64_t P, const int64_t* vtx_off, const double* V, LocRec* rec,
                         float4* qrec, double2* gen, int32_t* status, int32_t* flags,
                         hipStream_t stream);
hipError_t index_grid(int64_t P, LocRec* rec, int64_t cells, LocGrid* grid, int32_t* cnt,
                      unsigned long long* total, hipStream_t stream);
hipError_t index_fill(int64_t P, const LocRec* rec, const LocGrid* grid, int64_t cells,
                      int32_t* cnt, int32_t* cell_off, LocEntry* list, hipStream_t stream);
hipError_t launch_locate(const LocRec* rec, int64_t P, const float4* qrec, const double2* gen,
                         const LocGrid* grid, const int32_t* cell_off, const LocEntry* list,
                         const float* Q, int64_t m, int32_t* ids, int max_blocks,
                         hipStream_t stream);
hipError_t locate_max_blocks_per_cu(int* out);
size_t locate_binned_workspace(int nbins, int64_t m, size_t* o_cnt, size_t* o_off, size_t* o_fill,
                               size_t* o_pts);
hipError_t launch_locate_binned(const LocRec* rec, int64_t P, const float4* qrec,
                                const double2* gen, const LocGrid* grid,
                                const int32_t* cell_off, const LocEntry* list, int sf, int sgx,
                                int nbins, const float* Q, int64_t m, int32_t* ids, void* ws,
                                int cus, hipStream_t stream);
// Coverage raster: pixel (i, j) = (x0 + i dx, y0 + j dy), binary64.
struct RasterGrid {
    double x0, y0, dx, dy;
    int64_t width, height;
};
hipError_t launch_raster(const double* V, int n, const RasterGrid& G, uint32_t* labels,
                         int32_t* status, int radial, int early, int max_blocks,
                         hipStream_t stream);
hipError_t raster_max_blocks_per_cu(int radial, int* out);
struct CostLayout {
    size_t tab, part_cost, part_pose, part_gen, stage;
    int T;
    int64_t G;
};
int cost_max_edges();
size_t cost_workspace_layout(int n, int64_t K, int64_t m, CostLayout* L);
hipError_t launch_cost(bool backward, const float* F, int n, const float* pose, int64_t K,
                       const float* Q, int64_t m, const float* grad_cost, float* cost,
                       float* grad_pose, float* grad_F, float* residual, void* ws, int cull,
                       int pair, hipStream_t stream);
hipError_t launch_count_diff(const uint32_t* a, const uint32_t* b, int64_t nwords,
                             unsigned long long* out, hipStream_t stream);
// float32 screen table as the streaming screens derive it (factor: 4.05 for
// the vector screen, kMfmaScreenFactor for the matrix cores)
constexpr double kMfmaScreenFactor = 6.05;
hipError_t launch_screen_table(const double* V, int n, int kind, double factor, float* out,
                               hipStream_t stream);
hipError_t launch_generators_one(const double* V, int n, double* P, int32_t* status,
                                 hipStream_t stream);
hipError_t stream_max_blocks_per_cu(int kind, int qdt, int* out);

}  // namespace pipdev
