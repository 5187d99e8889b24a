// Differentiable collision cost of a convex footprint at many poses against
// a point cloud, built on the Voronoi margin (Section 4, Eq. 11).
//
// For edge i the margin m_i = |p - p_0|^2 - |p - p_i|^2 divided by
// -2|p_i - p_0| is the signed distance of p to edge line i, positive on the
// side of p_0:  d_i(p) = k_i - n_i.p,  n_i = h_i / |h_i|,
// k_i = n_i.p_0 + |h_i|/2,  h_i = p_i - p_0  (p_i = p_0 mirrored across the
// edge line, Eq. 8).  The cost of pose (t, theta) is
//     C = sum_j relu(min_i d_i(p_b,j)),   p_b = R(theta)^T (p_j - t),
// the total penetration depth of the cloud into the footprint.
//
//   k_cost_prepare   one wave: generators of the footprint in binary64
//                    (Algorithms 3-4), float32 line table (-n_x, -n_y, k, |h|)
//                    and p_0.
//   k_cost<false>    forward: workgroup = 1024-point tile x 64 poses; per
//                    (pose, point) body-frame coordinates, min over edges,
//                    relu; per-(pose, tile) partial sums in a fixed order.
//   k_cost<true>     backward: recomputes the minimising edge (lowest index on
//                    ties) and accumulates, for every contributing pair,
//                    d/dt = R n, d/dtheta = -n_x p_b,y + n_y p_b,x (pose
//                    partials) and the derivatives of d to p_i and p_0 (table
//                    partials: per pose, one wave sum per edge that a point of
//                    the wave presses on, added to the wave's LDS row; no
//                    float atomics, a fixed order).
//   k_cost_finish    per pose: binary64 sum of the partials in tile order.
//   k_gen_backward   binary64 sum of the table partials, then the chain rule
//                    through the reflection (Eq. 8) and the centroid
//                    (Algorithm 3) to the footprint vertices, one lane per
//                    edge.  The path
//                    through p_0 cancels in exact arithmetic (d_i depends on
//                    the edge line only); its float residual is reported.
#include "device.hpp"
#include "kernels.hpp"

using namespace pipdev;

namespace {

constexpr int kTile = kBlock * kPPL;  // 1024 points per workgroup
constexpr int kPG = 64;               // poses per workgroup
constexpr int kCostMaxEdges = kMaxEdges;  // footprint size limit of the cost path

struct CostTab {
    float4 line[kMaxEdges];  // (-n_x, -n_y, k, |h|)
    float4 pair[kMaxEdges / 2];  // antipodal pairs: (n_x, n_y, -(k_i - k_j) / 2, (k_i + k_j) / 2)
    float2 g0;
    int n, n4, status;
    float rad;  // largest vertex distance from p_0, rounded up (the footprint's disk)
    int npair;  // > 0: the footprint is centrally symmetric (edges i, i + n/2 antiparallel)
};

__global__ __launch_bounds__(kWave) void k_cost_prepare(const float* __restrict__ F, int n,
                                                      CostTab* __restrict__ tab) {
    __shared__ PolyLds S;
    const int lane = threadIdx.x;
    if (lane < n) S.vtx[lane] = make_double2((double)F[2 * lane], (double)F[2 * lane + 1]);
    if (lane == 0) S.n = n;
    __syncthreads();
    prepare_polygon(S, K_VORONOI, lane);
    __syncthreads();
    const int i = lane < n ? lane : 0;
    const double2 g0 = S.gen[0], gi = S.gen[1 + i];
    const double hx = gi.x - g0.x, hy = gi.y - g0.y;
    const double L = sqrt(hx * hx + hy * hy);
    const double nx = hx / L, ny = hy / L;
    const double k = (nx * g0.x + ny * g0.y) + 0.5 * L;
    tab->line[lane] = make_float4((float)(-nx), (float)(-ny), (float)k, (float)L);
    double dv = 0.0;
    if (lane < n) {
        const double dx = S.vtx[lane].x - g0.x, dy = S.vtx[lane].y - g0.y;
        dv = sqrt(dx * dx + dy * dy);
    }
    const double rmax = wave_max(dv);
    // Antipodal pairs: for a centrally symmetric footprint edge j = i + n/2
    // has n_j = -n_i, so d_i = h - t and d_j = h + t with
    // t = n_i.p - (k_i - k_j)/2, h = (k_i + k_j)/2: min(d_i, d_j) = h - |t|,
    // reached at edge i when t >= 0 (the lower index on a tie).  Used when
    // the normals cancel to 2^-20; the remaining asymmetry changes a distance
    // by at most 2^-20 |p| against the cost's 1e-4 relative tolerance.
    int npair = 0;
    if ((n & 1) == 0) {
        const int hn = n >> 1;
        const int q = lane < hn ? lane : 0;
        auto edge = [&](int e, double& ex, double& ey, double& ek) {
            const double gx = S.gen[1 + e].x - g0.x, gy = S.gen[1 + e].y - g0.y;
            const double l = sqrt(gx * gx + gy * gy);
            ex = gx / l;
            ey = gy / l;
            ek = (ex * g0.x + ey * g0.y) + 0.5 * l;
        };
        double ax, ay, ak, bx, by, bk;
        edge(q, ax, ay, ak);
        edge(q + hn, bx, by, bk);
        const double asym = wave_max(fmax(fabs(ax + bx), fabs(ay + by)));
        if (lane < hn)
            tab->pair[lane] = make_float4((float)(0.5 * (ax - bx)), (float)(0.5 * (ay - by)),
                                          (float)(-0.5 * (ak - bk)), (float)(0.5 * (ak + bk)));
        if (asym <= 9.5367431640625e-07 && S.status == 0) npair = hn;  // 2^-20
    }
    if (lane == 0) {
        tab->npair = npair;
        tab->rad = round_up_f32(rmax * (1.0 + 1.0 / 65536.0) + 1e-30);  // NaN -> +inf
        tab->g0 = make_float2((float)g0.x, (float)g0.y);
        tab->n = n;
        tab->n4 = (n + 3) & ~3;
        tab->status = S.status;
    }
}

struct PoseCS {
    float c, s, tx, ty;
    float wx, wy;  // world position of p_0 (centre of the footprint's disk)
};

__global__ void k_fill_zero(float* __restrict__ p, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0.f;
}

__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// grid: x = point tiles, y = pose groups of kPG.  CULL: a (pose, wave) pair
// whose footprint disk misses the wave's points contributes exactly zero
// (no point inside, relu of a non-positive minimum) and is skipped.
template <bool BWD, bool CULL, bool PAIR>
__global__ __launch_bounds__(kBlock) void k_cost(const CostTab* __restrict__ tab,
                                               const float* __restrict__ pose, int64_t K,
                                               const float2* __restrict__ Q, int64_t m,
                                               const float* __restrict__ grad_cost,
                                               float* __restrict__ part_cost,
                                               float* __restrict__ part_pose,
                                               float* __restrict__ part_gen, int T) {
    __shared__ float4 line_s[kMaxEdges];
    __shared__ float4 pair_s[kMaxEdges / 2];
    __shared__ PoseCS pose_s[kPG];
    __shared__ float red_s[kPG][kWavesPerBlock][3];
    // backward only: table partials of each wave, 2(n+1) components (p_0,
    // then p_i), each added by lane 0 of its wave in pose order
    __shared__ float accw[kWavesPerBlock][2 * (kMaxEdges + 1)];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int n = tab->n, n4 = tab->n4;
    const float2 g0 = tab->g0;
    const int64_t k0 = (int64_t)blockIdx.y * kPG;
    const int pg = (int)((K - k0) < kPG ? (K - k0) : kPG);
    const int t = blockIdx.x;

    if (tid < n4) line_s[tid] = tab->line[tid];
    const int np = PAIR ? tab->npair : 0;
    if (PAIR && tid < np) pair_s[tid] = tab->pair[tid];
    if (tid < pg) {
        const float* pp = pose + 3 * (k0 + tid);
        const double th = (double)pp[2];
        PoseCS P;
        P.c = (float)cos(th);
        P.s = (float)sin(th);
        P.tx = pp[0];
        P.ty = pp[1];
        P.wx = P.tx + (P.c * g0.x - P.s * g0.y);
        P.wy = P.ty + (P.s * g0.x + P.c * g0.y);
        pose_s[tid] = P;
    }
    const int ncomp = 2 * (n + 1);
    if constexpr (BWD) {
        for (int i = tid; i < kWavesPerBlock * 2 * (kMaxEdges + 1); i += kBlock)
            (&accw[0][0])[i] = 0.f;
    }
    const int64_t base = (int64_t)t * kTile + (int64_t)wv * kChunk;
    float x[kPPL], y[kPPL];
    bool valid[kPPL];
#pragma unroll
    for (int j = 0; j < kPPL; ++j) {
        const int64_t i = base + lane + kWave * j;
        valid[j] = i < m;
        const float2 p = Q[valid[j] ? i : 0];
        x[j] = p.x;
        y[j] = p.y;
        valid[j] = valid[j] && isfinite(p.x) && isfinite(p.y);  // contributes nothing otherwise
    }
    // box, distance range from the origin and coordinate scale of the wave's points
    float xlo = __builtin_huge_valf(), xhi = -__builtin_huge_valf();
    float ylo = __builtin_huge_valf(), yhi = -__builtin_huge_valf();
    float r2lo = __builtin_huge_valf(), r2hi = 0.f, amax = 0.f;
    if constexpr (CULL) {
#pragma unroll
        for (int j = 0; j < kPPL; ++j) {
            if (valid[j]) {
                xlo = fminf(xlo, x[j]);
                xhi = fmaxf(xhi, x[j]);
                ylo = fminf(ylo, y[j]);
                yhi = fmaxf(yhi, y[j]);
                const float r2 = fmaf(x[j], x[j], y[j] * y[j]);
                r2lo = fminf(r2lo, r2);
                r2hi = fmaxf(r2hi, r2);
                amax = fmaxf(amax, fmaxf(fabsf(x[j]), fabsf(y[j])));
            }
        }
        xlo = -wave_max_f(-xlo);
        xhi = wave_max_f(xhi);
        ylo = -wave_max_f(-ylo);
        yhi = wave_max_f(yhi);
        r2lo = -wave_max_f(-r2lo);
        r2hi = wave_max_f(r2hi);
        amax = wave_max_f(amax);
    }
    __syncthreads();

    for (int p = 0; p < pg; ++p) {
        const PoseCS P = pose_s[p];
        if constexpr (CULL) {
            // The footprint lies in the disk (p_0 world position, rad).  A
            // point the float32 evaluation counts inside is within a few ulps
            // of the footprint, far less than the slack 2^-12 x (coordinate
            // scale + disk), so a disk that misses the wave's box or distance
            // range (widened by the slack) means every term is exactly zero.
            const float R = tab->rad;
            const float Rs =
                R + (fabsf(P.wx) + fabsf(P.wy) + fabsf(P.tx) + fabsf(P.ty) + amax + R) *
                        (1.0f / 4096.0f);
            bool skip = P.wx + Rs < xlo || P.wx - Rs > xhi || P.wy + Rs < ylo || P.wy - Rs > yhi;
            const float dc = sqrtf(fmaf(P.wx, P.wx, P.wy * P.wy));
            const float hi = dc + Rs, lo = dc - Rs;
            const float sl = 1.0f / 65536.0f;
            skip = skip || hi * hi * (1.0f + sl) < r2lo * (1.0f - sl);
            skip = skip || (lo > 0.f && lo * lo * (1.0f - sl) > r2hi * (1.0f + sl));
            skip = skip && R < __builtin_huge_valf() && P.wx == P.wx && P.wy == P.wy;
            if (skip) {
                if (lane == 0) {
                    red_s[p][wv][0] = 0.f;
                    if constexpr (BWD) {
                        red_s[p][wv][1] = 0.f;
                        red_s[p][wv][2] = 0.f;
                    }
                }
                continue;
            }
        }
        float bx[kPPL], by[kPPL], dmin[kPPL];
        int arg[kPPL];
#pragma unroll
        for (int j = 0; j < kPPL; ++j) {
            const float dx = x[j] - P.tx, dy = y[j] - P.ty;
            bx[j] = fmaf(P.c, dx, P.s * dy);
            by[j] = fmaf(P.c, dy, -(P.s * dx));
            dmin[j] = __builtin_huge_valf();
            arg[j] = 0;
        }
        if (PAIR && np > 0) {
            for (int q = 0; q < np; ++q) {
                const float4 L = pair_s[q];
#pragma unroll
                for (int j = 0; j < kPPL; ++j) {
                    const float tq = fmaf(L.x, bx[j], fmaf(L.y, by[j], L.z));
                    const float d = L.w - fabsf(tq);
                    if constexpr (BWD) {
                        if (d < dmin[j]) {
                            dmin[j] = d;
                            arg[j] = tq < 0.f ? q + np : q;
                        }
                    } else {
                        dmin[j] = fminf(dmin[j], d);
                    }
                }
            }
        } else {
            for (int e = 0; e < n; ++e) {
                const float4 L = line_s[e];
#pragma unroll
                for (int j = 0; j < kPPL; ++j) {
                    const float d = fmaf(L.x, bx[j], fmaf(L.y, by[j], L.z));
                    if constexpr (BWD) {
                        if (d < dmin[j]) {
                            dmin[j] = d;
                            arg[j] = e;
                        }
                    } else {
                        dmin[j] = fminf(dmin[j], d);
                    }
                }
            }
        }
        if constexpr (!BWD) {
            float sum = 0.f;
#pragma unroll
            for (int j = 0; j < kPPL; ++j) sum += (valid[j] && dmin[j] > 0.f) ? dmin[j] : 0.f;
            sum = wave_sum(sum);
            if (lane == 0) red_s[p][wv][0] = sum;
        } else {
            const float w = grad_cost[k0 + p];
            float sx = 0.f, sy = 0.f, sth = 0.f, s0x = 0.f, s0y = 0.f;
            float ghx[kPPL], ghy[kPPL];
            uint64_t emask = 0;  // edges this lane's points press on
#pragma unroll
            for (int j = 0; j < kPPL; ++j) {
                ghx[j] = 0.f;
                ghy[j] = 0.f;
                if (valid[j] && dmin[j] > 0.f) {
                    const float4 L = line_s[arg[j]];
                    const float nx = -L.x, ny = -L.y, len = L.w;
                    sx += nx;
                    sy += ny;
                    sth += fmaf(-nx, by[j], ny * bx[j]);
                    // derivatives of d = |h|/2 - u.h/|h| (u = p_b - p_0) to h and p_0
                    const float ux = bx[j] - g0.x, uy = by[j] - g0.y;
                    const float un = fmaf(ux, nx, uy * ny);
                    const float dhx = 0.5f * nx - (ux - un * nx) / len;
                    const float dhy = 0.5f * ny - (uy - un * ny) / len;
                    ghx[j] = w * dhx;
                    ghy[j] = w * dhy;
                    s0x += w * (nx - dhx);
                    s0y += w * (ny - dhy);
                    emask |= 1ull << arg[j];
                }
            }
            sx = wave_sum(sx);
            sy = wave_sum(sy);
            sth = wave_sum(sth);
            if (lane == 0) {
                red_s[p][wv][0] = sx;
                red_s[p][wv][1] = sy;
                red_s[p][wv][2] = sth;
            }
            // table partials: p_0, then one wave sum per edge pressed on
            // (in increasing edge order), added by lane 0 in pose order
            if (__ballot(emask != 0)) {  // some point of the wave presses on the footprint
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) emask |= __shfl_xor(emask, o, kWave);
                emask = ((uint64_t)__builtin_amdgcn_readfirstlane((int)(emask >> 32)) << 32) |
                        (uint32_t)__builtin_amdgcn_readfirstlane((int)emask);
                s0x = wave_sum(s0x);
                s0y = wave_sum(s0y);
                if (lane == 0) {
                    accw[wv][0] += s0x;
                    accw[wv][1] += s0y;
                }
                while (emask) {
                    const int e = __builtin_ctzll(emask);
                    emask &= emask - 1;
                    float ex = 0.f, ey = 0.f;
#pragma unroll
                    for (int j = 0; j < kPPL; ++j) {
                        if (arg[j] == e) {  // 0 unless the point contributes
                            ex += ghx[j];
                            ey += ghy[j];
                        }
                    }
                    ex = wave_sum(ex);
                    ey = wave_sum(ey);
                    if (lane == 0) {
                        accw[wv][2 * (1 + e)] += ex;
                        accw[wv][2 * (1 + e) + 1] += ey;
                    }
                }
            }
        }
    }
    __syncthreads();
    // per-(pose, tile) partials, waves summed in a fixed order
    if constexpr (!BWD) {
        if (tid < pg) {
            float s = red_s[tid][0][0];
            for (int q = 1; q < kWavesPerBlock; ++q) s += red_s[tid][q][0];
            part_cost[(k0 + tid) * T + t] = s;
        }
    } else {
        if (tid < pg) {
            for (int c = 0; c < 3; ++c) {
                float s = red_s[tid][0][c];
                for (int q = 1; q < kWavesPerBlock; ++q) s += red_s[tid][q][c];
                part_pose[((k0 + tid) * T + t) * 3 + c] = s;
            }
        }
        // table partials of this workgroup: waves in a fixed order
        for (int c = tid; c < ncomp; c += kBlock) {
            float s = accw[0][c];
            for (int q = 1; q < kWavesPerBlock; ++q) s += accw[q][c];
            part_gen[((int64_t)blockIdx.y * T + t) * (2 * (kMaxEdges + 1)) + c] = s;
        }
    }
}

__global__ void k_cost_finish(const float* __restrict__ part_cost, int64_t K, int T,
                              float* __restrict__ cost) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    double s = 0.0;
    for (int t = 0; t < T; ++t) s += (double)part_cost[k * T + t];
    cost[k] = (float)s;
}

__global__ void k_pose_grad_finish(const float* __restrict__ part_pose, const float* __restrict__ pose,
                                   const float* __restrict__ grad_cost, int64_t K, int T,
                                   float* __restrict__ grad_pose) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    double sx = 0.0, sy = 0.0, st = 0.0;
    for (int t = 0; t < T; ++t) {
        sx += (double)part_pose[(k * T + t) * 3 + 0];
        sy += (double)part_pose[(k * T + t) * 3 + 1];
        st += (double)part_pose[(k * T + t) * 3 + 2];
    }
    const double th = (double)pose[3 * k + 2];
    const double c = (double)(float)cos(th), s = (double)(float)sin(th);
    const double w = (double)grad_cost[k];
    grad_pose[3 * k + 0] = (float)(w * (c * sx - s * sy));  // R n summed
    grad_pose[3 * k + 1] = (float)(w * (s * sx + c * sy));
    grad_pose[3 * k + 2] = (float)(w * st);
}

// Stage 1 of the table-gradient reduction: block b sums, in binary64 and in
// part order, its contiguous range of per-workgroup partials (thread c owns
// component c).
constexpr int kGenRedBlocks = 256;

__global__ __launch_bounds__(256) void k_gen_reduce1(const float* __restrict__ part_gen, int64_t nparts,
                                                   int ncomp, double* __restrict__ stage) {
    constexpr int NC = 2 * (kMaxEdges + 1);
    const int64_t per = (nparts + kGenRedBlocks - 1) / kGenRedBlocks;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < nparts ? lo + per : nparts;
    for (int c = threadIdx.x; c < ncomp; c += 256) {
        double s = 0.0;
        for (int64_t i = lo; i < hi; ++i) s += (double)part_gen[i * NC + c];
        stage[(int64_t)blockIdx.x * NC + c] = s;
    }
}

// Stage 2 (one wave): sums of the stage-1 results in block order, then the
// chain rule to the vertices, lane i taking edge i (its reflection, Eq. 8,
// and its share of the centroid, Algorithm 3); each vertex collects the
// terms of its two edges, and the path through p_0 is summed in edge order.
// residual (optional, [2]): |total gradient to p_0| and the scale it is
// measured against.
__global__ __launch_bounds__(kWave) void k_gen_backward(const float* __restrict__ F, int n,
                                                      const double* __restrict__ stage,
                                                      float* __restrict__ grad_F,
                                                      float* __restrict__ residual) {
    constexpr int NC = 2 * (kMaxEdges + 1);
    __shared__ double G[NC];
    __shared__ double vx[kMaxEdges], vy[kMaxEdges];
    __shared__ double tb[kMaxEdges][2], ta[kMaxEdges][2];  // terms to v_i and to v_{i-1}
    __shared__ double gg0[kMaxEdges][3];                    // edge i's terms to p_0, scale
    const int lane = threadIdx.x;
    const int ncomp = 2 * (n + 1);
    for (int c = lane; c < ncomp; c += kWave) {
        double s = 0.0;
        for (int b = 0; b < kGenRedBlocks; ++b) s += stage[b * NC + c];
        G[c] = s;
    }
    if (lane < n) {
        vx[lane] = (double)F[2 * lane];
        vy[lane] = (double)F[2 * lane + 1];
    }
    __syncthreads();
    // forward quantities in binary64 (Algorithms 3-4, same order as the
    // preparation kernel; every lane forms the same sums)
    double S = 0.0, Sx = 0.0, Sy = 0.0;
    for (int i = 0; i < n; ++i) {
        const int j = prev_edge(i, n);
        const double Ai = vx[j] * vy[i] - vx[i] * vy[j];
        S = S + Ai;
        Sx = Sx + (vx[i] + vx[j]) * Ai;
        Sy = Sy + (vy[i] + vy[j]) * Ai;
    }
    const double g0x = Sx / (3.0 * S), g0y = Sy / (3.0 * S);
    // reflections: g = (W g0 - 2 c [a; b]) / (a^2 + b^2), edge v_{i-1} -> v_i
    if (lane < n) {
        const int i = lane, j = prev_edge(i, n);
        const double bx = vx[i], by = vy[i], ax = vx[j], ay = vy[j];
        const double ea = by - ay, eb = ax - bx;
        const double ec = -(ea * bx + eb * by);
        const double den = ea * ea + eb * eb;
        const double w11 = eb * eb - ea * ea, w12 = -2.0 * ea * eb, w22 = ea * ea - eb * eb;
        const double Nx = w11 * g0x + w12 * g0y - 2.0 * ec * ea;
        const double Ny = w12 * g0x + w22 * g0y - 2.0 * ec * eb;
        const double Gx = G[2 * (1 + i)], Gy = G[2 * (1 + i) + 1];
        const double GNx = Gx / den, GNy = Gy / den;
        const double Gden = -(Gx * Nx + Gy * Ny) / (den * den);
        double Gea = 2.0 * ea * Gden, Geb = 2.0 * eb * Gden;
        Gea += GNx * (-2.0 * ea * g0x - 2.0 * eb * g0y - 2.0 * ec) + GNy * (-2.0 * eb * g0x + 2.0 * ea * g0y);
        Geb += GNx * (2.0 * eb * g0x - 2.0 * ea * g0y) + GNy * (-2.0 * ea * g0x - 2.0 * eb * g0y - 2.0 * ec);
        const double Gec = GNx * (-2.0 * ea) + GNy * (-2.0 * eb);
        gg0[i][0] = w11 * GNx + w12 * GNy;
        gg0[i][1] = w12 * GNx + w22 * GNy;
        gg0[i][2] = fabs(Gx) + fabs(Gy);
        // ec = -(ea bx + eb by); ea = by - ay, eb = ax - bx
        Gea += -bx * Gec;
        Geb += -by * Gec;
        tb[i][0] = -ea * Gec - Geb;  // to v_i
        tb[i][1] = -eb * Gec + Gea;
        ta[i][0] = Geb;              // to v_{i-1}
        ta[i][1] = -Gea;
    }
    __syncthreads();
    // path through p_0, summed in edge order (every lane the same)
    double Gg0x = G[0], Gg0y = G[1];
    double scale = fabs(G[0]) + fabs(G[1]);
    for (int i = 0; i < n; ++i) {
        Gg0x += gg0[i][0];
        Gg0y += gg0[i][1];
        scale += gg0[i][2];
    }
    // centroid: g0 = (Sx, Sy) / (3 S), edge i's partial area A_i
    const double GSx = Gg0x / (3.0 * S), GSy = Gg0y / (3.0 * S);
    const double GS = -(Gg0x * Sx + Gg0y * Sy) / (3.0 * S * S);
    double cb0 = 0.0, cb1 = 0.0, ca0 = 0.0, ca1 = 0.0;
    if (lane < n) {
        const int i = lane, j = prev_edge(i, n);
        const double Ai = vx[j] * vy[i] - vx[i] * vy[j];
        const double GA = GS + GSx * (vx[i] + vx[j]) + GSy * (vy[i] + vy[j]);
        cb0 = GSx * Ai - GA * vy[j];  // to v_i
        cb1 = GSy * Ai + GA * vx[j];
        ca0 = GSx * Ai + GA * vy[i];  // to v_{i-1}
        ca1 = GSy * Ai - GA * vx[i];
    }
    __syncthreads();
    if (lane < n) {
        ta[lane][0] += ca0;
        ta[lane][1] += ca1;
        tb[lane][0] += cb0;
        tb[lane][1] += cb1;
    }
    __syncthreads();
    if (lane < n) {  // vertex v: its edge v (as v_i) and edge v + 1 (as v_{i-1})
        const int nx = lane + 1 < n ? lane + 1 : 0;
        grad_F[2 * lane] = (float)(tb[lane][0] + ta[nx][0]);
        grad_F[2 * lane + 1] = (float)(tb[lane][1] + ta[nx][1]);
    }
    if (residual && lane == 0) {
        residual[0] = (float)sqrt(Gg0x * Gg0x + Gg0y * Gg0y);
        residual[1] = (float)scale;
    }
}

}  // namespace

namespace pipdev {

int cost_max_edges() { return kCostMaxEdges; }

size_t cost_workspace_layout(int n, int64_t K, int64_t m, CostLayout* L) {
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    (void)n;
    const int64_t T = (m + kTile - 1) / kTile;
    const int64_t G = (K + kPG - 1) / kPG;
    size_t off = 0;
    L->tab = off;
    off = up(off + sizeof(CostTab));
    L->part_cost = off;
    off = up(off + 4 * (size_t)(K * (T > 0 ? T : 1)));
    L->part_pose = off;
    off = up(off + 12 * (size_t)(K * (T > 0 ? T : 1)));
    L->part_gen = off;
    off = up(off + 4 * (size_t)(G * (T > 0 ? T : 1)) * 2 * (kMaxEdges + 1));
    L->stage = off;
    off = up(off + 8 * (size_t)kGenRedBlocks * 2 * (kMaxEdges + 1));
    L->T = (int)T;
    L->G = G;
    return off;
}

hipError_t launch_cost(bool backward, const float* F, int n, const float* pose, int64_t K,
                       const float* Q, int64_t m, const float* grad_cost, float* cost,
                       float* grad_pose, float* grad_F, float* residual, void* ws, int cull,
                       int pair, hipStream_t stream) {
    CostLayout L;
    cost_workspace_layout(n, K, m, &L);
    char* b = static_cast<char*>(ws);
    CostTab* tab = reinterpret_cast<CostTab*>(b + L.tab);
    float* pc = reinterpret_cast<float*>(b + L.part_cost);
    float* pp = reinterpret_cast<float*>(b + L.part_pose);
    float* pgn = reinterpret_cast<float*>(b + L.part_gen);
    hipLaunchKernelGGL(k_cost_prepare, dim3(1), dim3(kWave), 0, stream, F, n, tab);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int T = L.T > 0 ? L.T : 1;
    if (L.T > 0 && K > 0) {
        dim3 grid((unsigned)L.T, (unsigned)L.G);
        const float2* Q2 = reinterpret_cast<const float2*>(Q);
        auto kern = backward ? (cull ? (pair ? k_cost<true, true, true> : k_cost<true, true, false>)
                                     : (pair ? k_cost<true, false, true> : k_cost<true, false, false>))
                             : (cull ? (pair ? k_cost<false, true, true> : k_cost<false, true, false>)
                                     : (pair ? k_cost<false, false, true> : k_cost<false, false, false>));
        hipLaunchKernelGGL(kern, grid, dim3(kBlock), 0, stream, tab, pose, K, Q2,
                           m, grad_cost, pc, pp, pgn, T);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else {
        // no points: every partial is zero (a fill kernel, safe under graph capture)
        const int64_t nf = backward ? (int64_t)L.G * T * 2 * (kMaxEdges + 1) : (int64_t)K * T;
        if (nf > 0)
            hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, stream,
                               backward ? pgn : pc, nf);
        if (backward && K > 0)
            hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((K * T * 3 + 255) / 256)), dim3(256), 0,
                               stream, pp, K * T * 3);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const unsigned kb = (unsigned)((K + 255) / 256);
    if (!backward) {
        if (K > 0) hipLaunchKernelGGL(k_cost_finish, dim3(kb), dim3(256), 0, stream, pc, K, T, cost);
    } else {
        if (K > 0)
            hipLaunchKernelGGL(k_pose_grad_finish, dim3(kb), dim3(256), 0, stream, pp, pose, grad_cost,
                               K, T, grad_pose);
        double* stage = reinterpret_cast<double*>(b + L.stage);
        hipLaunchKernelGGL(k_gen_reduce1, dim3(kGenRedBlocks), dim3(256), 0, stream, pgn,
                           (int64_t)L.G * T, 2 * (n + 1), stage);
        hipLaunchKernelGGL(k_gen_backward, dim3(1), dim3(64), 0, stream, F, n, stage, grad_F,
                           residual);
    }
    return hipGetLastError();
}

}  // namespace pipdev
