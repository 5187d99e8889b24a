// Convex decomposition of a simple polygon (host code), for the union-of-
// pieces test of non-convex polygons (the extension Section 7 names).
//
// Ear clipping triangulates the polygon with exact orientation signs; then
// every diagonal whose removal leaves a convex piece (strictly convex at both
// of its ends) of at most max_piece_vertices vertices is removed, greedily
// in the order the triangles were cut (Hertel and Mehlhorn's rule: at most
// four times the minimum number of convex pieces).  Pieces list vertex
// indices of the polygon in the polygon's own cyclic order.
//
// Orientation signs are exact: a binary64 evaluation with an error bound
// decides most cases; otherwise the determinant is summed exactly as a
// floating-point expansion (exact products by fma, then error-free sums,
// Shewchuk's expansion arithmetic) and its sign is that of the largest
// component.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <unordered_map>
#include <vector>

#include "kernels.hpp"

namespace {

void two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// h = e + b for an expansion e of n nonoverlapping components in increasing
// magnitude; zero components are dropped.  Returns the length of h.
int grow_expansion(const double* e, int n, double b, double* h) {
    double q = b;
    int k = 0;
    for (int i = 0; i < n; ++i) {
        double s, t;
        two_sum(q, e[i], s, t);
        if (t != 0.0) h[k++] = t;
        q = s;
    }
    if (q != 0.0 || k == 0) h[k++] = q;
    return k;
}

// Sign of (b - a) x (c - a): +1 counter-clockwise, -1 clockwise, 0 collinear.
int orient_sign(const double* a, const double* b, const double* c) {
    const double l = (b[0] - a[0]) * (c[1] - a[1]);
    const double r = (b[1] - a[1]) * (c[0] - a[0]);
    const double det = l - r;
    const double bound = 1.0e-15 * (std::fabs(l) + std::fabs(r));
    if (det > bound) return 1;
    if (-det > bound) return -1;
    // exact: a_x b_y - a_y b_x + b_x c_y - b_y c_x + c_x a_y - c_y a_x
    const double t[6][2] = {{a[0], b[1]}, {-a[1], b[0]}, {b[0], c[1]},
                            {-b[1], c[0]}, {c[0], a[1]}, {-c[1], a[0]}};
    double e[32], h[32];
    int n = 0;
    for (int i = 0; i < 6; ++i) {
        const double p = t[i][0] * t[i][1];
        const double err = std::fma(t[i][0], t[i][1], -p);
        n = grow_expansion(e, n, p, h);
        std::memcpy(e, h, sizeof(double) * n);
        n = grow_expansion(e, n, err, h);
        std::memcpy(e, h, sizeof(double) * n);
    }
    const double top = e[n - 1];
    return top > 0.0 ? 1 : (top < 0.0 ? -1 : 0);
}

struct Ring {
    std::vector<int> prev, next;
    std::vector<char> alive;
};

}  // namespace

namespace pipdev {

// 0 on success; 1 bad input (non-finite, zero area); 2 not simple (no ear);
// 3 capacity exceeded.  off gets K+1 entries, idx the piece vertices.
int convex_decompose_host(const double* V, int n, int max_piece, std::vector<int32_t>& off,
                          std::vector<int32_t>& idx) {
    off.clear();
    idx.clear();
    for (int i = 0; i < 2 * n; ++i)
        if (!std::isfinite(V[i])) return 1;
    double area2 = 0.0;
    for (int i = 0; i < n; ++i) {
        const int j = i == 0 ? n - 1 : i - 1;
        area2 += V[2 * j] * V[2 * i + 1] - V[2 * i] * V[2 * j + 1];
    }
    if (!(area2 != 0.0) || !std::isfinite(area2)) return 1;
    const int s = area2 > 0.0 ? 1 : -1;
    auto P = [&](int i) { return V + 2 * i; };

    // --- ear clipping ---------------------------------------------------
    Ring R;
    R.prev.resize(n);
    R.next.resize(n);
    R.alive.assign(n, 1);
    for (int i = 0; i < n; ++i) {
        R.prev[i] = i == 0 ? n - 1 : i - 1;
        R.next[i] = i + 1 == n ? 0 : i + 1;
    }
    std::vector<int> reflex;  // candidates that can block an ear (non-convex vertices)
    auto is_convex = [&](int i) { return s * orient_sign(P(R.prev[i]), P(i), P(R.next[i])) > 0; };
    auto refresh_reflex = [&]() {
        reflex.clear();
        for (int i = 0; i < n; ++i)
            if (R.alive[i] && !is_convex(i)) reflex.push_back(i);
    };
    refresh_reflex();
    auto is_ear = [&](int i) {
        const int a = R.prev[i], c = R.next[i];
        if (!is_convex(i)) return false;
        for (int p : reflex) {
            if (!R.alive[p] || p == a || p == i || p == c) continue;
            if (s * orient_sign(P(a), P(i), P(p)) >= 0 && s * orient_sign(P(i), P(c), P(p)) >= 0 &&
                s * orient_sign(P(c), P(a), P(p)) >= 0)
                return false;
        }
        return true;
    };
    std::vector<int32_t> tris;
    tris.reserve(3 * (size_t)n);
    int left = n, cur = 0, since = 0;
    while (left > 3) {
        if (since > left) return 2;  // a full turn without an ear
        const int a = R.prev[cur], c = R.next[cur];
        const int o = orient_sign(P(a), P(cur), P(c));
        bool cut = false;
        if (o == 0) {
            // collinear with both neighbours: between them it lies on the
            // remaining chain's edge a-c and is dropped; a spike is not simple
            const double* pa = P(a);
            const double* pb = P(cur);
            const double* pc = P(c);
            const double dot = (pb[0] - pa[0]) * (pc[0] - pb[0]) + (pb[1] - pa[1]) * (pc[1] - pb[1]);
            if (!(dot > 0.0)) return 2;
            cut = true;
        } else if (is_ear(cur)) {
            tris.push_back(a);
            tris.push_back(cur);
            tris.push_back(c);
            cut = true;
        }
        if (cut) {
            R.alive[cur] = 0;
            R.next[a] = c;
            R.prev[c] = a;
            --left;
            since = 0;
            // a neighbour may have turned convex; reflex candidates only shrink
            if (!reflex.empty()) {
                size_t w = 0;
                for (size_t t = 0; t < reflex.size(); ++t) {
                    const int p = reflex[t];
                    if (R.alive[p] && !is_convex(p)) reflex[w++] = p;
                }
                reflex.resize(w);
            }
            cur = c;
        } else {
            cur = c;
            ++since;
        }
    }
    {
        const int a = R.prev[cur], c = R.next[cur];
        if (orient_sign(P(a), P(cur), P(c)) != 0) {
            tris.push_back(a);
            tris.push_back(cur);
            tris.push_back(c);
        }
    }
    const int T = (int)(tris.size() / 3);
    if (T == 0) return 1;

    // --- greedy merge across diagonals -----------------------------------
    std::vector<std::vector<int>> piece(T);
    std::vector<int> root(T);
    for (int t = 0; t < T; ++t) {
        piece[t] = {tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
        root[t] = t;
    }
    auto find = [&](int t) {
        while (root[t] != t) t = root[t] = root[root[t]];
        return t;
    };
    std::unordered_map<uint64_t, int> edge_tri;  // directed edge u->v -> triangle
    auto key = [](int u, int v) { return ((uint64_t)(uint32_t)u << 32) | (uint32_t)v; };
    for (int t = 0; t < T; ++t)
        for (int q = 0; q < 3; ++q) edge_tri[key(tris[3 * t + q], tris[3 * t + (q + 1) % 3])] = t;
    auto pos = [](const std::vector<int>& p, int v) {
        for (size_t i = 0; i < p.size(); ++i)
            if (p[i] == v) return (int)i;
        return -1;
    };
    for (int t = 0; t < T; ++t) {
        for (int q = 0; q < 3; ++q) {
            const int u = tris[3 * t + q], v = tris[3 * t + (q + 1) % 3];
            auto it = edge_tri.find(key(v, u));
            if (it == edge_tri.end() || it->second < t) continue;  // boundary, or seen
            const int A = find(t), B = find(it->second);
            if (A == B) continue;
            std::vector<int>& pa = piece[A];
            std::vector<int>& pb = piece[B];
            if ((int)(pa.size() + pb.size()) - 2 > max_piece) continue;
            const int iu = pos(pa, u), iv = pos(pa, v), ju = pos(pb, u), jv = pos(pb, v);
            if (iu < 0 || iv < 0 || ju < 0 || jv < 0) continue;
            const int na = (int)pa.size(), nb = (int)pb.size();
            if ((iu + 1) % na != iv || (jv + 1) % nb != ju) continue;  // not the shared edge
            const int pred_u = pa[(iu + na - 1) % na], succ_u = pb[(ju + 1) % nb];
            const int pred_v = pb[(jv + nb - 1) % nb], succ_v = pa[(iv + 1) % na];
            if (s * orient_sign(P(pred_u), P(u), P(succ_u)) <= 0) continue;
            if (s * orient_sign(P(pred_v), P(v), P(succ_v)) <= 0) continue;
            std::vector<int> m;
            m.reserve(na + nb - 2);
            for (int k = 0; k < na; ++k) m.push_back(pa[(iv + k) % na]);       // v .. u
            for (int k = 1; k + 1 < nb; ++k) m.push_back(pb[(ju + k) % nb]);  // after u .. before v
            pa.swap(m);
            pb.clear();
            root[B] = A;
        }
    }
    off.push_back(0);
    for (int t = 0; t < T; ++t) {
        if (find(t) != t) continue;
        for (int v : piece[t]) idx.push_back(v);
        off.push_back((int32_t)idx.size());
    }
    return 0;
}

}  // namespace pipdev
