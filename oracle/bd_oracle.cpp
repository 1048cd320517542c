// =============================================================================
// CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
//
// A plain, sequential, FP64 reference for one time step of the Brownian
// hard-disk method of Carter, Hitschfeld, Navarro and Soto, "GPU parallel
// simulation algorithm of Brownian particles with excluded volume using
// Delaunay triangulations" (arXiv:1703.02484).  Only the test-suite, the smoke
// check and the benchmark's CPU-baseline leg may load this library; the GPU
// library never does.  It shares no source with the GPU path.
//
// Build: g++ -std=c++17 -O2 -ffp-contract=off (no fast-math), single thread.
//
// Readings of the paper that this file adopts where the paper is silent,
// ambiguous or garbled (each is restated where it is used):
//   * hard walls with mirror reflection instead of the paper's periodic box;
//   * translational noise amplitude sqrt(2 D dt) (mean-square displacement
//     4 D t in 2D), the rotational rule of Sec. 7 already carries the 2;
//   * general S x S strength matrix K[a][b] = strength on species a from b,
//     which is mu_a alpha_b in the paper's two-charge model (Sec. 2.2);
//   * overlap displacement along the unit vector (Sec. 2.3 equation), summed
//     Jacobi-style over all overlapping Delaunay edges (Sec. 4.4, Algorithm 2),
//     the per-particle sum truncated to length cap_frac * r_i (Sec. 4.4: the
//     sigma/4 heuristic, half a radius), rounds repeated until no Delaunay
//     edge overlaps (Sec. 4.4) with a round cap; "overlapping" means
//     d < (r_i + r_j)(1 - contact_tol): with the contact factor 1/2 a pair is
//     moved exactly to contact and rounding may leave it an ulp short, which a
//     bare strict test would keep correcting forever;
//   * the triangulation is recomputed from scratch (Bowyer-Watson) whenever
//     positions change, including after every overlap round: the Delaunay
//     triangulation is unique in general position, so this is the plain
//     definition that the GPU's flip rounds (Sec. 4.1, 4.3) reach faster;
//   * the triangulated point set is the disks plus a fixed frame of points
//     outside the walls (see wall_frame): the paper triangulates a periodic
//     box, which has no boundary; with walls, disks pressed against a wall are
//     nearly collinear and the bare Delaunay triangulation degenerates into
//     super-thin triangles along the walls, which the frame prevents.  No frame
//     point lies in the diametral circle of an overlapping pair, so the
//     closest overlapping pair is still a Delaunay edge;
//   * the inverted-triangle predicate of Sec. 4.3 is evaluated for both
//     orderings of the two opposite vertices (the printed formula tests the
//     wrong triangle and contradicts its own figure).
//
// Functions with no independent pin say "parity unpinned" in their comment.
// =============================================================================
#include <cmath>
#include <cstdint>
#include <cstring>
#include <unordered_map>
#include <vector>
#include <algorithm>

namespace {

// ----------------------------------------------------------------------------
// Philox4x32-10, written from Salmon, Moraes, Dror and Shaw, "Parallel random
// numbers: as easy as 1, 2, 3" (SC'11).  The paper itself draws XORWOW numbers
// from a closed library; a counter-based generator replaces it so that noise is
// a pure function of (seed, step, particle id, stream).
// ----------------------------------------------------------------------------
struct Words4 { uint32_t w[4]; };

Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
    const uint64_t MA = 0xD2511F53u, MB = 0xCD9E8D57u;      // round multipliers
    const uint32_t WA = 0x9E3779B9u, WB = 0xBB67AE85u;      // key schedule (Weyl) increments
    for (int round = 0; round < 10; ++round) {
        uint64_t pa = MA * (uint64_t)c0;
        uint64_t pb = MB * (uint64_t)c2;
        uint32_t hi_a = (uint32_t)(pa >> 32), lo_a = (uint32_t)pa;
        uint32_t hi_b = (uint32_t)(pb >> 32), lo_b = (uint32_t)pb;
        uint32_t n0 = hi_b ^ c1 ^ k0;
        uint32_t n1 = lo_b;
        uint32_t n2 = hi_a ^ c3 ^ k1;
        uint32_t n3 = lo_a;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += WA; k1 += WB;
    }
    Words4 r;
    r.w[0] = c0; r.w[1] = c1; r.w[2] = c2; r.w[3] = c3;
    return r;
}

// Two standard normals for (seed, step, id, stream) by Box and Muller (1958):
// u1 in (0,1] from words 0,1 and u2 in [0,1) from words 2,3, 53 bits each.
void normal_pair(uint64_t seed, int64_t step, uint32_t id, uint32_t stream, double &z0, double &z1) {
    uint64_t st = (uint64_t)step;
    Words4 w = philox4x32_10(id, (uint32_t)st, (uint32_t)(st >> 32), stream,
                             (uint32_t)seed, (uint32_t)(seed >> 32));
    uint64_t m1 = ((((uint64_t)w.w[0]) << 32) | w.w[1]) >> 11;
    uint64_t m2 = ((((uint64_t)w.w[2]) << 32) | w.w[3]) >> 11;
    double u1 = ((double)m1 + 1.0) * 0x1.0p-53;
    double u2 = (double)m2 * 0x1.0p-53;
    double rho = std::sqrt(-2.0 * std::log(u1));
    double ang = 2.0 * M_PI * u2;
    z0 = rho * std::cos(ang);
    z1 = rho * std::sin(ang);
}

// ----------------------------------------------------------------------------
// Geometric predicates, plain FP64 in translated form.
// ----------------------------------------------------------------------------
inline double orient2(double ax, double ay, double bx, double by, double cx, double cy) {
    // twice the signed area of (a, b, c); > 0 when counter-clockwise
    return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
}

inline double incircle(double ax, double ay, double bx, double by, double cx, double cy, double dx, double dy) {
    // > 0 when d lies strictly inside the circle through the CCW triangle (a, b, c)
    double adx = ax - dx, ady = ay - dy;
    double bdx = bx - dx, bdy = by - dy;
    double cdx = cx - dx, cdy = cy - dy;
    double alift = adx * adx + ady * ady;
    double blift = bdx * bdx + bdy * bdy;
    double clift = cdx * cdx + cdy * cdy;
    return alift * (bdx * cdy - cdx * bdy) - blift * (adx * cdy - cdx * ady) + clift * (adx * bdy - bdx * ady);
}

// Sec. 4.3: is point p inside the closed triangle (v1, v2, v3)?  Barycentric
// form: p - v1 = s (v2 - v1) + t (v3 - v1); inside when s, t >= 0 and s + t <= 1.
// The comparisons are multiplied through by the signed doubled area so that
// either orientation of the triangle is handled, as in the paper's two cases.
bool point_in_closed_triangle(const double *v1, const double *v2, const double *v3, const double *p) {
    double e0x = v2[0] - v1[0], e0y = v2[1] - v1[1];
    double e1x = v3[0] - v1[0], e1y = v3[1] - v1[1];
    double ex = p[0] - v1[0], ey = p[1] - v1[1];
    double area = e0x * e1y - e0y * e1x;          // (v2 - v1) x (v3 - v1)
    double s = ex * e1y - ey * e1x;               // (p - v1) x (v3 - v1)  = s * area
    double t = e0x * ey - e0y * ex;               // (v2 - v1) x (p - v1)  = t * area
    if (area < 0.0) return (s <= 0.0) && (t <= 0.0) && (s + t >= area);
    return (s >= 0.0) && (t >= 0.0) && (s + t <= area);
}

// Sec. 4.3 flip criterion for edge (v1, v2) whose opposite vertices are v3 and
// v4: flip when either opposite vertex lies in the closed triangle formed by
// the edge and the other opposite vertex.
bool inverted_edge_flip(const double *v1, const double *v2, const double *v3, const double *v4) {
    return point_in_closed_triangle(v1, v2, v3, v4) || point_in_closed_triangle(v1, v2, v4, v3);
}

// ----------------------------------------------------------------------------
// Delaunay triangulation by Bowyer-Watson insertion with an infinite vertex.
// A ghost triangle (u, v, INF) stands for the outside of hull edge v -> u; a
// point conflicts with it when it lies strictly outside that edge or on the
// open edge itself.  A finite triangle conflicts when the point is strictly
// inside its circumcircle.  Each insertion removes the connected set of
// conflicting triangles and joins the new point to the cavity boundary.
// ----------------------------------------------------------------------------
const int INF = -1;

struct Tri {
    int v[3];    // CCW; at most one entry is INF
    int nb[3];   // nb[k]: triangle across edge (v[k], v[(k+1)%3])
    bool alive;
};

struct Delaunay {
    const double *xy = nullptr;
    int n = 0;
    std::vector<Tri> tris;
    std::vector<int> free_list;
    int last = 0;

    bool is_ghost(const Tri &t) const { return t.v[0] == INF || t.v[1] == INF || t.v[2] == INF; }
    const double *P(int i) const { return xy + 2 * i; }

    bool conflicts(int ti, const double *p) const {
        const Tri &t = tris[ti];
        if (!is_ghost(t)) {
            const double *a = P(t.v[0]), *b = P(t.v[1]), *c = P(t.v[2]);
            return incircle(a[0], a[1], b[0], b[1], c[0], c[1], p[0], p[1]) > 0.0;
        }
        int k = 0;
        while (t.v[k] != INF) ++k;
        int u = t.v[(k + 1) % 3], v = t.v[(k + 2) % 3];   // ghost reads (u, v, INF) after rotation
        const double *pu = P(u), *pv = P(v);
        double o = orient2(pu[0], pu[1], pv[0], pv[1], p[0], p[1]);
        if (o > 0.0) return true;   // strictly outside hull edge v -> u
        if (o < 0.0) return false;
        // collinear with the hull edge: conflict only on the open segment
        double dot = (p[0] - pu[0]) * (pv[0] - pu[0]) + (p[1] - pu[1]) * (pv[1] - pu[1]);
        double len2 = (pv[0] - pu[0]) * (pv[0] - pu[0]) + (pv[1] - pu[1]) * (pv[1] - pu[1]);
        return dot > 0.0 && dot < len2;
    }

    int new_tri(int a, int b, int c) {
        Tri t;
        t.v[0] = a; t.v[1] = b; t.v[2] = c;
        t.nb[0] = t.nb[1] = t.nb[2] = -1;
        t.alive = true;
        if (!free_list.empty()) {
            int id = free_list.back();
            free_list.pop_back();
            tris[id] = t;
            return id;
        }
        tris.push_back(t);
        return (int)tris.size() - 1;
    }

    // Walk from `last` towards p across edges that p lies strictly beyond.
    int locate(const double *p) {
        int ti = last;
        if (!tris[ti].alive) {
            for (ti = 0; ti < (int)tris.size() && !tris[ti].alive; ++ti) {}
        }
        if (is_ghost(tris[ti])) {
            const Tri &g = tris[ti];
            int k = 0;
            while (g.v[k] != INF) ++k;
            ti = g.nb[(k + 1) % 3];   // finite triangle across the ghost's hull edge
        }
        size_t guard = 0, limit = 4 * tris.size() + 16;
        for (;;) {
            const Tri &t = tris[ti];
            if (is_ghost(t)) return ti;
            int moved = -1;
            for (int e = 0; e < 3; ++e) {
                int k = (e + (int)(guard % 3)) % 3;
                const double *a = P(t.v[k]), *b = P(t.v[(k + 1) % 3]);
                if (orient2(a[0], a[1], b[0], b[1], p[0], p[1]) < 0.0) { moved = t.nb[k]; break; }
            }
            if (moved < 0) return ti;
            ti = moved;
            if (++guard > limit) return -1;
        }
    }

    bool insert(int pi) {
        const double *p = P(pi);
        int start = locate(p);
        if (start < 0) return false;
        if (!conflicts(start, p)) {
            // the located triangle contains p; if it does not conflict, p
            // coincides with a vertex (excluded by the hard-disk input).
            return false;
        }
        std::vector<int> cavity, stack;
        cavity.reserve(16);
        stack.push_back(start);
        tris[start].alive = false;   // mark as taken into the cavity
        while (!stack.empty()) {
            int ti = stack.back();
            stack.pop_back();
            cavity.push_back(ti);
            for (int k = 0; k < 3; ++k) {
                int nb = tris[ti].nb[k];
                if (nb >= 0 && tris[nb].alive && conflicts(nb, p)) {
                    tris[nb].alive = false;
                    stack.push_back(nb);
                }
            }
        }
        // boundary edges (u, v) of the cavity, each seen from its cavity triangle
        struct BEdge { int u, v, outside; };
        std::vector<BEdge> boundary;
        for (int ti : cavity) {
            for (int k = 0; k < 3; ++k) {
                int nb = tris[ti].nb[k];
                if (nb < 0 || tris[nb].alive) boundary.push_back({tris[ti].v[k], tris[ti].v[(k + 1) % 3], nb});
            }
        }
        for (int ti : cavity) free_list.push_back(ti);
        std::unordered_map<int, int> starts;   // boundary start vertex -> new triangle
        std::vector<int> created;
        created.reserve(boundary.size());
        for (const BEdge &be : boundary) {
            int t = new_tri(be.u, be.v, pi);
            tris[t].nb[0] = be.outside;
            if (be.outside >= 0) {
                Tri &o = tris[be.outside];
                for (int k = 0; k < 3; ++k)
                    if (o.v[k] == be.v && o.v[(k + 1) % 3] == be.u) o.nb[k] = t;
            }
            starts[be.u] = t;
            created.push_back(t);
        }
        for (int t : created) {
            int v = tris[t].v[1];
            int u = tris[t].v[0];
            // edge (v, p) borders the new triangle starting at v
            auto it = starts.find(v);
            if (it == starts.end()) return false;
            tris[t].nb[1] = it->second;
            tris[it->second].nb[2] = t;
            (void)u;
        }
        for (int t : created)
            if (!is_ghost(tris[t])) { last = t; break; }
        return true;
    }

    // Builds DT(xy).  Returns false when all points are collinear or the
    // input has coincident points.
    bool build(const double *pts, int npts) {
        xy = pts;
        n = npts;
        tris.clear();
        free_list.clear();
        if (n < 3) return false;
        int i0 = 0, i1 = 1, i2 = -1;
        for (int k = 2; k < n; ++k) {
            const double *a = P(i0), *b = P(i1), *c = P(k);
            if (orient2(a[0], a[1], b[0], b[1], c[0], c[1]) != 0.0) { i2 = k; break; }
        }
        if (i2 < 0) return false;
        {
            const double *a = P(i0), *b = P(i1), *c = P(i2);
            if (orient2(a[0], a[1], b[0], b[1], c[0], c[1]) < 0.0) std::swap(i1, i2);
        }
        int t0 = new_tri(i0, i1, i2);
        int g0 = new_tri(i1, i0, INF);
        int g1 = new_tri(i2, i1, INF);
        int g2 = new_tri(i0, i2, INF);
        // link by matching reversed edges
        std::vector<int> all = {t0, g0, g1, g2};
        for (int a : all)
            for (int ka = 0; ka < 3; ++ka)
                for (int b : all) {
                    if (a == b) continue;
                    for (int kb = 0; kb < 3; ++kb)
                        if (tris[a].v[ka] == tris[b].v[(kb + 1) % 3] && tris[a].v[(ka + 1) % 3] == tris[b].v[kb])
                            tris[a].nb[ka] = b;
                }
        last = t0;
        for (int k = 0; k < n; ++k) {
            if (k == i0 || k == i1 || k == i2) continue;
            if (!insert(k)) return false;
        }
        return true;
    }

    void finite_triangles(std::vector<int> &out) const {
        out.clear();
        for (const Tri &t : tris)
            if (t.alive && !is_ghost(t)) { out.push_back(t.v[0]); out.push_back(t.v[1]); out.push_back(t.v[2]); }
    }

    // unique finite edges (i < j)
    void finite_edges(std::vector<std::pair<int, int>> &out) const {
        out.clear();
        for (const Tri &t : tris) {
            if (!t.alive || is_ghost(t)) continue;
            for (int k = 0; k < 3; ++k) {
                int a = t.v[k], b = t.v[(k + 1) % 3];
                int nbv = t.nb[k];
                // each interior edge is seen twice; keep it from the side with a < b,
                // hull edges (ghost neighbour) once
                bool nb_ghost = nbv >= 0 && is_ghost(tris[nbv]);
                if (a < b || nb_ghost) out.push_back({std::min(a, b), std::max(a, b)});
            }
        }
        std::sort(out.begin(), out.end());
        out.erase(std::unique(out.begin(), out.end()), out.end());
    }
};

// ----------------------------------------------------------------------------
// Pair forces, Sec. 2.2: F_i = sum_{j != i} K[s_i][s_j] g(d_ij) (r_i - r_j)/d_ij,
// g(d) = d^-q (power law; q = 2 is the paper's long-range r/r^3, q = 6 its
// short-range r/r^7) or g(d) = A exp(-d/lam)/d (screened), zero beyond an
// inclusive cutoff when cutoff > 0 (Sec. 2.2 cutoff rule, no force shift).
// Brute force over all ordered pairs; no neighbour list.
// ----------------------------------------------------------------------------
struct ForceModel {
    int S = 1;
    std::vector<double> K;     // S*S row-major
    int kind = 0;              // 0 power, 1 screened
    double q = 2.0, A = 1.0, lam = 1.0, cutoff = 0.0;
    double period = 0.0;       // > 0: periodic box of this side, separations by the minimum image (Sec. 2.1)
};

// Sec. 2.1 minimum-image convention: the separation component v of two
// points of a periodic box of side L taken from the nearest image, in
// [-L/2, L/2] (ties to even).
inline double min_image(double v, double L) { return L > 0.0 ? v - L * std::nearbyint(v / L) : v; }

// A coordinate of a periodic box of side L folded into [0, L).
inline double wrap(double c, double L) {
    double r = c - L * std::floor(c / L);
    return r >= L ? r - L : r;
}

inline double pair_scale(const ForceModel &fm, double d) {
    // returns g(d)/d so that the force is scale * (r_i - r_j)
    if (fm.kind == 0) {
        if (fm.q == 2.0) return 1.0 / (d * d * d);
        return std::pow(d, -fm.q) / d;
    }
    return fm.A * std::exp(-d / fm.lam) / d / d;
}

void forces_subset(const ForceModel &fm, int n, const double *xy, const int *sp, const int *idx, int m,
                   double *out) {
    for (int a = 0; a < m; ++a) {
        int i = idx ? idx[a] : a;
        double fx = 0.0, fy = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = min_image(xy[2 * i] - xy[2 * j], fm.period);
            double dy = min_image(xy[2 * i + 1] - xy[2 * j + 1], fm.period);
            double d = std::sqrt(dx * dx + dy * dy);
            if (fm.cutoff > 0.0 && d > fm.cutoff) continue;
            double k = fm.K[sp[i] * fm.S + sp[j]];
            double s = k * pair_scale(fm, d);
            fx += s * dx;
            fy += s * dy;
        }
        out[2 * a] = fx;
        out[2 * a + 1] = fy;
    }
}

// ----------------------------------------------------------------------------
// Forward-mode derivatives (tangents) of one step.  Not part of the paper's
// method: they define what its adjoint must compute.  The step is
// differentiated as written, with every discrete decision held fixed -- the
// overlapping edges of each correction round (the correction acts as a
// projection onto the contact set of that round), the cap branch, the wall
// branches, the cutoff -- so the tangent is that of the smooth map on the
// current branch.  For the pair term u = r_i - r_j, d = |u|, s(d) = g(d)/d:
//   d[K s(d) u] = K (s I + (s'(d)/d) u u^T) du + dK s u.
// ----------------------------------------------------------------------------
inline double pair_scale_slope(const ForceModel &fm, double d) {
    // returns s'(d) / d for s = pair_scale
    if (fm.kind == 0) return -(fm.q + 1.0) * std::pow(d, -fm.q - 3.0);
    const double e = fm.A * std::exp(-d / fm.lam);
    return e * (-1.0 / (fm.lam * d * d * d) - 2.0 / (d * d * d * d));
}

void force_tangent(const ForceModel &fm, int n, const double *xy, const int *sp, const double *txy,
                   const double *tK, double *out) {
    for (int i = 0; i < n; ++i) {
        double fx = 0.0, fy = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double ux = xy[2 * i] - xy[2 * j], uy = xy[2 * i + 1] - xy[2 * j + 1];
            double d = std::sqrt(ux * ux + uy * uy);
            if (fm.cutoff > 0.0 && d > fm.cutoff) continue;
            double dux = txy[2 * i] - txy[2 * j], duy = txy[2 * i + 1] - txy[2 * j + 1];
            double k = fm.K[sp[i] * fm.S + sp[j]];
            double tk = tK[sp[i] * fm.S + sp[j]];
            double sc = pair_scale(fm, d);
            double sl = pair_scale_slope(fm, d);
            double ud = ux * dux + uy * duy;
            fx += k * (sc * dux + sl * ux * ud) + tk * sc * ux;
            fy += k * (sc * duy + sl * uy * ud) + tk * sc * uy;
        }
        out[2 * i] = fx;
        out[2 * i + 1] = fy;
    }
}

// Hard walls: mirror reflection about the shifted wall, then a safety clamp.
inline double wall(double c, double r, double L) {
    double lo = r, hi = L - r;
    if (c < lo) c = 2.0 * lo - c;
    if (c > hi) c = 2.0 * hi - c;
    if (c < lo) c = lo;
    if (c > hi) c = hi;
    return c;
}

// Derivative of wall() at c: -1 per reflection, 0 where the clamp acts.
inline double wall_slope(double c, double r, double L) {
    double lo = r, hi = L - r, sl = 1.0;
    if (c < lo) { c = 2.0 * lo - c; sl = -sl; }
    if (c > hi) { c = 2.0 * hi - c; sl = -sl; }
    if (c < lo || c > hi) return 0.0;
    return sl;
}

// Frame of fixed points outside the walls of [0, L]^2: four arcs at
// 2 rmax beyond the wall lines (bottom, right, top, left, counter-clockwise),
// one point per 2 rmax along a side of length L + 4 rmax, pushed outwards by
// (rmax / 2) 4u(1 - u) at relative position u so that all of them are strict
// hull corners; side j holds K + j points, K = ceil((L + 4 rmax) / (2 rmax)),
// and starts at its corner.
void wall_frame(double L, double rmax, std::vector<double> &out) {
    out.clear();
    const double a = 2.0 * rmax;
    const double span = L + 2.0 * a;
    const double bow_max = 0.5 * rmax;
    const int K = (int)std::ceil(span / (2.0 * rmax));
    for (int side = 0; side < 4; ++side) {
        const int count = K + side;
        for (int k = 0; k < count; ++k) {
            const double u = (double)k / (double)count;
            const double bow = bow_max * (4.0 * u * (1.0 - u));
            const double t = u * span;
            double px = 0.0, py = 0.0;
            switch (side) {
                case 0: px = t - a; py = -a - bow; break;
                case 1: px = L + a + bow; py = t - a; break;
                case 2: px = L + a - t; py = L + a + bow; break;
                default: px = -a - bow; py = L + a - t; break;
            }
            out.push_back(px);
            out.push_back(py);
        }
    }
}

struct Stats {
    int64_t steps = 0;
    int64_t overlap_rounds_total = 0;
    int64_t overlap_rounds_max = 0;
    int64_t overlap_edges_total = 0;
    int64_t cap_hits = 0;
    int64_t reversals = 0;
    int64_t noise_clamps = 0;
    int64_t dt_halvings = 0;   // moves discarded after an edge reversal and redone as two halves
};

// One Jacobi overlap round over the given edges, Sec. 2.3 and Sec. 4.4:
// every overlapping edge (d < (r_i + r_j)(1 - tol)) moves both ends apart along the unit
// vector by f (r_i + r_j - d); the summed move of each particle is truncated to
// length cap_frac * r_i; walls are applied.  Returns the number of overlapping
// edges found (0: nothing moved).
inline bool overlapping(double d, double contact, double tol) { return d < contact * (1.0 - tol); }

// With txy non-NULL the tangent of the positions is carried through the round
// (overlapping set, cap branch and wall branches fixed):
//   d[f (sigma - d) u / d] = f ((sigma/d - 1) I - (sigma/d) n n^T) du,  n = u/d,
//   d[c D/|D|] = (c/|D|)(I - e e^T) dD,  e = D/|D|  (when the cap acts).
int64_t overlap_round(int n, double *xy, const double *rad, double L, double f, double cap_frac, double tol,
                      const std::vector<std::pair<int, int>> &edges, int64_t *cap_hits, double *txy = nullptr,
                      bool periodic = false) {
    std::vector<double> disp(2 * (size_t)n, 0.0);
    std::vector<double> tdisp(txy ? 2 * (size_t)n : 0, 0.0);
    std::vector<char> touched(n, 0);
    int64_t count = 0;
    for (const auto &e : edges) {
        int i = e.first, j = e.second;
        double dx = xy[2 * i] - xy[2 * j], dy = xy[2 * i + 1] - xy[2 * j + 1];
        if (periodic) {
            dx = min_image(dx, L);
            dy = min_image(dy, L);
        }
        double d = std::sqrt(dx * dx + dy * dy);
        double contact = rad[i] + rad[j];
        if (!overlapping(d, contact, tol)) continue;
        ++count;
        double s = f * (contact - d) / d;
        disp[2 * i] += s * dx;
        disp[2 * i + 1] += s * dy;
        disp[2 * j] -= s * dx;
        disp[2 * j + 1] -= s * dy;
        touched[i] = touched[j] = 1;
        if (txy) {
            double nx = dx / d, ny = dy / d;
            double dux = txy[2 * i] - txy[2 * j], duy = txy[2 * i + 1] - txy[2 * j + 1];
            double a = contact / d, nd = nx * dux + ny * duy;
            double ax = f * ((a - 1.0) * dux - a * nx * nd);
            double ay = f * ((a - 1.0) * duy - a * ny * nd);
            tdisp[2 * i] += ax;
            tdisp[2 * i + 1] += ay;
            tdisp[2 * j] -= ax;
            tdisp[2 * j + 1] -= ay;
        }
    }
    if (count == 0) return 0;
    for (int i = 0; i < n; ++i) {
        if (!touched[i]) continue;
        double ddx = disp[2 * i], ddy = disp[2 * i + 1];
        double len = std::sqrt(ddx * ddx + ddy * ddy);
        double cap = cap_frac * rad[i];
        double tdx = txy ? tdisp[2 * i] : 0.0, tdy = txy ? tdisp[2 * i + 1] : 0.0;
        if (len > cap) {
            double sc = cap / len;
            if (txy) {
                double ex = ddx / len, ey = ddy / len, et = ex * tdx + ey * tdy;
                tdx = sc * (tdx - ex * et);
                tdy = sc * (tdy - ey * et);
            }
            ddx = ddx * sc;
            ddy = ddy * sc;
            if (cap_hits) ++*cap_hits;
        }
        if (txy) {
            txy[2 * i] = wall_slope(xy[2 * i] + ddx, rad[i], L) * (txy[2 * i] + tdx);
            txy[2 * i + 1] = wall_slope(xy[2 * i + 1] + ddy, rad[i], L) * (txy[2 * i + 1] + tdy);
        }
        if (periodic) {
            xy[2 * i] = wrap(xy[2 * i] + ddx, L);
            xy[2 * i + 1] = wrap(xy[2 * i + 1] + ddy, L);
            continue;
        }
        xy[2 * i] = wall(xy[2 * i] + ddx, rad[i], L);
        xy[2 * i + 1] = wall(xy[2 * i + 1] + ddy, rad[i], L);
    }
    return count;
}

// Sec. 5 short-range variant of the overlap test: every pair of disks closer
// than contact, by brute force over all pairs (the plain definition that the
// library's neighbour lists reach faster); no triangulation is involved.
void overlapping_pairs(int n, const double *xy, const double *rad, double tol, std::vector<std::pair<int, int>> &out,
                       double period = 0.0) {
    out.clear();
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double dx = min_image(xy[2 * i] - xy[2 * j], period);
            double dy = min_image(xy[2 * i + 1] - xy[2 * j + 1], period);
            if (overlapping(std::sqrt(dx * dx + dy * dy), rad[i] + rad[j], tol)) out.push_back({i, j});
        }
}

// Noise of the two halves of interval (level, index) of step `step`, length h,
// whose increments are W (2 per disk) and Th: a Brownian bridge.  Given the
// increment W over h, the increment over the first half is W/2 plus an
// independent normal of variance 2 D (h/2)(h/2)/h = D h / 2 per component; the
// second half takes the rest.  The normals are Philox draws keyed by the step
// and the particle like the step's own, on stream 2^31 + level' 2^24 + 2 index
// (translation, clamped like the step's draws) and that + 1 (rotation, first
// normal of the pair, not clamped), level' = level + 1.
void bridge_noise(int n, uint64_t seed, int64_t step, int level, uint32_t index, double h, double D, double Dr,
                  double clip, const double *W, const double *Th, double *WL, double *WR, double *ThL, double *ThR) {
    const uint32_t key = 0x80000000u | ((uint32_t)(level + 1) << 24) | (index << 1);
    const double at = std::sqrt(0.5 * D * h), ar = std::sqrt(0.5 * Dr * h);
    for (int i = 0; i < n; ++i) {
        double ex, ey, er, unused;
        normal_pair(seed, step, (uint32_t)i, key, ex, ey);
        normal_pair(seed, step, (uint32_t)i, key | 1u, er, unused);
        ex = ex > clip ? clip : (ex < -clip ? -clip : ex);
        ey = ey > clip ? clip : (ey < -clip ? -clip : ey);
        WL[2 * i] = 0.5 * W[2 * i] + at * ex;
        WL[2 * i + 1] = 0.5 * W[2 * i + 1] + at * ey;
        WR[2 * i] = W[2 * i] - WL[2 * i];
        WR[2 * i + 1] = W[2 * i + 1] - WL[2 * i + 1];
        ThL[i] = 0.5 * Th[i] + ar * er;
        ThR[i] = Th[i] - ThL[i];
    }
}

struct Sim {
    int n = 0;
    int overlap_method = 0;                    // 0: Delaunay edges (Sec. 4.4); 1: all pairs (Sec. 5 lists)
    int max_halvings = 0;                      // 0: a reversal is only counted
    bool periodic = false;                     // periodic box (Sec. 2.1) instead of hard walls
    std::vector<int> torus_tris;               // periodic: triangles of the torus triangulation (3 ids each)
    std::vector<double> xy, rad, theta;
    std::vector<int> sp;
    ForceModel fm;
    double L = 0, D = 0, dt = 0, v0 = 0, Dr = 0;
    uint64_t seed = 0;
    int64_t step = 0;
    double f = 1.0, cap_frac = 0.5, clip = 3.0, tol = 1e-9;
    int max_rounds = 10000;
    Stats st;
    Delaunay dt_now;
    std::vector<double> frame;                 // 2m coordinates
    std::vector<double> pts;                   // disks then frame, the triangulated set
    std::vector<std::pair<int, int>> edges;    // Delaunay edges between two disks
    std::vector<double> forces;
    int last_rounds = 0;
    // forward-mode tangents (off unless set): positions and strength matrix
    bool tan_on = false;
    std::vector<double> txy, tK, tforce;

    // Periodic box: the Delaunay triangulation of the flat torus, from the
    // Delaunay triangulation of the 3 x 3 periodic copies of the points.  A
    // torus triangle appears there once per copy; the one kept is the copy
    // whose vertex of smallest id lies in the central box.  Triangles near the
    // outer border of the copies (where the copied triangulation is not the
    // periodic one) are never kept, since every edge is far shorter than L.
    // Every torus triangulation of n points has 2n triangles and 3n edges.
    bool retriangulate_torus() {
        pts.clear();
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox)
                for (int i = 0; i < n; ++i) {
                    pts.push_back(xy[2 * i] + ox * L);
                    pts.push_back(xy[2 * i + 1] + oy * L);
                }
        if (!dt_now.build(pts.data(), 9 * n)) return false;
        std::vector<int> all;
        dt_now.finite_triangles(all);
        torus_tris.clear();
        for (size_t t = 0; t < all.size(); t += 3) {
            int m = 0;
            for (int k = 1; k < 3; ++k)
                if (all[t + k] % n < all[t + m] % n) m = k;
            if (all[t + m] / n != 4) continue;   // the central copy is number 4
            for (int k = 0; k < 3; ++k) torus_tris.push_back(all[t + k] % n);
        }
        if ((int)torus_tris.size() != 6 * n) return false;
        edges.clear();
        for (size_t t = 0; t < torus_tris.size(); t += 3)
            for (int k = 0; k < 3; ++k) {
                int a = torus_tris[t + k], b = torus_tris[t + (k + 1) % 3];
                edges.push_back({std::min(a, b), std::max(a, b)});
            }
        std::sort(edges.begin(), edges.end());
        edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
        return (int)edges.size() == 3 * n;
    }

    bool retriangulate() {
        if (periodic) return retriangulate_torus();
        pts.assign(xy.begin(), xy.end());
        pts.insert(pts.end(), frame.begin(), frame.end());
        if (!dt_now.build(pts.data(), (int)(pts.size() / 2))) return false;
        std::vector<std::pair<int, int>> all;
        dt_now.finite_edges(all);
        edges.clear();
        for (const auto &e : all)
            if (e.first < n && e.second < n) edges.push_back(e);
        return true;
    }

    // One step, in the order of Algorithm 1 with the overlap loop of Sec. 4.4.
    // Returns 0, -3 (round cap exceeded) or -4 (triangulation failed).
    // The translational noise of the step is W = sqrt(2 D dt) xi and the
    // rotational one sqrt(2 Dr dt) n (xi clamped, n not); with
    // max_halvings > 0 a move that reverses a Delaunay edge is discarded and
    // the step is redone as two halves (Sec. 4.3), see substep().
    int advance() {
        const double amp = std::sqrt(2.0 * D * dt);
        const double amp_r = std::sqrt(2.0 * Dr * dt);
        std::vector<double> W(2 * (size_t)n), Th(n);
        for (int i = 0; i < n; ++i) {
            double zx, zy, nr, unused;
            normal_pair(seed, step, (uint32_t)i, 0u, zx, zy);
            if (zx > clip) { zx = clip; ++st.noise_clamps; }
            if (zx < -clip) { zx = -clip; ++st.noise_clamps; }
            if (zy > clip) { zy = clip; ++st.noise_clamps; }
            if (zy < -clip) { zy = -clip; ++st.noise_clamps; }
            normal_pair(seed, step, (uint32_t)i, 1u, nr, unused);
            W[2 * i] = amp * zx;
            W[2 * i + 1] = amp * zy;
            Th[i] = amp_r * nr;
        }
        int rounds = 0;
        int rc = substep(0, 0, W, Th, dt, rounds);
        if (rc != 0) return rc;
        last_rounds = rounds;
        st.overlap_rounds_total += rounds;
        if (rounds > st.overlap_rounds_max) st.overlap_rounds_max = rounds;
        ++st.steps;
        ++step;
        return 0;
    }

    void bridge(int level, uint32_t index, double h, const std::vector<double> &W, const std::vector<double> &Th,
                std::vector<double> &WL, std::vector<double> &WR, std::vector<double> &ThL,
                std::vector<double> &ThR) const {
        WL.resize(2 * (size_t)n);
        WR.resize(2 * (size_t)n);
        ThL.resize(n);
        ThR.resize(n);
        bridge_noise(n, seed, step, level, index, h, D, Dr, clip, W.data(), Th.data(), WL.data(), WR.data(),
                     ThL.data(), ThR.data());
    }

    // Interval (level, index) of the step: forces at the current positions,
    // the Euler-Maruyama move over h with noise increments W, Th, walls, the
    // reversal test on the Delaunay edges before the move (Sec. 4.3), then the
    // triangulation of the new positions and the overlap rounds.  A move that
    // reversed an edge is discarded and the interval redone as two halves
    // while level < max_halvings.  rounds accumulates the overlap rounds.
    int substep(int level, uint32_t index, const std::vector<double> &W, const std::vector<double> &Th, double h,
                int &rounds) {
        forces.assign(2 * (size_t)n, 0.0);
        forces_subset(fm, n, xy.data(), sp.data(), nullptr, n, forces.data());
        if (tan_on) {
            tforce.assign(2 * (size_t)n, 0.0);
            force_tangent(fm, n, xy.data(), sp.data(), txy.data(), tK.data(), tforce.data());
        }
        std::vector<double> nxy(2 * (size_t)n), nth(n), ntxy;
        if (tan_on) ntxy = txy;
        for (int i = 0; i < n; ++i) {
            double th = theta[i];
            double vx = forces[2 * i] + v0 * std::cos(th);
            double vy = forces[2 * i + 1] + v0 * std::sin(th);
            double x = xy[2 * i] + vx * h + W[2 * i];
            double y = xy[2 * i + 1] + vy * h + W[2 * i + 1];
            nxy[2 * i] = periodic ? wrap(x, L) : wall(x, rad[i], L);
            nxy[2 * i + 1] = periodic ? wrap(y, L) : wall(y, rad[i], L);
            if (tan_on) {
                ntxy[2 * i] = wall_slope(x, rad[i], L) * (txy[2 * i] + h * tforce[2 * i]);
                ntxy[2 * i + 1] = wall_slope(y, rad[i], L) * (txy[2 * i + 1] + h * tforce[2 * i + 1]);
            }
            nth[i] = th + Th[i];
        }
        if (overlap_method == 1) {
            xy.swap(nxy);
            theta.swap(nth);
            if (tan_on) txy.swap(ntxy);
            return pair_rounds(rounds);
        }
        // Sec. 4.3: an edge whose vector reversed means the pair passed through each other
        int64_t rev = 0;
        for (const auto &e : edges) {
            int i = e.first, j = e.second;
            const double P = periodic ? L : 0.0;
            double ox = min_image(xy[2 * j] - xy[2 * i], P), oy = min_image(xy[2 * j + 1] - xy[2 * i + 1], P);
            double mx = min_image(nxy[2 * j] - nxy[2 * i], P), my = min_image(nxy[2 * j + 1] - nxy[2 * i + 1], P);
            if (ox * mx + oy * my < 0.0) ++rev;
        }
        st.reversals += rev;
        if (rev > 0 && level < max_halvings) {
            ++st.dt_halvings;
            std::vector<double> WL, WR, ThL, ThR;
            bridge(level, index, h, W, Th, WL, WR, ThL, ThR);
            int rc = substep(level + 1, 2 * index, WL, ThL, 0.5 * h, rounds);
            if (rc != 0) return rc;
            return substep(level + 1, 2 * index + 1, WR, ThR, 0.5 * h, rounds);
        }
        xy.swap(nxy);
        theta.swap(nth);
        if (tan_on) txy.swap(ntxy);
        if (!retriangulate()) return -4;
        for (int done = 0;;) {
            int64_t cnt = overlap_round(n, xy.data(), rad.data(), L, f, cap_frac, tol, edges, &st.cap_hits,
                                        tan_on ? txy.data() : nullptr, periodic);
            if (cnt == 0) break;
            ++done;
            ++rounds;
            st.overlap_edges_total += cnt;
            if (!retriangulate()) return -4;
            if (done >= max_rounds) {
                // still overlapping after the cap?
                bool any = false;
                for (const auto &e : edges) {
                    int i = e.first, j = e.second;
                    const double P = periodic ? L : 0.0;
                    double dx = min_image(xy[2 * i] - xy[2 * j], P), dy = min_image(xy[2 * i + 1] - xy[2 * j + 1], P);
                    if (overlapping(std::sqrt(dx * dx + dy * dy), rad[i] + rad[j], tol)) { any = true; break; }
                }
                if (any) return -3;
                break;
            }
        }
        return 0;
    }

    // Overlap rounds of the short-range variant (Sec. 5): over every
    // overlapping pair, no triangulation.
    int pair_rounds(int &rounds) {
        std::vector<std::pair<int, int>> pairs;
        for (int done = 0;;) {
            overlapping_pairs(n, xy.data(), rad.data(), tol, pairs, periodic ? L : 0.0);
            if (pairs.empty()) return 0;
            if (done >= max_rounds) return -3;
            int64_t cnt = overlap_round(n, xy.data(), rad.data(), L, f, cap_frac, tol, pairs, &st.cap_hits,
                                        tan_on ? txy.data() : nullptr, periodic);
            ++done;
            ++rounds;
            st.overlap_edges_total += cnt;
        }
    }
};

}  // namespace

// =============================================================================
// C interface for the test-suite (ctypes).
// =============================================================================
extern "C" {

void orc_philox4x32_10(const uint32_t *ctr, const uint32_t *key, uint32_t *out) {
    Words4 w = philox4x32_10(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1]);
    for (int k = 0; k < 4; ++k) out[k] = w.w[k];
}

// Raw (unclamped) normal pairs for ids 0..n-1 of one (seed, step, stream).
void orc_normals(int n, uint64_t seed, int64_t step, uint32_t stream, double *out) {
    for (int i = 0; i < n; ++i) normal_pair(seed, step, (uint32_t)i, stream, out[2 * i], out[2 * i + 1]);
}

double orc_orient2(const double *a, const double *b, const double *c) {
    return orient2(a[0], a[1], b[0], b[1], c[0], c[1]);
}

double orc_incircle(const double *a, const double *b, const double *c, const double *d) {
    return incircle(a[0], a[1], b[0], b[1], c[0], c[1], d[0], d[1]);
}

int orc_inverted_edge_flip(const double *v1, const double *v2, const double *v3, const double *v4) {
    return inverted_edge_flip(v1, v2, v3, v4) ? 1 : 0;
}

int orc_point_in_closed_triangle(const double *v1, const double *v2, const double *v3, const double *p) {
    return point_in_closed_triangle(v1, v2, v3, p) ? 1 : 0;
}

// Finite Delaunay triangles (CCW) of n points; tri_out holds 3*cap ints.
// Returns the triangle count, or -1 on failure, -2 when cap is too small.
int orc_delaunay(int n, const double *xy, int *tri_out, int cap) {
    Delaunay d;
    if (!d.build(xy, n)) return -1;
    std::vector<int> t;
    d.finite_triangles(t);
    int nt = (int)(t.size() / 3);
    if (nt > cap) return -2;
    std::memcpy(tri_out, t.data(), t.size() * sizeof(int));
    return nt;
}

// Forces for the particles listed in idx (m of them; idx NULL = all n), in a
// periodic box of side period (minimum-image separations; period 0: no box).
void orc_forces_periodic(int n, const double *xy, const int *sp, int S, const double *K, int kind, double q, double A,
                         double lam, double cutoff, double period, const int *idx, int m, double *out) {
    ForceModel fm;
    fm.period = period;
    fm.S = S;
    fm.K.assign(K, K + S * S);
    fm.kind = kind; fm.q = q; fm.A = A; fm.lam = lam; fm.cutoff = cutoff;
    forces_subset(fm, n, xy, sp, idx, idx ? m : n, out);
}

// The same without a periodic box.
void orc_forces(int n, const double *xy, const int *sp, int S, const double *K, int kind, double q, double A,
                double lam, double cutoff, const int *idx, int m, double *out) {
    orc_forces_periodic(n, xy, sp, S, K, kind, q, A, lam, cutoff, 0.0, idx, m, out);
}

// Tangent of the pair forces: d F / d(xy, K) applied to (txy, tK) (S*S, may be NULL).
void orc_force_tangent(int n, const double *xy, const int *sp, int S, const double *K, int kind, double q,
                       double A, double lam, double cutoff, const double *txy, const double *tK, double *out) {
    ForceModel fm;
    fm.S = S;
    fm.K.assign(K, K + S * S);
    fm.kind = kind; fm.q = q; fm.A = A; fm.lam = lam; fm.cutoff = cutoff;
    std::vector<double> zero(S * S, 0.0);
    force_tangent(fm, n, xy, sp, txy, tK ? tK : zero.data(), out);
}

double orc_wall(double c, double r, double L) { return wall(c, r, L); }

// One overlap round over the current Delaunay edges of xy (in place).
// Returns the number of overlapping edges, -4 if the triangulation failed.
int64_t orc_overlap_round(int n, double *xy, const double *rad, double L, double f, double cap_frac, double tol,
                          int64_t *cap_hits) {
    Delaunay d;
    if (!d.build(xy, n)) return -4;
    std::vector<std::pair<int, int>> e;
    d.finite_edges(e);
    return overlap_round(n, xy, rad, L, f, cap_frac, tol, e, cap_hits);
}

// One overlap round over every overlapping pair of xy (in place), the
// short-range variant; returns the number of overlapping pairs.
int64_t orc_overlap_round_pairs(int n, double *xy, const double *rad, double L, double f, double cap_frac, double tol,
                                int64_t *cap_hits) {
    std::vector<std::pair<int, int>> pairs;
    overlapping_pairs(n, xy, rad, tol, pairs);
    return overlap_round(n, xy, rad, L, f, cap_frac, tol, pairs, cap_hits);
}

// Frame points (2 doubles each) into out (room for cap points); returns m or -2.
int orc_frame(double L, double rmax, double *out, int cap) {
    std::vector<double> f;
    wall_frame(L, rmax, f);
    int m = (int)(f.size() / 2);
    if (m > cap) return -2;
    std::memcpy(out, f.data(), f.size() * sizeof(double));
    return m;
}

// --- simulation handle -------------------------------------------------------
void *orc_sim_new(int n, const double *xy, const double *rad, const int *sp, const double *theta, int S,
                  const double *K, int kind, double q, double A, double lam, double cutoff, double L, double D,
                  double dt, double v0, double Dr, uint64_t seed, int64_t step0, double f, double cap_frac,
                  double clip, double tol, int max_rounds) {
    Sim *s = new Sim();
    s->n = n;
    s->xy.assign(xy, xy + 2 * (size_t)n);
    s->rad.assign(rad, rad + n);
    s->sp.assign(sp, sp + n);
    if (theta) s->theta.assign(theta, theta + n); else s->theta.assign(n, 0.0);
    s->fm.S = S;
    s->fm.K.assign(K, K + S * S);
    s->fm.kind = kind; s->fm.q = q; s->fm.A = A; s->fm.lam = lam; s->fm.cutoff = cutoff;
    s->L = L; s->D = D; s->dt = dt; s->v0 = v0; s->Dr = Dr;
    s->seed = seed; s->step = step0;
    s->f = f; s->cap_frac = cap_frac; s->clip = clip; s->tol = tol; s->max_rounds = max_rounds;
    double rmax = 0.0;
    for (int i = 0; i < n; ++i) rmax = std::max(rmax, rad[i]);
    wall_frame(L, rmax, s->frame);
    if (!s->retriangulate()) { delete s; return nullptr; }
    return s;
}

int orc_sim_step(void *h, int64_t nsteps) {
    Sim *s = (Sim *)h;
    for (int64_t k = 0; k < nsteps; ++k) {
        int rc = s->advance();
        if (rc != 0) return rc;
    }
    return 0;
}

int orc_sim_last_rounds(void *h) { return ((Sim *)h)->last_rounds; }

// 0: overlap rounds over Delaunay edges (default); 1: over all overlapping pairs, no triangulation.
void orc_sim_set_overlap_method(void *h, int method) { ((Sim *)h)->overlap_method = method; }

// Periodic box of side L (Sec. 2.1): minimum-image separations, positions
// folded into [0, L), the torus triangulation, no walls and no frame.
// Returns 0, or -4 if the torus triangulation fails.
int orc_sim_set_periodic(void *h) {
    Sim *s = (Sim *)h;
    s->periodic = true;
    s->fm.period = s->L;
    s->frame.clear();
    for (int i = 0; i < 2 * s->n; ++i) s->xy[i] = wrap(s->xy[i], s->L);
    return s->retriangulate() ? 0 : -4;
}

// Torus triangulation of n points in [0, L)^2 (3 ids per triangle, CCW); returns the count or < 0.
int orc_torus_delaunay(int n, const double *xy, double L, int *tri_out, int cap) {
    Sim s;
    s.n = n;
    s.L = L;
    s.periodic = true;
    s.xy.assign(xy, xy + 2 * (size_t)n);
    if (!s.retriangulate()) return -1;
    int nt = (int)(s.torus_tris.size() / 3);
    if (nt > cap) return -2;
    std::memcpy(tri_out, s.torus_tris.data(), s.torus_tris.size() * sizeof(int));
    return nt;
}

// Levels of halving of a move that reversed a Delaunay edge (0: only counted).
void orc_sim_set_max_halvings(void *h, int levels) { ((Sim *)h)->max_halvings = levels; }

int64_t orc_sim_dt_halvings(void *h) { return ((Sim *)h)->st.dt_halvings; }

void orc_bridge(int n, uint64_t seed, int64_t step, int level, uint32_t index, double h, double D, double Dr,
                double clip, const double *W, const double *Th, double *WL, double *WR, double *ThL, double *ThR) {
    bridge_noise(n, seed, step, level, index, h, D, Dr, clip, W, Th, WL, WR, ThL, ThR);
}

void orc_sim_get(void *h, double *xy, double *theta, int64_t *step, int64_t *stats7) {
    Sim *s = (Sim *)h;
    if (xy) std::memcpy(xy, s->xy.data(), s->xy.size() * sizeof(double));
    if (theta) std::memcpy(theta, s->theta.data(), s->theta.size() * sizeof(double));
    if (step) *step = s->step;
    if (stats7) {
        stats7[0] = s->st.steps;
        stats7[1] = s->st.overlap_rounds_total;
        stats7[2] = s->st.overlap_rounds_max;
        stats7[3] = s->st.overlap_edges_total;
        stats7[4] = s->st.cap_hits;
        stats7[5] = s->st.reversals;
        stats7[6] = s->st.noise_clamps;
    }
}

// Forces at the current positions (the ones the next step will use).
void orc_sim_forces(void *h, double *out) {
    Sim *s = (Sim *)h;
    forces_subset(s->fm, s->n, s->xy.data(), s->sp.data(), nullptr, s->n, out);
}

// Starts carrying forward-mode tangents: txy (2n) of the positions and tK
// (S*S, may be NULL for zero) of the strength matrix.
void orc_sim_set_tangent(void *h, const double *txy, const double *tK) {
    Sim *s = (Sim *)h;
    s->tan_on = true;
    s->txy.assign(txy, txy + 2 * (size_t)s->n);
    if (tK)
        s->tK.assign(tK, tK + s->fm.S * s->fm.S);
    else
        s->tK.assign(s->fm.S * s->fm.S, 0.0);
}

void orc_sim_get_tangent(void *h, double *out) {
    Sim *s = (Sim *)h;
    if (s->tan_on) std::memcpy(out, s->txy.data(), s->txy.size() * sizeof(double));
}

int orc_sim_frame_count(void *h) { return (int)(((Sim *)h)->frame.size() / 2); }

int orc_sim_triangles(void *h, int *tri_out, int cap) {
    Sim *s = (Sim *)h;
    std::vector<int> t;
    if (s->periodic)
        t = s->torus_tris;
    else
        s->dt_now.finite_triangles(t);
    int nt = (int)(t.size() / 3);
    if (nt > cap) return -2;
    std::memcpy(tri_out, t.data(), t.size() * sizeof(int));
    return nt;
}

void orc_sim_free(void *h) { delete (Sim *)h; }

}  // extern "C"
