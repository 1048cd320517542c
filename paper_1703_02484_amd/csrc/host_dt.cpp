// Host construction of the initial Delaunay triangulation (Sec. 4.1: built
// once on the host, then kept on the device) and of the fallback rebuild.
//
// Incremental insertion with edge flips (Lawson): points are inserted in
// Hilbert-curve order so the locating walk is short; each point splits the
// triangle containing it (or the two triangles sharing the edge it lies on,
// or the ghost triangle beyond the hull edge it sees), and the edges opposite
// the new point are legalised with the same flip rule the device uses
// (in-circle for finite quads, convexity for edges to the infinite vertex).
// Output is the device half-edge layout: triangle t owns half-edges 3t..3t+2.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <unordered_map>
#include <vector>

#include "bd_internal.h"
#include "geom.h"

namespace bd {

// Distance of cell (x, y) along the Hilbert curve over a 2^bits x 2^bits grid
// (the rotate-and-reflect recursion of the curve, one bit level at a time).
uint64_t hilbert_index(uint32_t x, uint32_t y, int bits) {
    uint64_t d = 0;
    for (uint32_t s = 1u << (bits - 1); s > 0; s >>= 1) {
        uint32_t rx = (x & s) ? 1 : 0;
        uint32_t ry = (y & s) ? 1 : 0;
        d += (uint64_t)s * s * ((3 * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = s - 1 - x;
                y = s - 1 - y;
            }
            uint32_t t = x;
            x = y;
            y = t;
        }
    }
    return d;
}

namespace {

struct Mesh {
    int n, inf;
    const double *x, *y;
    std::vector<int> V, Tw;
    int ntri = 0;
    std::vector<int> stack;

    bool ghost(int t) const { return V[3 * t] == inf || V[3 * t + 1] == inf || V[3 * t + 2] == inf; }

    int add(int a, int b, int c) {
        int t = ntri++;
        V[3 * t] = a;
        V[3 * t + 1] = b;
        V[3 * t + 2] = c;
        Tw[3 * t] = Tw[3 * t + 1] = Tw[3 * t + 2] = -1;
        return t;
    }
    void set(int t, int a, int b, int c) {
        V[3 * t] = a;
        V[3 * t + 1] = b;
        V[3 * t + 2] = c;
    }
    void link(int h, int g) {
        Tw[h] = g;
        if (g >= 0) Tw[g] = h;
    }

    double orient_p(int a, int b, double px, double py) const { return bd_orient(x[a], y[a], x[b], y[b], px, py); }

    // Lawson flip of the edge h (a -> b) between (a, b, c) and (b, a, d):
    // the triangles become (c, a, d) and (d, b, c) in the same slots.
    void flip(int h) {
        const int t1 = h / 3, g = Tw[h], t2 = g / 3;
        const int hb = bd_next(h), hc = bd_prev(h), ga = bd_next(g), gd = bd_prev(g);
        const int a = V[h], b = V[hb], c = V[hc], d = V[gd];
        const int Thb = Tw[hb], Thc = Tw[hc], Tga = Tw[ga], Tgd = Tw[gd];
        set(t1, c, a, d);
        set(t2, d, b, c);
        link(3 * t1 + 0, Thc);
        link(3 * t1 + 1, Tga);
        link(3 * t2 + 0, Tgd);
        link(3 * t2 + 1, Thb);
        link(3 * t1 + 2, 3 * t2 + 2);
    }

    // Legalise the half-edges on the stack; each lies in a triangle whose
    // third vertex is the point just inserted (slot: opposite vertex = prev).
    void legalize() {
        while (!stack.empty()) {
            int h = stack.back();
            stack.pop_back();
            int g = Tw[h];
            int a = V[h], b = V[bd_next(h)], c = V[bd_prev(h)], d = V[bd_prev(g)];
            if (bd_flip_rule(a, b, c, d, inf, x, y, false) == BD_NOFLIP) continue;
            int t1 = h / 3, t2 = g / 3;
            flip(h);
            // new (c, a, d): edge a -> d is slot 1; new (d, b, c): edge d -> b is slot 0
            stack.push_back(3 * t1 + 1);
            stack.push_back(3 * t2 + 0);
        }
    }

    // 1 -> 3 split of triangle t = (a, b, c) by point p (finite or ghost).
    void split3(int t, int p) {
        const int a = V[3 * t], b = V[3 * t + 1], c = V[3 * t + 2];
        const int Tab = Tw[3 * t], Tbc = Tw[3 * t + 1], Tca = Tw[3 * t + 2];
        const int t0 = t;
        set(t0, a, b, p);
        const int t1 = add(b, c, p);
        const int t2 = add(c, a, p);
        link(3 * t0 + 0, Tab);
        link(3 * t1 + 0, Tbc);
        link(3 * t2 + 0, Tca);
        link(3 * t0 + 1, 3 * t1 + 2);   // b -> p  /  p -> b
        link(3 * t1 + 1, 3 * t2 + 2);   // c -> p  /  p -> c
        link(3 * t2 + 1, 3 * t0 + 2);   // a -> p  /  p -> a
        stack.push_back(3 * t0);
        stack.push_back(3 * t1);
        stack.push_back(3 * t2);
    }

    // 2 -> 4 split: p lies on the edge h = a -> b of (a, b, c); twin in (b, a, d).
    void split4(int h, int p) {
        const int t1 = h / 3, g = Tw[h], t2 = g / 3;
        const int hb = bd_next(h), hc = bd_prev(h), ga = bd_next(g), gd = bd_prev(g);
        const int a = V[h], b = V[hb], c = V[hc], d = V[gd];
        const int Tbc = Tw[hb], Tca = Tw[hc], Tad = Tw[ga], Tdb = Tw[gd];
        set(t1, c, a, p);
        set(t2, b, c, p);
        const int t3 = add(d, b, p);
        const int t4 = add(a, d, p);
        link(3 * t1 + 0, Tca);
        link(3 * t2 + 0, Tbc);
        link(3 * t3 + 0, Tdb);
        link(3 * t4 + 0, Tad);
        link(3 * t1 + 1, 3 * t4 + 2);   // a -> p / p -> a
        link(3 * t2 + 1, 3 * t1 + 2);   // c -> p / p -> c
        link(3 * t3 + 1, 3 * t2 + 2);   // b -> p / p -> b
        link(3 * t4 + 1, 3 * t3 + 2);   // d -> p / p -> d
        stack.push_back(3 * t1);
        stack.push_back(3 * t2);
        stack.push_back(3 * t3);
        stack.push_back(3 * t4);
    }

    // Walk to the triangle containing p.  mode 0: strictly inside finite t;
    // 1: on the edge `h`; 2: ghost t (p beyond its hull edge); -1: duplicate.
    int locate(double px, double py, int start, int &t_out, int &h_out) const {
        int t = start;
        if (ghost(t)) {
            const int g = t;
            for (int k = 0; k < 3; ++k) {
                const int h = 3 * g + k;
                if (V[h] != inf && V[bd_next(h)] != inf) {
                    t = Tw[h] / 3;   // the finite triangle across the ghost's hull edge
                    break;
                }
            }
        }
        int rot = 0;
        for (long guard = 0; guard < 4L * ntri + 64; ++guard) {
            if (ghost(t)) {
                t_out = t;
                return 2;
            }
            int moved = -1, zeros = 0, zk = -1;
            for (int e = 0; e < 3; ++e) {
                int k = (e + rot) % 3;
                int h = 3 * t + k;
                double o = orient_p(V[h], V[bd_next(h)], px, py);
                if (o < 0.0) {
                    moved = Tw[h] / 3;
                    break;
                }
                if (o == 0.0) {
                    ++zeros;
                    zk = h;
                }
            }
            ++rot;
            if (moved >= 0) {
                t = moved;
                continue;
            }
            t_out = t;
            if (zeros == 0) return 0;
            if (zeros == 1) {
                h_out = zk;
                return 1;
            }
            return -1;
        }
        return -1;
    }
};

}  // namespace

// The frame: four bowed arcs just outside the walls, at distance a = 2 rmax
// beyond each wall line, one point every s = 2 rmax, bowed outwards by up to
// rmax / 2 so that every frame point is a strict convex-hull corner; side j
// (bottom, right, top, left, counter-clockwise) has K + j points so that no
// two sides mirror each other.  Each side contributes its starting corner.
void frame_points(double L, double rmax, std::vector<double> &fx, std::vector<double> &fy) {
#pragma clang fp contract(off)
    const double a = 2.0 * rmax;
    const double s = 2.0 * rmax;
    const double bow_max = 0.5 * rmax;
    const double span = L + 2.0 * a;
    const int K = (int)std::ceil(span / s);
    fx.clear();
    fy.clear();
    for (int side = 0; side < 4; ++side) {
        const int cnt = K + side;
        for (int k = 0; k < cnt; ++k) {
            const double u = (double)k / (double)cnt;
            const double bow = bow_max * (4.0 * u * (1.0 - u));
            const double t = u * span;
            double px, py;
            if (side == 0) {
                px = t - a;
                py = -a - bow;
            } else if (side == 1) {
                px = L + a + bow;
                py = t - a;
            } else if (side == 2) {
                px = L + a - t;
                py = L + a + bow;
            } else {
                px = -a - bow;
                py = L + a - t;
            }
            fx.push_back(px);
            fy.push_back(py);
        }
    }
}

int host_delaunay(int n, const double *x, const double *y, std::vector<int> &he_v, std::vector<int> &he_twin) {
    if (n < 3) return -1;
    Mesh m;
    m.n = n;
    m.inf = n;
    m.x = x;
    m.y = y;
    const int T = 2 * n - 2;
    m.V.assign(3 * (size_t)T, -1);
    m.Tw.assign(3 * (size_t)T, -1);
    // Hilbert order over the bounding box
    double x0 = x[0], x1 = x[0], y0 = y[0], y1 = y[0];
    for (int i = 1; i < n; ++i) {
        x0 = std::min(x0, x[i]);
        x1 = std::max(x1, x[i]);
        y0 = std::min(y0, y[i]);
        y1 = std::max(y1, y[i]);
    }
    const double span = std::max(x1 - x0, y1 - y0);
    const double scale = span > 0 ? 65535.0 / span : 0.0;
    std::vector<uint64_t> key(n);
    for (int i = 0; i < n; ++i)
        key[i] = hilbert_index((uint32_t)((x[i] - x0) * scale), (uint32_t)((y[i] - y0) * scale), 16);
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
    // first non-degenerate triangle
    int i0 = order[0], i1 = order[1], i2 = -1, pos2 = -1;
    for (int k = 2; k < n; ++k) {
        int c = order[k];
        if (bd_orient(x[i0], y[i0], x[i1], y[i1], x[c], y[c]) != 0.0) {
            i2 = c;
            pos2 = k;
            break;
        }
    }
    if (i2 < 0) return -1;
    if (bd_orient(x[i0], y[i0], x[i1], y[i1], x[i2], y[i2]) < 0.0) std::swap(i1, i2);
    const int inf = n;
    int t0 = m.add(i0, i1, i2);
    int g0 = m.add(i1, i0, inf);
    int g1 = m.add(i2, i1, inf);
    int g2 = m.add(i0, i2, inf);
    m.link(3 * t0 + 0, 3 * g0 + 0);   // i0->i1 / i1->i0
    m.link(3 * t0 + 1, 3 * g1 + 0);   // i1->i2 / i2->i1
    m.link(3 * t0 + 2, 3 * g2 + 0);   // i2->i0 / i0->i2
    m.link(3 * g0 + 1, 3 * g2 + 2);   // i0->inf / inf->i0
    m.link(3 * g1 + 1, 3 * g0 + 2);   // i1->inf / inf->i1
    m.link(3 * g2 + 1, 3 * g1 + 2);   // i2->inf / inf->i2
    int last = t0;
    for (int k = 2; k < n; ++k) {
        if (k == pos2) continue;
        int p = order[k];
        if (p == i0 || p == i1 || p == i2) continue;
        int t = -1, h = -1;
        int mode = m.locate(x[p], y[p], last, t, h);
        if (mode < 0) return -1;
        if (mode == 1) {
            m.split4(h, p);
        } else {
            m.split3(t, p);
        }
        m.legalize();
        last = t;
    }
    if (m.ntri != T) return -1;
    he_v.swap(m.V);
    he_twin.swap(m.Tw);
    return 0;
}

// Delaunay triangulation of the flat torus [0, L)^2 (the periodic box of
// Sec. 2.1, whose triangulation the paper builds with a periodic Delaunay
// library) as half-edges over the ids 0..n-1, 2n triangles, no infinite
// vertex.  The planar triangulation of the points and of their periodic
// copies inside a band of width w around the box equals the periodic one
// near the box; every torus triangle appears there once per copy, and the
// copy kept is the one whose vertex of smallest id lies in the box itself.  A
// kept triangle whose circumcircle leaves the band may be wrong (a copy
// outside the band could lie inside it): the band is then widened.  Twins pair
// the directed edges a -> b and b -> a, which are unique while every edge is
// shorter than L / 2.  Returns 0, or -1 (degenerate input or a box too small
// for its points).
int host_torus_delaunay(int n, const double *x, const double *y, double L, std::vector<int> &he_v,
                        std::vector<int> &he_twin) {
    if (n < 3 || !(L > 0)) return -1;
    double w = std::min(L, 6.0 * std::sqrt(L * L / n));
    for (;;) {
        std::vector<double> px, py;
        std::vector<int> id, cp;   // original id and copy (ox + 1) + 3 (oy + 1); the box itself is copy 4
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox)
                for (int i = 0; i < n; ++i) {
                    const double X = x[i] + ox * L, Y = y[i] + oy * L;
                    if (X < -w || X >= L + w || Y < -w || Y >= L + w) continue;
                    px.push_back(X);
                    py.push_back(Y);
                    id.push_back(i);
                    cp.push_back((ox + 1) + 3 * (oy + 1));
                }
        std::vector<int> V, Tw;
        const int m = (int)px.size();
        if (host_delaunay(m, px.data(), py.data(), V, Tw) != 0) return -1;
        std::vector<int> tri;
        bool narrow = false;
        for (size_t t = 0; 3 * t < V.size(); ++t) {
            const int a = V[3 * t], b = V[3 * t + 1], c = V[3 * t + 2];
            if (a >= m || b >= m || c >= m) continue;   // ghost
            int lo = a;
            if (id[b] < id[lo]) lo = b;
            if (id[c] < id[lo]) lo = c;
            if (cp[lo] != 4) continue;
            // circumcircle of the kept triangle inside the band
            const double bx = px[b] - px[a], by = py[b] - py[a], cx = px[c] - px[a], cy = py[c] - py[a];
            const double d = 2.0 * (bx * cy - by * cx);
            const double b2 = bx * bx + by * by, c2 = cx * cx + cy * cy;
            const double ux = (cy * b2 - by * c2) / d, uy = (bx * c2 - cx * b2) / d;
            const double r = std::sqrt(ux * ux + uy * uy), ox = px[a] + ux, oy = py[a] + uy;
            if (ox - r < -w || ox + r > L + w || oy - r < -w || oy + r > L + w) narrow = true;
            tri.push_back(id[a]);
            tri.push_back(id[b]);
            tri.push_back(id[c]);
        }
        if (narrow && w < L) {
            w = std::min(L, 2.0 * w);
            continue;
        }
        if ((int)tri.size() != 6 * n) return -1;
        he_v = tri;
        he_twin.assign(tri.size(), -1);
        std::unordered_map<uint64_t, int> dir;
        dir.reserve(tri.size() * 2);
        auto key = [](int a, int b) { return ((uint64_t)(uint32_t)a << 32) | (uint32_t)b; };
        for (size_t h = 0; h < tri.size(); ++h) {
            const int a = tri[h], b = tri[bd_next((int)h)];
            if (!dir.emplace(key(a, b), (int)h).second) return -1;   // the same directed edge twice
        }
        for (size_t h = 0; h < tri.size(); ++h) {
            auto it = dir.find(key(tri[bd_next((int)h)], tri[h]));
            if (it == dir.end()) return -1;
            he_twin[h] = it->second;
        }
        return 0;
    }
}

}  // namespace bd
