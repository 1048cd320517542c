// FP64 geometric predicates and the edge-flip rule of the triangulation
// repair, used by the device kernels and by the library's host triangulator.
//
// All predicates are plain FP64 in translated form with floating-point
// contraction disabled, so host and device evaluate them identically.  The
// triangulation has one infinite vertex (id = inf) that closes the convex
// hull: a ghost triangle (q, p, inf) lies beyond hull edge p -> q.
#pragma once

#include <hip/hip_runtime.h>

#define BD_HD __host__ __device__ __forceinline__

// Twice the signed area of (a, b, c); > 0 for a counter-clockwise turn.
// Translated to a: (b - a) x (c - a), the fixed expression form both the
// device and the host evaluate.
BD_HD double bd_orient(double ax, double ay, double bx, double by, double cx, double cy) {
#pragma clang fp contract(off)
    double bax = bx - ax, bay = by - ay;
    double cax = cx - ax, cay = cy - ay;
    return bax * cay - bay * cax;
}

// > 0 when d is strictly inside the circle through the CCW triangle (a, b, c).
BD_HD double bd_incircle(double ax, double ay, double bx, double by, double cx, double cy, double dx,
                         double dy) {
#pragma clang fp contract(off)
    double adx = ax - dx, ady = ay - dy;
    double bdx = bx - dx, bdy = by - dy;
    double cdx = cx - dx, cdy = cy - dy;
    double ab = adx * bdy - bdx * ady;
    double bc = bdx * cdy - cdx * bdy;
    double ca = cdx * ady - adx * cdy;
    double alift = adx * adx + ady * ady;
    double blift = bdx * bdx + bdy * bdy;
    double clift = cdx * cdx + cdy * cdy;
    return alift * bc + blift * ca + clift * ab;
}

// Sec. 4.3 point-in-triangle test in barycentric form, valid for either
// orientation of the triangle: p = v1 + s (v2 - v1) + t (v3 - v1) lies in
// the closed triangle when s >= 0, t >= 0 and s + t <= 1.  The coordinates
// are kept multiplied by the doubled signed area w, hence the two cases.
BD_HD bool bd_in_closed_tri(double v1x, double v1y, double v2x, double v2y, double v3x, double v3y, double px,
                            double py) {
#pragma clang fp contract(off)
    double e0x = v2x - v1x, e0y = v2y - v1y;
    double e1x = v3x - v1x, e1y = v3y - v1y;
    double qx = px - v1x, qy = py - v1y;
    double w = e0x * e1y - e0y * e1x;
    double s = qx * e1y - qy * e1x;
    double t = e0x * qy - e0y * qx;
    if (w < 0.0) return (s <= 0.0) && (t <= 0.0) && (s + t >= w);
    return (s >= 0.0) && (t >= 0.0) && (s + t <= w);
}

enum { BD_NOFLIP = 0, BD_FLIP_LAWSON = 1, BD_FLIP_INVERSION = 2 };

// Flip decision for a quad of four finite points: the edge a -> b shared by
// the triangles (a, b, c) and (b, a, d).  With an inverted (or flat) triangle:
// flip when one opposite vertex lies in the closed triangle formed by the edge
// and the other opposite vertex (Sec. 4.3, evaluated for both orderings);
// otherwise the Lawson flip when d is strictly inside the circumcircle of
// (a, b, c) (Sec. 4.1).
BD_HD int bd_flip_rule_quad(double ax, double ay, double bx, double by, double cx, double cy, double dx, double dy,
                            bool allow_inversion, bool *inverted) {
    const double o1 = bd_orient(ax, ay, bx, by, cx, cy);
    const double o2 = bd_orient(bx, by, ax, ay, dx, dy);
    if (o1 <= 0.0 || o2 <= 0.0) {
        if (inverted) *inverted = true;
        if (!allow_inversion) return BD_NOFLIP;
        bool f = bd_in_closed_tri(ax, ay, bx, by, cx, cy, dx, dy) || bd_in_closed_tri(ax, ay, bx, by, dx, dy, cx, cy);
        return f ? BD_FLIP_INVERSION : BD_NOFLIP;
    }
    return bd_incircle(ax, ay, bx, by, cx, cy, dx, dy) > 0.0 ? BD_FLIP_LAWSON : BD_NOFLIP;
}

// Flip decision for the edge a -> b shared by triangles (a, b, c) and
// (b, a, d), any of a, b, c, d possibly an infinite vertex (ids >= inf; a
// batch of independent triangulations has one infinite vertex each).
//   * Finite quad with an inverted (or flat) triangle: flip when one
//     opposite vertex lies in the closed triangle formed by the edge and the
//     other opposite vertex (Sec. 4.3, evaluated for both orderings).
//   * Finite quad, both triangles positive: Lawson flip when d is strictly
//     inside the circumcircle of (a, b, c) (Sec. 4.1).
//   * Edge to the infinite vertex: flip when its finite end is no longer a
//     convex hull corner (the hull chain turns right there).
//   * Hull edge with a ghost on one side: flip when the finite opposite
//     vertex has crossed to the outside of the hull edge.
// `allow_inversion` = false restricts the rule to valid triangulations.
// *inverted is set when a finite triangle of the quad is inverted or flat.
BD_HD int bd_flip_rule(int a, int b, int c, int d, int inf, const double *x, const double *y,
                       bool allow_inversion, bool *inverted = nullptr) {
    if (inverted) *inverted = false;
    if (b >= inf) return bd_orient(x[d], y[d], x[a], y[a], x[c], y[c]) < 0.0 ? BD_FLIP_INVERSION : BD_NOFLIP;
    if (a >= inf) return bd_orient(x[c], y[c], x[b], y[b], x[d], y[d]) < 0.0 ? BD_FLIP_INVERSION : BD_NOFLIP;
    if (c >= inf) {
        bool bad = bd_orient(x[b], y[b], x[a], y[a], x[d], y[d]) < 0.0;
        if (inverted) *inverted = bad;
        return bad ? BD_FLIP_INVERSION : BD_NOFLIP;
    }
    if (d >= inf) {
        bool bad = bd_orient(x[a], y[a], x[b], y[b], x[c], y[c]) < 0.0;
        if (inverted) *inverted = bad;
        return bad ? BD_FLIP_INVERSION : BD_NOFLIP;
    }
    return bd_flip_rule_quad(x[a], y[a], x[b], y[b], x[c], y[c], x[d], y[d], allow_inversion, inverted);
}

// bd_flip_rule with the four positions already loaded (an infinite vertex's
// coordinates are never read).
BD_HD int bd_flip_rule_xy(int a, int b, int c, int d, int inf, double ax, double ay, double bx, double by, double cx,
                          double cy, double dx, double dy, bool allow_inversion, bool *inverted = nullptr) {
    if (inverted) *inverted = false;
    if (b >= inf) return bd_orient(dx, dy, ax, ay, cx, cy) < 0.0 ? BD_FLIP_INVERSION : BD_NOFLIP;
    if (a >= inf) return bd_orient(cx, cy, bx, by, dx, dy) < 0.0 ? BD_FLIP_INVERSION : BD_NOFLIP;
    if (c >= inf) {
        bool bad = bd_orient(bx, by, ax, ay, dx, dy) < 0.0;
        if (inverted) *inverted = bad;
        return bad ? BD_FLIP_INVERSION : BD_NOFLIP;
    }
    if (d >= inf) {
        bool bad = bd_orient(ax, ay, bx, by, cx, cy) < 0.0;
        if (inverted) *inverted = bad;
        return bad ? BD_FLIP_INVERSION : BD_NOFLIP;
    }
    return bd_flip_rule_quad(ax, ay, bx, by, cx, cy, dx, dy, allow_inversion, inverted);
}

// Hard walls: reflect about the shifted wall [r, L - r], then clamp.
BD_HD double bd_wall(double c, double r, double L) {
#pragma clang fp contract(off)
    const double lo = r, hi = L - r;
    if (c < lo) c = 2.0 * lo - c;
    if (c > hi) c = 2.0 * hi - c;
    c = c < lo ? lo : c;
    c = c > hi ? hi : c;
    return c;
}

// Periodic box of side L (Sec. 2.1): a separation component from the nearest
// image (minimum-image convention, ties to even), and a coordinate folded into
// [0, L).
BD_HD double bd_min_image(double v, double L) {
#pragma clang fp contract(off)
    return v - L * rint(v / L);
}

BD_HD double bd_wrap(double c, double L) {
#pragma clang fp contract(off)
    const double r = c - L * floor(c / L);
    return r >= L ? r - L : r;
}

// Slope of bd_wall at c: -1 per reflection, 0 where the clamp acts.
BD_HD signed char bd_wall_slope(double c, double r, double L) {
#pragma clang fp contract(off)
    const double lo = r, hi = L - r;
    signed char sl = 1;
    if (c < lo) {
        c = 2.0 * lo - c;
        sl = -sl;
    }
    if (c > hi) {
        c = 2.0 * hi - c;
        sl = -sl;
    }
    return (c < lo || c > hi) ? (signed char)0 : sl;
}

// Half-edges of triangle t are 3t, 3t+1, 3t+2 in counter-clockwise order.
BD_HD int bd_next(int h) { return (h % 3 == 2) ? h - 2 : h + 1; }
BD_HD int bd_prev(int h) { return (h % 3 == 0) ? h + 2 : h - 1; }
