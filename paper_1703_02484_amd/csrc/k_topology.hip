// Device-resident Delaunay triangulation: parallel edge-flip repair (Sec. 4.1
// and 4.3) and overlap correction over Delaunay edges (Sec. 2.3, 4.4,
// Algorithm 2).
//
// Triangulation layout (SoA, ghosts included).  Vertices are the n disks
// (ids 0..n-1), the fixed frame points outside the walls (n..nv-1) and the
// infinite vertex (nv); T = 2 nv - 2 triangles.
//   he_v[h]     origin vertex of half-edge h; triangle t owns h = 3t..3t+2 CCW
//   he_twin[h]  opposite half-edge
//   vert_he[v]  one outgoing half-edge of vertex v
//
// One flip round is three launches:
//   eval   every candidate edge (all edges, or a worklist) applies the flip
//          rule; a flipping edge claims both of its triangles with a 64-bit
//          atomicMax of (round << 32 | ~edge): the newest round wins over stale
//          claims and, inside a round, the lowest edge id wins, independent of
//          scheduling.
//   apply  an edge that holds both claims rewrites its two triangles in place,
//          records where its four outer half-edges moved and stamps the two
//          triangles with the round.
//   fix    each flipped quad repairs the twin links of its outer half-edges
//          (through `moved` when the neighbour flipped in the same round) and
//          pushes the edges whose status may have changed to the next
//          worklist; a candidate that lost without any neighbour flipping
//          re-queues itself.
// The globally lowest candidate always wins both claims, so every round with a
// candidate makes progress.
#include <hip/hip_runtime.h>

#include "bd_internal.h"
#include "geom.h"

namespace bd {
namespace {

struct Topo {
    int n, inf, T;
    const double *x, *y, *xo, *yo, *rad;
    int *he_v, *he_twin, *vert_he;
    unsigned long long *claim;
    int *tri_stamp, *moved, *edge_stamp, *vstamp;
    int2 *cand;
    int *cand_won;
    int *wl_in, *wl_out;
    int *touched;
    double2 *newpos, *oldpos;
    int *ctr;
    unsigned long long *acc;
};

Topo topo_of(Sim &s) {
    Topo t;
    t.n = s.n;
    t.inf = s.inf;
    t.T = s.T;
    t.x = s.x;
    t.y = s.y;
    t.xo = s.xo;
    t.yo = s.yo;
    t.rad = s.rad;
    t.he_v = s.he_v;
    t.he_twin = s.he_twin;
    t.vert_he = s.vert_he;
    t.claim = s.claim;
    t.tri_stamp = s.tri_stamp;
    t.moved = s.moved;
    t.edge_stamp = s.edge_stamp;
    t.vstamp = s.vstamp;
    t.cand = s.cand;
    t.cand_won = s.cand_won;
    t.wl_in = s.wl[s.wl_cur];
    t.wl_out = s.wl[s.wl_cur ^ 1];
    t.touched = s.touched;
    t.newpos = s.newpos;
    t.oldpos = s.oldpos;
    t.ctr = s.ctr;
    t.acc = s.acc;
    return t;
}

// Range guards: a corrupt triangulation must never turn into an out-of-bounds
// access; it is reported through C_TOPO_ERR and repaired on the host.
__device__ __forceinline__ bool bad_he(const Topo &t, int h) { return (unsigned)h >= (unsigned)(3 * t.T); }
__device__ __forceinline__ bool bad_v(const Topo &t, int v) { return (unsigned)v > (unsigned)t.inf; }
__device__ __forceinline__ void topo_err(const Topo &t) { atomicAdd(&t.ctr[C_TOPO_ERR], 1); }

__device__ __forceinline__ unsigned long long claim_key(int round, int e) {
    return ((unsigned long long)(unsigned)round << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)e);
}

__device__ __forceinline__ void push_edge(const Topo &t, int e, int stamp) {
    if (atomicExch(&t.edge_stamp[e], stamp) != stamp) {
        int slot = atomicAdd(&t.ctr[C_WL_NEXT], 1);
        t.wl_out[slot] = e;
    }
}

// Evaluates the canonical edge h (h < twin) and, if it must flip, registers
// it as a candidate and claims its two triangles.
__device__ __forceinline__ void eval_edge(const Topo &t, int h, int tw, int round, bool reversal) {
    if (bad_he(t, tw)) return topo_err(t);
    const int t1 = h / 3, t2 = tw / 3;
    const int a = t.he_v[h], b = t.he_v[bd_next(h)], c = t.he_v[bd_prev(h)];
    const int d = t.he_v[bd_prev(tw)];
    if (bad_v(t, a) || bad_v(t, b) || bad_v(t, c) || bad_v(t, d)) return topo_err(t);
    if (reversal && a < t.n && b < t.n) {
        // Sec. 4.3: the pair passed through each other if the edge vector reversed
        double ox = t.xo[b] - t.xo[a], oy = t.yo[b] - t.yo[a];
        double mx = t.x[b] - t.x[a], my = t.y[b] - t.y[a];
        if (ox * mx + oy * my < 0.0) atomicAdd(&t.acc[A_REVERSALS], 1ull);
    }
    bool inverted = false;
    const int rule = bd_flip_rule(a, b, c, d, t.inf, t.x, t.y, true, &inverted);
    if (inverted) atomicAdd(&t.ctr[C_INVERTED], 1);
    if (rule == BD_NOFLIP) return;
    int slot = atomicAdd(&t.ctr[C_CAND], 1);
    t.cand[slot] = make_int2(h, t2 | (rule == BD_FLIP_INVERSION ? (int)0x80000000 : 0));
    const unsigned long long key = claim_key(round, h);
    atomicMax(&t.claim[t1], key);
    atomicMax(&t.claim[t2], key);
}

__global__ void k_flip_eval_full(Topo t, int round, int reversal) {
    int tri = blockIdx.x * blockDim.x + threadIdx.x;
    if (tri >= t.T) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        int h = 3 * tri + k;
        int tw = t.he_twin[h];
        if (h < tw) eval_edge(t, h, tw, round, reversal != 0);
    }
}

__global__ void k_flip_eval_list(Topo t, int round, int count) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= count) return;
    int h = t.wl_in[idx];
    if (bad_he(t, h)) return topo_err(t);
    int tw = t.he_twin[h];
    if (bad_he(t, tw)) return topo_err(t);
    if (tw < h) {
        int s = h;
        h = tw;
        tw = s;
    }
    eval_edge(t, h, tw, round, false);
}

__global__ void k_flip_apply(Topo t, int round, int ncand) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ncand) return;
    const int2 cd = t.cand[idx];
    const int h = cd.x, t1 = h / 3, t2 = cd.y & 0x7FFFFFFF;
    const unsigned long long key = claim_key(round, h);
    const bool won = t.claim[t1] == key && t.claim[t2] == key;
    t.cand_won[idx] = 0;
    if (!won) return;
    // the quad is owned by this thread: (a, b, c) = t1 from h, (b, a, d) = t2 from its twin
    const int hb = bd_next(h), hc = bd_prev(h);
    const int g = t.he_twin[h];
    if (g / 3 != t2) return topo_err(t);
    const int ga = bd_next(g), gd = bd_prev(g);
    const int a = t.he_v[h], b = t.he_v[hb], c = t.he_v[hc], d = t.he_v[gd];
    const int Thb = t.he_twin[hb], Thc = t.he_twin[hc], Tga = t.he_twin[ga], Tgd = t.he_twin[gd];
    if (bad_v(t, a) || bad_v(t, b) || bad_v(t, c) || bad_v(t, d) || bad_he(t, Thb) || bad_he(t, Thc) ||
        bad_he(t, Tga) || bad_he(t, Tgd))
        return topo_err(t);
    const int s1 = 3 * t1, s2 = 3 * t2;
    // new t1 = (c, a, d), new t2 = (d, b, c); the diagonal c-d is slot 2 of both
    t.he_v[s1 + 0] = c;
    t.he_v[s1 + 1] = a;
    t.he_v[s1 + 2] = d;
    t.he_v[s2 + 0] = d;
    t.he_v[s2 + 1] = b;
    t.he_v[s2 + 2] = c;
    t.he_twin[s1 + 0] = Thc;   // c -> a, old neighbour index (fixed in k_flip_fix)
    t.he_twin[s1 + 1] = Tga;   // a -> d
    t.he_twin[s1 + 2] = s2 + 2;
    t.he_twin[s2 + 0] = Tgd;   // d -> b
    t.he_twin[s2 + 1] = Thb;   // b -> c
    t.he_twin[s2 + 2] = s1 + 2;
    t.moved[hc] = s1 + 0;
    t.moved[ga] = s1 + 1;
    t.moved[gd] = s2 + 0;
    t.moved[hb] = s2 + 1;
    t.tri_stamp[t1] = round;
    t.tri_stamp[t2] = round;
    // every flip rewrites the outgoing half-edge of all four vertices, so each
    // entry stays valid whichever concurrent flip writes it last
    t.vert_he[a] = s1 + 1;
    t.vert_he[b] = s2 + 1;
    t.vert_he[c] = s1 + 0;
    t.vert_he[d] = s2 + 0;
    t.cand_won[idx] = 1;
    atomicAdd(&t.acc[A_FLIPS], 1ull);
    if (cd.y & (int)0x80000000) atomicAdd(&t.acc[A_INV_FLIPS], 1ull);
}

__global__ void k_flip_fix(Topo t, int round, int ncand) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ncand) return;
    const int2 cd = t.cand[idx];
    const int h = cd.x, t1 = h / 3, t2 = cd.y & 0x7FFFFFFF;
    const int next = round + 1;
    if (!t.cand_won[idx]) {
        if (t.tri_stamp[t1] != round && t.tri_stamp[t2] != round) push_edge(t, h, next);
        return;
    }
    const int outer[4] = {3 * t1 + 0, 3 * t1 + 1, 3 * t2 + 0, 3 * t2 + 1};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int nh = outer[k];
        const int o = t.he_twin[nh];
        if (bad_he(t, o)) {
            topo_err(t);
            continue;
        }
        int tw;
        if (t.tri_stamp[o / 3] == round) {
            tw = t.moved[o];
            if (bad_he(t, tw)) {
                topo_err(t);
                continue;
            }
            t.he_twin[nh] = tw;
        } else {
            tw = o;
            t.he_twin[o] = nh;
        }
        push_edge(t, nh < tw ? nh : tw, next);
    }
    const int d1 = 3 * t1 + 2, d2 = 3 * t2 + 2;
    push_edge(t, d1 < d2 ? d1 : d2, next);
}

__global__ void k_validate(Topo t) {
    int tri = blockIdx.x * blockDim.x + threadIdx.x;
    if (tri >= t.T) return;
    int a = t.he_v[3 * tri], b = t.he_v[3 * tri + 1], c = t.he_v[3 * tri + 2];
    if (bad_v(t, a) || bad_v(t, b) || bad_v(t, c)) {
        atomicAdd(&t.ctr[C_INVALID], 1);
        return topo_err(t);
    }
    if (a == t.inf || b == t.inf || c == t.inf) return;
    if (bd_orient(t.x[a], t.y[a], t.x[b], t.y[b], t.x[c], t.y[c]) <= 0.0) atomicAdd(&t.ctr[C_INVALID], 1);
}

// ---------------------------------------------------------------- overlaps
// Detect: every finite Delaunay edge with d < r_i + r_j (Algorithm 2 test,
// Sec. 2.3 contact distance generalised to r_i + r_j); both ends are queued
// once per round.
__device__ __forceinline__ void mark_touched(const Topo &t, int v, int stamp) {
    if (atomicExch(&t.vstamp[v], stamp) != stamp) {
        int slot = atomicAdd(&t.ctr[C_TOUCHED], 1);
        t.touched[slot] = v;
    }
}

__global__ void k_ovl_detect(Topo t, int stamp, double keep) {
#pragma clang fp contract(off)
    int tri = blockIdx.x * blockDim.x + threadIdx.x;
    int found = 0;
    if (tri < t.T) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            int h = 3 * tri + k;
            int tw = t.he_twin[h];
            if (h > tw) continue;
            int a = t.he_v[h], b = t.he_v[bd_next(h)];
            if (bad_v(t, a) || bad_v(t, b)) {
                topo_err(t);
                continue;
            }
            if (a >= t.n || b >= t.n) continue;   // frame points and the infinite vertex never overlap
            double dx = t.x[a] - t.x[b], dy = t.y[a] - t.y[b];
            double d = sqrt(dx * dx + dy * dy);
            if (d < (t.rad[a] + t.rad[b]) * keep) {
                ++found;
                mark_touched(t, a, stamp);
                mark_touched(t, b, stamp);
            }
        }
    }
    if (found) atomicAdd(&t.ctr[C_OVL_EDGES], found);
}

// Gather: for a queued vertex, sum the Jacobi displacement over its star
// (Sec. 2.3 displacement along the unit vector, factor f), starting at the
// neighbour of smallest id so the summation order is independent of flip
// history; truncate the sum to cap_frac * r (Sec. 4.4); reflect at the walls.
__global__ void k_ovl_gather(Topo t, int ntouched, double f, double cap_frac, double L, double keep) {
#pragma clang fp contract(off)
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ntouched) return;
    const int v = t.touched[idx];
    const double xv = t.x[v], yv = t.y[v], rv = t.rad[v];
    const int h0 = t.vert_he[v];
    if (bad_he(t, h0)) {
        topo_err(t);
        t.newpos[idx] = make_double2(xv, yv);
        return;
    }
    int best = h0, bestid = 0x7FFFFFFF;
    int h = h0;
    int guard = 0;
    do {
        int w = t.he_v[bd_next(h)];
        if (bad_v(t, w)) {
            topo_err(t);
            t.newpos[idx] = make_double2(xv, yv);
            return;
        }
        if (w != t.inf && w < bestid) {
            bestid = w;
            best = h;
        }
        h = t.he_twin[bd_prev(h)];
        if (bad_he(t, h) || ++guard > 4096) {
            atomicAdd(&t.ctr[C_STAR_OVF], 1);
            t.newpos[idx] = make_double2(xv, yv);
            return;
        }
    } while (h != h0);
    double sx = 0.0, sy = 0.0;
    h = best;
    do {
        int w = t.he_v[bd_next(h)];
        if (w < t.n) {
            double dx = xv - t.x[w], dy = yv - t.y[w];
            double d = sqrt(dx * dx + dy * dy);
            double contact = rv + t.rad[w];
            if (d < contact * keep) {
                double s = f * (contact - d) / d;
                sx += s * dx;
                sy += s * dy;
            }
        }
        h = t.he_twin[bd_prev(h)];
    } while (h != best);
    const double len = sqrt(sx * sx + sy * sy);
    const double cap = cap_frac * rv;
    if (len > cap) {
        double sc = cap / len;
        sx = sx * sc;
        sy = sy * sc;
        atomicAdd(&t.acc[A_CAP_HITS], 1ull);
    }
    t.newpos[idx] = make_double2(bd_wall(xv + sx, rv, L), bd_wall(yv + sy, rv, L));
}

// Apply: write the new positions and queue every edge of the moved vertex's
// triangles (incident edges and link edges) for the following flip repair.
__global__ void k_ovl_apply(Topo t, int ntouched, int next_round) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ntouched) return;
    const int v = t.touched[idx];
    const double2 np = t.newpos[idx];
    t.oldpos[idx] = make_double2(t.x[v], t.y[v]);
    ((double *)t.x)[v] = np.x;
    ((double *)t.y)[v] = np.y;
    const int h0 = t.vert_he[v];
    if (bad_he(t, h0)) return topo_err(t);
    int h = h0, guard = 0;
    do {
        int tw = t.he_twin[h];
        int l = bd_next(h);
        int lt = t.he_twin[l];
        if (bad_he(t, tw) || bad_he(t, lt)) return topo_err(t);
        push_edge(t, h < tw ? h : tw, next_round);
        push_edge(t, l < lt ? l : lt, next_round);
        h = t.he_twin[bd_prev(h)];
        if (bad_he(t, h)) return topo_err(t);
    } while (h != h0 && ++guard < 4096);
}

__global__ void k_scatter_oldpos(Topo t, int ntouched, double *xa, double *ya) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ntouched) return;
    const int v = t.touched[idx];
    xa[v] = t.oldpos[idx].x;
    ya[v] = t.oldpos[idx].y;
}

__global__ void k_interp(int n, int i, int k, const double *xa, const double *ya, const double *xb,
                         const double *yb, double *x, double *y) {
#pragma clang fp contract(off)
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    if (i == k) {
        x[v] = xb[v];
        y[v] = yb[v];
    } else {
        const double s = (double)i / (double)k;
        x[v] = xa[v] + s * (xb[v] - xa[v]);
        y[v] = ya[v] + s * (yb[v] - ya[v]);
    }
}

inline int nb256(int n) { return (n + 255) / 256; }

}  // namespace

void launch_flip_eval_full(Sim &s, int round, bool reversal) {
    Topo t = topo_of(s);
    hipLaunchKernelGGL(k_flip_eval_full, dim3(nb256(s.T)), dim3(256), 0, s.stream, t, round, reversal ? 1 : 0);
}

void launch_flip_eval_list(Sim &s, int round, int count) {
    if (count <= 0) return;
    Topo t = topo_of(s);
    hipLaunchKernelGGL(k_flip_eval_list, dim3(nb256(count)), dim3(256), 0, s.stream, t, round, count);
}

void launch_flip_apply(Sim &s, int round, int ncand) {
    if (ncand <= 0) return;
    Topo t = topo_of(s);
    hipLaunchKernelGGL(k_flip_apply, dim3(nb256(ncand)), dim3(256), 0, s.stream, t, round, ncand);
}

void launch_flip_fix(Sim &s, int round, int ncand) {
    if (ncand <= 0) return;
    Topo t = topo_of(s);
    hipLaunchKernelGGL(k_flip_fix, dim3(nb256(ncand)), dim3(256), 0, s.stream, t, round, ncand);
}

void launch_validate(Sim &s) {
    Topo t = topo_of(s);
    hipLaunchKernelGGL(k_validate, dim3(nb256(s.T)), dim3(256), 0, s.stream, t);
}

void launch_ovl_detect(Sim &s, int vstamp) {
    Topo t = topo_of(s);
    hipLaunchKernelGGL(k_ovl_detect, dim3(nb256(s.T)), dim3(256), 0, s.stream, t, vstamp, 1.0 - s.p.contact_tol);
}

void launch_ovl_gather(Sim &s, int ntouched) {
    if (ntouched <= 0) return;
    Topo t = topo_of(s);
    hipLaunchKernelGGL(k_ovl_gather, dim3(nb256(ntouched)), dim3(256), 0, s.stream, t, ntouched,
                       s.p.overlap_factor, s.p.cap_frac, s.p.L, 1.0 - s.p.contact_tol);
}

void launch_ovl_apply(Sim &s, int ntouched, int next_round) {
    if (ntouched <= 0) return;
    Topo t = topo_of(s);
    hipLaunchKernelGGL(k_ovl_apply, dim3(nb256(ntouched)), dim3(256), 0, s.stream, t, ntouched, next_round);
}

void launch_scatter_oldpos(Sim &s, int ntouched) {
    if (ntouched <= 0) return;
    Topo t = topo_of(s);
    hipLaunchKernelGGL(k_scatter_oldpos, dim3(nb256(ntouched)), dim3(256), 0, s.stream, t, ntouched, s.xa, s.ya);
}

void launch_interp(Sim &s, int i, int k) {
    hipLaunchKernelGGL(k_interp, dim3(nb256(s.n)), dim3(256), 0, s.stream, s.n, i, k, s.xa, s.ya, s.xb, s.yb, s.x,
                       s.y);
}

}  // namespace bd
