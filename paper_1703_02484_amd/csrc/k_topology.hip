// Device-resident Delaunay triangulation: parallel edge-flip repair (Sec. 4.1
// and 4.3) and overlap correction over Delaunay edges (Sec. 2.3, 4.4,
// Algorithm 2).
//
// Triangulation layout (SoA, ghosts included).  A handle holds R independent
// systems (R = 1 for one system).  Vertex ids: the disks of all systems
// (0..n-1, system by system), their fixed frame points outside the walls
// (n..nv-1), then one infinite vertex per system (nv..nv+R-1); system r has
// 2 nv_r - 2 triangles and no edge between two systems.
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
//
// Control.  Work counts live in the device control block `ctl` in per-round
// and per-overlap-round slots, so a whole step can be enqueued without the
// host reading anything back: every kernel reads its count from `ctl` and
// returns at once when the step has halted (an error or an exhausted budget,
// left for the host to finish) or the overlap loop is done.
#include <hip/hip_runtime.h>

#include "bd_internal.h"
#include "geom.h"

namespace bd {
namespace {

constexpr int kMaxGrid = 512;      // full scans over triangles that take per-workgroup atomics
constexpr int kScanGrid = 4096;    // full scans without them (many waves in flight hide the gathers' latency)
constexpr int kScanBlock = 1024;   // full scans with per-workgroup atomics: few workgroups, many waves
constexpr int kListGridMax = 256;  // worklist-driven launches (usually a few hundred items, often none)

struct Topo {
    int n, inf, nvert, T;   // disks, first infinite-vertex id, all vertex ids, triangles
    double P;               // > 0: periodic box of this side (torus triangulation, minimum-image geometry)
    double ru;              // > 0: every disk has this radius (a contact distance is 2 ru, radii are not loaded)
    const int *rep_of;      // replica of each disk
    const double *Lr;       // box side of each replica
    const double *x, *y, *xo, *yo, *rad;
    const double2 *xy;      // (x, y) pairs, kept equal to x, y: the gathers of other vertices' positions load these
    int *he_v, *he_twin, *vert_he;
    unsigned long long *claim;
    int *tri_stamp, *moved, *edge_stamp, *vstamp;
    int2 *cand;
    int *cand_won;
    int *wl0, *wl1;
    int *touched;           // [2][n], by overlap-round parity
    int *det_stamp, *fl_stamp, *fl, *vt_stamp, *vt;
    double2 *newpos, *oldpos;
    int *ctl;
    unsigned long long *acc;
    const StepBase *base;   // stamps passed to kernels are relative to base->rbase / base->vbase
    // adjoint tape (null unless a segment is being recorded)
    int *tev, *tecnt, *tenb;
    double2 *teold, *tedisp;
    signed char *tewf;
    int2 *tdir;
    int tent_base, tdir_base, tcap_ent, tcap_dir;
};

Topo topo_of(Sim &s) {
    Topo t;
    t.n = s.n;
    t.inf = s.inf;
    t.P = s.period;
    t.ru = s.rad_uni;
    t.nvert = s.inf + s.R;
    t.rep_of = s.rep_of;
    t.Lr = s.Lr;
    t.T = s.T;
    t.x = s.x;
    t.y = s.y;
    t.xy = s.xy;
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
    t.wl0 = s.wl[0];
    t.wl1 = s.wl[1];
    t.touched = s.touched;
    t.det_stamp = s.det_stamp;
    t.fl_stamp = s.fl_stamp;
    t.fl = s.fl;
    t.vt_stamp = s.vt_stamp;
    t.vt = s.vt;
    t.newpos = s.newpos;
    t.oldpos = s.oldpos;
    t.ctl = s.ctl;
    t.acc = s.acc;
    t.base = s.dbase;
    const Tape &tp = s.adj.tape;
    const bool rec = tp.on;
    t.tev = rec ? tp.ev : nullptr;
    t.tecnt = tp.ecnt;
    t.tenb = tp.enb;
    t.teold = tp.eold;
    t.tedisp = tp.edisp;
    t.tewf = tp.ewf;
    t.tdir = tp.dir;
    t.tent_base = tp.ent_base;
    t.tdir_base = tp.dir_base;
    t.tcap_ent = tp.cap_ent;
    t.tcap_dir = tp.cap_dir;
    return t;
}

__device__ __forceinline__ bool stopped(const int *ctl) { return (ctl[K_HALT] | ctl[K_DONE]) != 0; }
// Read of a counter that other workgroups of the running launch update with atomics.
__device__ __forceinline__ int ctl_read(const int *ctl, int i) {
    return __hip_atomic_load(ctl + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Disks queued by overlap round k (two buffers, so a round can read the previous round's list).
__device__ __forceinline__ int *touched_of(const Topo &t, int k) { return t.touched + (size_t)(k & 1) * t.n; }
__device__ __forceinline__ int *wl_of(const Topo &t, int slot) { return (slot & 1) ? t.wl1 : t.wl0; }

// Range guards: a corrupt triangulation must never turn into an out-of-bounds
// access; it is reported through K_TOPO and repaired on the host.
__device__ __forceinline__ bool bad_he(const Topo &t, int h) { return (unsigned)h >= (unsigned)(3 * t.T); }
__device__ __forceinline__ bool bad_v(const Topo &t, int v) { return (unsigned)v >= (unsigned)t.nvert; }
__device__ __forceinline__ void topo_err(const Topo &t) { atomicAdd(&t.ctl[K_TOPO], 1); }

// Geometry of the triangulation.  With walls the vertex positions are used as
// they are.  In a periodic box (P > 0) a triangle or a quad is read in the
// frame of its first vertex, every other vertex at its nearest image: every
// edge of the torus triangulation is far shorter than P / 2, so that image is
// the one the triangle spans.
__device__ __forceinline__ double sep_p(double v, double P) { return P > 0.0 ? bd_min_image(v, P) : v; }

__device__ __forceinline__ int flip_rule_of(const Topo &t, int a, int b, int c, int d, bool *inverted) {
    const double2 pa = t.xy[a], pb = t.xy[b], pc = t.xy[c], pd = t.xy[d];
    if (t.P <= 0.0) return bd_flip_rule_xy(a, b, c, d, t.inf, pa.x, pa.y, pb.x, pb.y, pc.x, pc.y, pd.x, pd.y, true, inverted);
    return bd_flip_rule_quad(0.0, 0.0, sep_p(pb.x - pa.x, t.P), sep_p(pb.y - pa.y, t.P), sep_p(pc.x - pa.x, t.P),
                             sep_p(pc.y - pa.y, t.P), sep_p(pd.x - pa.x, t.P), sep_p(pd.y - pa.y, t.P), true,
                             inverted);
}

__device__ __forceinline__ double orient_of(const Topo &t, int a, int b, int c) {
    const double2 pa = t.xy[a], pb = t.xy[b], pc = t.xy[c];
    if (t.P <= 0.0) return bd_orient(pa.x, pa.y, pb.x, pb.y, pc.x, pc.y);
    return bd_orient(0.0, 0.0, sep_p(pb.x - pa.x, t.P), sep_p(pb.y - pa.y, t.P), sep_p(pc.x - pa.x, t.P),
                     sep_p(pc.y - pa.y, t.P));
}

__device__ __forceinline__ unsigned long long claim_key(int round, int e) {
    return ((unsigned long long)(unsigned)round << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)e);
}

// Counters shared by the whole grid are updated once per wavefront: lanes
// that take a list position get consecutive ones from a single atomic, and
// event counts are summed over the wavefront first (same-address atomics
// serialise in the cache, and thousands of them per launch dominate a scan).
__device__ __forceinline__ int wave_reserve(int *counter, bool want) {
    const unsigned long long m = __ballot(want);
    if (m == 0) return -1;
    const int lane = __lane_id();
    const int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, leader);
    return want ? base + __popcll(m & ((1ull << lane) - 1ull)) : -1;
}

// Sum over the (fully active) wavefront, added by one lane.
__device__ __forceinline__ void wave_sum_add(int *counter, int v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (__lane_id() == 0 && v != 0) atomicAdd(counter, v);
}

__device__ __forceinline__ void wave_count(int *counter, bool event) {
    const unsigned long long m = __ballot(event);
    if (m != 0 && __lane_id() == __ffsll((unsigned long long)m) - 1) atomicAdd(counter, __popcll(m));
}

__device__ __forceinline__ void wave_count64(unsigned long long *counter, bool event) {
    const unsigned long long m = __ballot(event);
    if (m != 0 && __lane_id() == __ffsll((unsigned long long)m) - 1)
        atomicAdd(counter, (unsigned long long)__popcll(m));
}

// Whether the calling workgroup is the last of the grid to get here; every
// thread of every workgroup calls it once, at the end of the kernel, thread 0
// with released = true if it added to a counter the check reads.  The last
// one sees those counters complete (each adder releases before its ticket,
// the last taker acquires after) and resets the ticket for the next launch.
// An index error (K_TOPO) may reach the check late; the host reads it at the
// end of the step.  A check
// that would otherwise be a one-thread launch of its own runs there.
__device__ __forceinline__ bool last_workgroup(int *ctl, bool released) {
    __shared__ int last;
    // the counters a check reads are added by thread 0 of each workgroup: it
    // releases them before the ticket is taken (no acquire here, which would
    // drop the cache for the wavefronts still running)
    if (released) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        last = atomicAdd(&ctl[K_TICKET], 1) == (int)gridDim.x - 1;
        if (last) {
            atomicExch(&ctl[K_TICKET], 0);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
    }
    __syncthreads();
    return last != 0;
}

// Workgroup staging of worklist appends (LDS): lanes take stage positions
// with one LDS atomic per wavefront; at the end of the launch the workgroup
// reserves its entries on the shared counter with one atomic and copies them
// out.  Entries beyond the stage's capacity go to the list directly.
template <int CAP>
struct Stage {
    int buf[CAP];
    int cnt, base;
};

template <int CAP>
__device__ __forceinline__ void stage_init(Stage<CAP> &st) {
    if (threadIdx.x == 0) st.cnt = 0;
    __syncthreads();
}

// Every thread of the workgroup calls it once, at the end.
template <int CAP>
__device__ __forceinline__ void stage_flush(Stage<CAP> &st, int *counter, int *list) {
    __syncthreads();
    const int n = st.cnt < CAP ? st.cnt : CAP;
    if (threadIdx.x == 0 && n > 0) st.base = atomicAdd(counter, n);
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) list[st.base + i] = st.buf[i];
}

// Appends edge e to the worklist of round slot `slot` once per stamp.  The
// lanes of a wavefront that push at the same time take their positions with
// one atomic, on the workgroup's stage when there is one, else on the shared
// counter.
template <int CAP = 1>
__device__ __forceinline__ void push_edge(const Topo &t, int e, int stamp, int slot, Stage<CAP> *st = nullptr) {
    const bool fresh = atomicExch(&t.edge_stamp[e], stamp) != stamp;
    const unsigned long long m = __ballot(fresh);
    if (m == 0) return;
    const int lane = __lane_id();
    const int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(st ? &st->cnt : &t.ctl[K_WL + slot], __popcll(m));
    base = __shfl(base, leader);
    if (!fresh) return;
    const int pos = base + __popcll(m & ((1ull << lane) - 1ull));
    if (!st)
        wl_of(t, slot)[pos] = e;
    else if (pos < CAP)
        st->buf[pos] = e;
    else
        wl_of(t, slot)[atomicAdd(&t.ctl[K_WL + slot], 1)] = e;
}

// Is d already a neighbour of the finite vertex c?  A flip of (a, b) into
// (c, d) is only a flip if c-d is not an edge yet: on an embedded
// triangulation that always holds, but on a folded one (several inverted
// triangles around a disk that crossed more than one edge) the inverted-
// triangle rule can ask for it, and performing it would glue a duplicate edge.
// The star is read during evaluation, before any flip of the round.
__device__ __forceinline__ bool adjacent(const Topo &t, int c, int d) {
    const int h0 = t.vert_he[c];
    if (bad_he(t, h0)) return true;
    int h = h0, guard = 0;
    do {
        if (t.he_v[bd_next(h)] == d) return true;
        h = t.he_twin[bd_prev(h)];
        if (bad_he(t, h) || ++guard > 4096) return true;
    } while (h != h0);
    return false;
}

// Workgroup staging of flip candidates (LDS), for the full evaluation: lanes
// take stage positions with one LDS atomic per wavefront; at the end the
// workgroup reserves its candidates in the round's list with one atomic and
// copies them out (same-address atomics from every CU serialise).  Candidates
// beyond the stage's capacity go to the list directly.
template <int CAP>
struct CandStage {
    int2 buf[CAP];
    int cnt, base;
};

// The flip decision `rule` for the canonical edge h (twin tw, opposite vertices
// c and d): count an inverted quad; a flipping edge becomes a candidate of
// round slot `slot` and claims its two triangles.
template <int CAP = 1>
__device__ __forceinline__ void register_flip(const Topo &t, int h, int tw, int c, int d, int rule, bool inverted,
                                              int round, int slot, CandStage<CAP> *st = nullptr) {
    wave_count(&t.ctl[K_INVQ + slot], inverted);
    if (rule == BD_NOFLIP) return;
    if (c < t.inf ? adjacent(t, c, d) : adjacent(t, d, c)) {
        // blocked for now (c-d may disappear in this very round): look again next round
        push_edge(t, h, round + 1, slot + 1 == MAXR ? 0 : slot + 1);
        return;
    }
    const int t1 = h / 3, t2 = tw / 3;
    const int2 cand = make_int2(h, t2 | (rule == BD_FLIP_INVERSION ? (int)0x80000000 : 0));
    if (st) {
        const int p = wave_reserve(&st->cnt, true);
        if (p < CAP)
            st->buf[p] = cand;
        else
            t.cand[atomicAdd(&t.ctl[K_CAND + slot], 1)] = cand;
    } else {
        t.cand[wave_reserve(&t.ctl[K_CAND + slot], true)] = cand;
    }
    const unsigned long long key = claim_key(round, h);
    atomicMax(&t.claim[t1], key);
    atomicMax(&t.claim[t2], key);
}

// Evaluates the canonical edge h (h < twin) and, if it must flip, registers
// it as a candidate of round slot `slot` and claims its two triangles.
template <int CAP = 1>
__device__ __forceinline__ void eval_edge(const Topo &t, int h, int tw, int round, int slot, int reversal,
                                          CandStage<CAP> *st = nullptr) {
    if (bad_he(t, tw)) return topo_err(t);
    const int a = t.he_v[h], b = t.he_v[bd_next(h)], c = t.he_v[bd_prev(h)];
    const int d = t.he_v[bd_prev(tw)];
    if (bad_v(t, a) || bad_v(t, b) || bad_v(t, c) || bad_v(t, d)) return topo_err(t);
    if (reversal) {
        // Sec. 4.3: the pair passed through each other if the edge vector reversed
        bool rev = false;
        if (a < t.n && b < t.n) {
            const double ox = sep_p(t.xo[b] - t.xo[a], t.P), oy = sep_p(t.yo[b] - t.yo[a], t.P);
            const double2 pa = t.xy[a], pb = t.xy[b];
            const double mx = sep_p(pb.x - pa.x, t.P), my = sep_p(pb.y - pa.y, t.P);
            rev = ox * mx + oy * my < 0.0;
        }
        wave_count64(&t.acc[A_REVERSALS], rev);
        if (reversal == 2) wave_count(&t.ctl[K_REV], rev);
    }
    bool inverted = false;
    const int rule = flip_rule_of(t, a, b, c, d, &inverted);
    register_flip<CAP>(t, h, tw, c, d, rule, inverted, round, slot, st);
}

// Full evaluation after a move: one thread per triangle.  The triangle's three
// vertices and their positions are read once for its canonical edges (h <
// twin), and the far vertices of those edges are read together, so a thread
// issues its loads in three dependent waves instead of one chain per edge.
// The decisions are those of eval_edge.
constexpr int kEvalStage = 2048;
// Workgroup and grid of the full evaluation: 256-, 512- and 1024-thread workgroups with the same number
// of threads in the grid measured within 3 % of each other on 1M disks.
constexpr int kEvalBlock = 1024, kEvalGrid = 512;

// Every thread of the workgroup calls it once, at the end: the staged
// candidates are reserved in the round's list with one atomic and copied out.
template <int CAP>
__device__ __forceinline__ void cand_flush(const Topo &t, int slot, CandStage<CAP> &st) {
    __syncthreads();
    const int n = st.cnt < CAP ? st.cnt : CAP;
    if (threadIdx.x == 0 && n > 0) st.base = atomicAdd(&t.ctl[K_CAND + slot], n);
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) t.cand[st.base + i] = st.buf[i];
}

__global__ __launch_bounds__(kEvalBlock) void k_flip_eval_full(Topo t, int round, int slot, int reversal) {
    __shared__ CandStage<kEvalStage> st;
    if (stopped(t.ctl)) return;   // nothing in this launch writes the stop flags: uniform
    if (threadIdx.x == 0) st.cnt = 0;
    __syncthreads();
    round += t.base->rbase;
    for (int tri = xcd_block() * blockDim.x + threadIdx.x; tri < t.T; tri += gridDim.x * blockDim.x) {
        const int h0 = 3 * tri;
        int v[3], tw[3], d[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            v[k] = t.he_v[h0 + k];
            tw[k] = t.he_twin[h0 + k];
        }
        bool own[3], ok = true;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            own[k] = h0 + k < tw[k];
            if (own[k] && bad_he(t, tw[k])) own[k] = false, ok = false;
            d[k] = own[k] ? t.he_v[bd_prev(tw[k])] : v[k];
            if (bad_v(t, v[k]) || bad_v(t, d[k])) ok = false;
        }
        if (!ok) {
            topo_err(t);
            continue;
        }
        double px[3], py[3], qx[3], qy[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double2 pv = t.xy[v[k]];
            px[k] = pv.x;
            py[k] = pv.y;
            if (own[k]) {   // the far vertex of a canonical edge (the others are not evaluated here)
                const double2 pd = t.xy[d[k]];
                qx[k] = pd.x;
                qy[k] = pd.y;
            } else {
                qx[k] = pv.x;
                qy[k] = pv.y;
            }
        }
        if (reversal) {
            double ox[3], oy[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                ox[k] = t.xo[v[k]];
                oy[k] = t.yo[v[k]];
            }
            // Sec. 4.3: the pair passed through each other if the edge vector reversed
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int k1 = k == 2 ? 0 : k + 1;
                bool rev = false;
                if (own[k] && v[k] < t.n && v[k1] < t.n) {
                    const double rx = sep_p(ox[k1] - ox[k], t.P), ry = sep_p(oy[k1] - oy[k], t.P);
                    const double mx = sep_p(px[k1] - px[k], t.P), my = sep_p(py[k1] - py[k], t.P);
                    rev = rx * mx + ry * my < 0.0;
                }
                wave_count64(&t.acc[A_REVERSALS], rev);
                if (reversal == 2) wave_count(&t.ctl[K_REV], rev);
            }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (!own[k]) continue;
            const int k1 = k == 2 ? 0 : k + 1, k2 = k == 0 ? 2 : k - 1;
            const int a = v[k], b = v[k1], c = v[k2];
            bool inverted = false;
            int rule;
            if (t.P > 0.0) {
                const double ax = px[k], ay = py[k];
                rule = bd_flip_rule_quad(0.0, 0.0, sep_p(px[k1] - ax, t.P), sep_p(py[k1] - ay, t.P),
                                         sep_p(px[k2] - ax, t.P), sep_p(py[k2] - ay, t.P), sep_p(qx[k] - ax, t.P),
                                         sep_p(qy[k] - ay, t.P), true, &inverted);
            } else {
                rule = bd_flip_rule_xy(a, b, c, d[k], t.inf, px[k], py[k], px[k1], py[k1], px[k2], py[k2], qx[k],
                                       qy[k], true, &inverted);
            }
            register_flip<kEvalStage>(t, h0 + k, tw[k], c, d[k], rule, inverted, round, slot, &st);
        }
    }
    cand_flush(t, slot, st);
}

template <int CAP = 1>
__device__ __forceinline__ void flip_eval_list_body(const Topo &t, int round, int slot, int i0, int stride,
                                                    CandStage<CAP> *st = nullptr) {
    if (stopped(t.ctl)) return;
    round += t.base->rbase;
    const int count = t.ctl[K_WL + slot];
    const int *wl = wl_of(t, slot);
    for (int idx = i0; idx < count; idx += stride) {
        int h = wl[idx];
        if (bad_he(t, h)) {
            topo_err(t);
            continue;
        }
        int tw = t.he_twin[h];
        if (bad_he(t, tw)) {
            topo_err(t);
            continue;
        }
        if (tw < h) {
            int s = h;
            h = tw;
            tw = s;
        }
        eval_edge<CAP>(t, h, tw, round, slot, 0, st);
    }
}

__global__ void k_flip_eval_list(Topo t, int round, int slot) {
    __shared__ CandStage<kEvalStage> st;
    if (stopped(t.ctl)) return;   // nothing in this launch writes the stop flags: uniform
    if (threadIdx.x == 0) st.cnt = 0;
    __syncthreads();
    flip_eval_list_body<kEvalStage>(t, round, slot, xcd_block() * blockDim.x + threadIdx.x, gridDim.x * blockDim.x,
                                    &st);
    cand_flush(t, slot, st);
}

__device__ __forceinline__ void flip_apply_body(const Topo &t, int round, int slot, int i0, int stride) {
    round += t.base->rbase;
    if (stopped(t.ctl)) return;
    const int ncand = t.ctl[K_CAND + slot];
    const int epoch = t.ctl[K_FL_EPOCH];
    for (int idx = i0; idx < ncand; idx += stride) {
        const int2 cd = t.cand[idx];
        const int h = cd.x, t1 = h / 3, t2 = cd.y & 0x7FFFFFFF;
        const unsigned long long key = claim_key(round, h);
        const bool won = t.claim[t1] == key && t.claim[t2] == key;
        t.cand_won[idx] = 0;
        if (!won) continue;
        // the quad is owned by this thread: (a, b, c) = t1 from h, (b, a, d) = t2 from its twin
        const int hb = bd_next(h), hc = bd_prev(h);
        const int g = t.he_twin[h];
        if (g / 3 != t2) {
            topo_err(t);
            continue;
        }
        const int ga = bd_next(g), gd = bd_prev(g);
        const int a = t.he_v[h], b = t.he_v[hb], c = t.he_v[hc], d = t.he_v[gd];
        const int Thb = t.he_twin[hb], Thc = t.he_twin[hc], Tga = t.he_twin[ga], Tgd = t.he_twin[gd];
        if (bad_v(t, a) || bad_v(t, b) || bad_v(t, c) || bad_v(t, d) || bad_he(t, Thb) || bad_he(t, Thc) ||
            bad_he(t, Tga) || bad_he(t, Tgd)) {
            topo_err(t);
            continue;
        }
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
        // the new diagonal joins two disks that may never have been tested for overlap
        const int e = s1 + 2 < s2 + 2 ? s1 + 2 : s2 + 2;
        const bool new_e = atomicExch(&t.fl_stamp[e], epoch) != epoch;
        const int pe = wave_reserve(&t.ctl[K_FL_N], new_e);
        if (new_e) t.fl[pe] = e;
        // both rewritten triangles, for the validation that ends the repair
        const bool new_t1 = atomicExch(&t.vt_stamp[t1], epoch) != epoch;
        const bool new_t2 = atomicExch(&t.vt_stamp[t2], epoch) != epoch;
        const int p1 = wave_reserve(&t.ctl[K_VT_N], new_t1);
        const int p2 = wave_reserve(&t.ctl[K_VT_N], new_t2);
        if (new_t1) t.vt[p1] = t1;
        if (new_t2) t.vt[p2] = t2;
        wave_count64(&t.acc[A_FLIPS], true);
        wave_count64(&t.acc[A_INV_FLIPS], (cd.y & (int)0x80000000) != 0);
    }
}

__global__ void k_flip_apply(Topo t, int round, int slot) {
    flip_apply_body(t, round, slot, xcd_block() * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

template <int CAP = 1>
__device__ __forceinline__ void flip_fix_body(const Topo &t, int round, int slot, int i0, int stride,
                                              Stage<CAP> *st = nullptr) {
    round += t.base->rbase;
    if (stopped(t.ctl)) return;
    const int ncand = t.ctl[K_CAND + slot];
    const int next = round + 1;
    const int nslot = slot + 1 == MAXR ? 0 : slot + 1;   // slots are used circularly
    for (int idx = i0; idx < ncand; idx += stride) {
        const int2 cd = t.cand[idx];
        const int h = cd.x, t1 = h / 3, t2 = cd.y & 0x7FFFFFFF;
        if (!t.cand_won[idx]) {
            if (t.tri_stamp[t1] != round && t.tri_stamp[t2] != round) push_edge(t, h, next, nslot, st);
            continue;
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
            push_edge(t, nh < tw ? nh : tw, next, nslot, st);
        }
        const int d1 = 3 * t1 + 2, d2 = 3 * t2 + 2;
        push_edge(t, d1 < d2 ? d1 : d2, next, nslot, st);
    }
}

constexpr int kFixStage = 2048;

__global__ void k_flip_fix(Topo t, int round, int slot) {
    __shared__ Stage<kFixStage> st;
    if (stopped(t.ctl)) return;   // nothing in this launch writes the stop flags: uniform
    stage_init(st);
    flip_fix_body(t, round, slot, xcd_block() * blockDim.x + threadIdx.x, gridDim.x * blockDim.x, &st);
    const int nslot = slot + 1 == MAXR ? 0 : slot + 1;
    stage_flush(st, &t.ctl[K_WL + nslot], wl_of(t, nslot));
}

// Counts finite triangles that are not positively oriented after repair `rep`.
// inv: the repair's invalid-triangle counter, or a workgroup's share of it in LDS
__device__ __forceinline__ void validate_tri(const Topo &t, int tri, int *inv) {
    const int a = t.he_v[3 * tri], b = t.he_v[3 * tri + 1], c = t.he_v[3 * tri + 2];
    if (bad_v(t, a) || bad_v(t, b) || bad_v(t, c)) {
        atomicAdd(inv, 1);
        topo_err(t);
        return;
    }
    if (a >= t.inf || b >= t.inf || c >= t.inf) return;
    if (orient_of(t, a, b, c) <= 0.0) atomicAdd(inv, 1);
}

// After the repair that follows overlap round k the triangulation was valid
// before the round, so a triangle can only have lost its orientation if one
// of its disks moved in round k or a flip rewrote it: only those are checked
// (a triangle may be checked more than once; the count only has to be > 0).
__device__ __forceinline__ void validate_local_body(const Topo &t, int *inv, int k, int i0, int stride) {
    if (stopped(t.ctl)) return;
    const int nmoved = t.ctl[K_TOUCH + k];
    const int nvt = t.ctl[K_VT_N];
    const int *moved = touched_of(t, k);
    for (int idx = i0; idx < nmoved + nvt; idx += stride) {
        if (idx >= nmoved) {
            const int tri = t.vt[idx - nmoved];
            if ((unsigned)tri >= (unsigned)t.T) {
                topo_err(t);
                continue;
            }
            validate_tri(t, tri, inv);
            continue;
        }
        const int v = moved[idx];
        const int h0 = t.vert_he[v];
        if (bad_he(t, h0)) {
            topo_err(t);
            continue;
        }
        int h = h0, guard = 0;
        do {
            validate_tri(t, h / 3, inv);
            h = t.he_twin[bd_prev(h)];
            if (bad_he(t, h) || ++guard > 4096) {
                atomicAdd(inv, 1);
                topo_err(t);
                break;
            }
        } while (h != h0);
    }
}

// End of repair `rep` whose last round used slot `last`: halt the step when the
// repair did not finish inside its round budget or left an invalid triangle.
__device__ __forceinline__ void repair_check_body(int *ctl, int rep, int last) {
    if (stopped(ctl)) return;
    int reason = 0;
    if (ctl_read(ctl, K_TOPO) != 0)
        reason = HALT_TOPOLOGY;
    else if (ctl_read(ctl, K_REV) != 0)   // only ever set by a move whose reversals halve the step
        reason = HALT_REVERSAL;
    else if (ctl_read(ctl, K_CAND + last) != 0)
        reason = HALT_REPAIR_BUDGET;
    else if (ctl_read(ctl, K_INV + rep) != 0)
        reason = HALT_INVALID;
    if (reason) {
        ctl[K_REASON] = reason;
        ctl[K_STAGE] = rep;
        ctl[K_LAST] = last;
        ctl[K_HALT] = 1;
    }
}

// Validation of repair `rep`; with last >= 0 the last workgroup also runs the
// repair's check (last: slot of its final round).
// Adds a workgroup's count (in LDS) to a shared counter from thread 0; every
// thread calls it.  Returns true in thread 0 when it added something.
__device__ __forceinline__ bool add_block_count(int *counter, const int *block_count) {
    __syncthreads();
    if (threadIdx.x != 0 || *block_count == 0) return false;
    atomicAdd(counter, *block_count);
    return true;
}

__global__ __launch_bounds__(kScanBlock) void k_validate(Topo t, int rep, int last) {
    __shared__ int inv;
    if (stopped(t.ctl)) return;   // nothing in this launch writes the stop flags: uniform
    if (threadIdx.x == 0) inv = 0;
    __syncthreads();
    for (int tri = xcd_block() * blockDim.x + threadIdx.x; tri < t.T; tri += gridDim.x * blockDim.x)
        validate_tri(t, tri, &inv);
    const bool added = add_block_count(&t.ctl[K_INV + rep], &inv);
    if (last >= 0 && last_workgroup(t.ctl, added) && threadIdx.x == 0) repair_check_body(t.ctl, rep, last);
}

__global__ void k_validate_local(Topo t, int rep, int k, int last) {
    __shared__ int inv;
    if (stopped(t.ctl)) return;
    if (threadIdx.x == 0) inv = 0;
    __syncthreads();
    validate_local_body(t, &inv, k, xcd_block() * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
    const bool added = add_block_count(&t.ctl[K_INV + rep], &inv);
    if (last >= 0 && last_workgroup(t.ctl, added) && threadIdx.x == 0) repair_check_body(t.ctl, rep, last);
}

// ---------------------------------------------------------------- overlaps
// Detect: every Delaunay edge between two disks with d < (r_i + r_j)(1 - tol)
// (Algorithm 2 test, Sec. 2.3 contact distance); both ends are queued once
// per round.
// Queues disk v for overlap round k once per stamp; with a workgroup stage the
// position is taken in LDS (the stage is copied out at the end of the launch).
template <int CAP = 1>
__device__ __forceinline__ void mark_touched(const Topo &t, int v, int stamp, int k, Stage<CAP> *st = nullptr) {
    const bool fresh = atomicExch(&t.vstamp[v], stamp) != stamp;
    if (st) {
        const int pos = wave_reserve(&st->cnt, fresh);
        if (!fresh) return;
        if (pos < CAP)
            st->buf[pos] = v;
        else
            touched_of(t, k)[atomicAdd(&t.ctl[K_TOUCH + k], 1)] = v;
        return;
    }
    const int pos = wave_reserve(&t.ctl[K_TOUCH + k], fresh);
    if (fresh) touched_of(t, k)[pos] = v;
}

__device__ __forceinline__ void ovl_check_body(int *ctl, int k, int stamp, const StepBase *base);
__device__ __forceinline__ void final_check_body(int *ctl, int k);

// Check after detection k (check = 1), and the final check after the last
// budgeted detection (check = 2), run by the detection's last workgroup.
__device__ __forceinline__ void detect_checks(const Topo &t, int k, int stamp, int check, bool released) {
    if (check == 0 || !last_workgroup(t.ctl, released) || threadIdx.x != 0) return;
    ovl_check_body(t.ctl, k, stamp, t.base);
    if (check == 2) final_check_body(t.ctl, k);
}

// Full detection.  A step's first detection finds tens of thousands of
// overlapping pairs on a large system; the disks it marks are staged in the
// workgroup's LDS and copied out with one reservation on the shared counter
// per kDetStage entries, not one per wavefront and edge (same-address
// atomics from every CU serialise and dominated this scan).
constexpr int kDetBlock = kScanBlock;
constexpr int kDetStage = 16384;   // 64 KiB of LDS
constexpr int kDetPerIter = 6 * kDetBlock;   // at most two disks for each of three edges per thread

__device__ __forceinline__ void det_flush(const Topo &t, int k, int *buf, int &cnt, int &base) {
    // every thread of the workgroup is here, after a barrier
    if (threadIdx.x == 0) base = atomicAdd(&t.ctl[K_TOUCH + k], cnt);
    __syncthreads();
    int *out = touched_of(t, k) + base;
    for (int i = threadIdx.x; i < cnt; i += kDetBlock) out[i] = buf[i];
    __syncthreads();
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
}

// vrep >= 0: the same pass also validates every triangle for the repair in
// slot vrep (last round slot vlast), whose check the last workgroup runs
// before the detection's.
__global__ __launch_bounds__(kDetBlock) void k_ovl_detect(Topo t, int rstamp, double keep, int k, int check, int vrep,
                                                          int vlast) {
#pragma clang fp contract(off)
    __shared__ int buf[kDetStage];
    __shared__ int cnt, base, nfound, inv;
    if (stopped(t.ctl)) return;   // nothing in this launch writes the stop flags before its last workgroup
    const int stamp = rstamp + t.base->vbase;
    if (threadIdx.x == 0) {
        cnt = 0;
        nfound = 0;
        inv = 0;
    }
    __syncthreads();
    int found = 0;
    for (int t0 = xcd_block() * kDetBlock; t0 < t.T; t0 += gridDim.x * kDetBlock) {   // same trip count for the workgroup
        const int tri = t0 + threadIdx.x;
        if (tri < t.T) {
            // the triangle's vertices, positions and radii read once for its validation and its
            // canonical edges
            int v[3], tw[3];
            double px[3], py[3], pr[3];
            bool ok = true;
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                v[e] = t.he_v[3 * tri + e];
                tw[e] = t.he_twin[3 * tri + e];
                if (bad_v(t, v[e])) ok = false;
            }
            if (!ok) topo_err(t);
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                const bool fin = ok && v[e] < t.inf;
                const double2 pv = fin ? t.xy[v[e]] : make_double2(0.0, 0.0);
                px[e] = pv.x;
                py[e] = pv.y;
                pr[e] = fin ? (t.ru > 0.0 ? t.ru : t.rad[v[e]]) : 0.0;
            }
            if (vrep >= 0) {   // as validate_tri
                if (!ok) {
                    atomicAdd(&inv, 1);
                } else if (v[0] < t.inf && v[1] < t.inf && v[2] < t.inf) {
                    const double o = t.P > 0.0 ? bd_orient(0.0, 0.0, sep_p(px[1] - px[0], t.P), sep_p(py[1] - py[0], t.P),
                                                           sep_p(px[2] - px[0], t.P), sep_p(py[2] - py[0], t.P))
                                               : bd_orient(px[0], py[0], px[1], py[1], px[2], py[2]);
                    if (o <= 0.0) atomicAdd(&inv, 1);
                }
            }
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                const int h = 3 * tri + e;
                const int e1 = e == 2 ? 0 : e + 1;
                if (!ok || h > tw[e]) continue;
                const int a = v[e], b = v[e1];
                if (a >= t.n || b >= t.n) continue;
                const double dx = sep_p(px[e] - px[e1], t.P), dy = sep_p(py[e] - py[e1], t.P);
                const double d = sqrt(dx * dx + dy * dy);
                if (d < (pr[e] + pr[e1]) * keep) {
                    ++found;
                    const bool fa = atomicExch(&t.vstamp[a], stamp) != stamp;
                    const bool fb = atomicExch(&t.vstamp[b], stamp) != stamp;
                    if (fa || fb) {
                        int p = atomicAdd(&cnt, (fa ? 1 : 0) + (fb ? 1 : 0));
                        if (fa) buf[p++] = a;
                        if (fb) buf[p] = b;
                    }
                }
            }
        }
        __syncthreads();
        if (cnt > kDetStage - kDetPerIter) det_flush(t, k, buf, cnt, base);
    }
    for (int off = 32; off > 0; off >>= 1) found += __shfl_xor(found, off);
    if (__lane_id() == 0 && found) atomicAdd(&nfound, found);
    __syncthreads();
    if (cnt > 0) det_flush(t, k, buf, cnt, base);
    const bool a_ovl = threadIdx.x == 0 && nfound != 0;
    if (a_ovl) atomicAdd(&t.ctl[K_OVL + k], nfound);
    const bool a_inv = vrep >= 0 && add_block_count(&t.ctl[K_INV + vrep], &inv);
    if (check == 0) return;
    if (last_workgroup(t.ctl, a_ovl || a_inv) && threadIdx.x == 0) {
        if (vrep >= 0) repair_check_body(t.ctl, vrep, vlast);
        ovl_check_body(t.ctl, k, rstamp, t.base);
        if (check == 2) final_check_body(t.ctl, k);
    }
}

// Detection after overlap round kprev of the same step.  A Delaunay edge can
// only overlap now if one of its disks moved in round kprev (every disk of an
// edge that overlapped at round kprev's detection moved) or if a flip since
// that detection created it; every other edge was tested then and neither of
// its disks has moved.  So only the stars of the disks moved by round kprev
// and the flipped list are tested, each edge once (det_stamp).
template <int CAP = 1>
__device__ __forceinline__ void detect_edge(const Topo &t, int h, int stamp, double keep, int k, int &found,
                                            Stage<CAP> *st = nullptr) {
    const int tw = t.he_twin[h];
    if (bad_he(t, tw)) return topo_err(t);
    const int e = h < tw ? h : tw;
    if (atomicExch(&t.det_stamp[e], stamp) == stamp) return;
    const int a = t.he_v[e], b = t.he_v[bd_next(e)];
    if (bad_v(t, a) || bad_v(t, b)) return topo_err(t);
    if (a >= t.n || b >= t.n) return;
    const double2 pa = t.xy[a], pb = t.xy[b];
    const double dx = sep_p(pa.x - pb.x, t.P), dy = sep_p(pa.y - pb.y, t.P);
    const double d = sqrt(dx * dx + dy * dy);
    if (d < (t.ru > 0.0 ? t.ru + t.ru : t.rad[a] + t.rad[b]) * keep) {
        ++found;
        mark_touched(t, a, stamp, k, st);
        mark_touched(t, b, stamp, k, st);
    }
}

// Returns the overlapping edges this thread found (the caller adds them to K_OVL + k).
__device__ __forceinline__ int ovl_detect_local_body(const Topo &t, int stamp, double keep, int k, int kprev, int i0, int stride) {
#pragma clang fp contract(off)
    if (stopped(t.ctl)) return 0;
    stamp += t.base->vbase;
    const int nprev = t.ctl[K_TOUCH + kprev];
    const int nfl = t.ctl[K_FL_N];
    const int *prev = touched_of(t, kprev);
    int found = 0;
    for (int idx = i0; idx < nprev + nfl; idx += stride) {
        if (idx >= nprev) {
            const int e = t.fl[idx - nprev];
            if (bad_he(t, e)) {
                topo_err(t);
                continue;
            }
            detect_edge(t, e, stamp, keep, k, found);
            continue;
        }
        const int v = prev[idx];
        const int h0 = t.vert_he[v];
        if (bad_he(t, h0)) {
            topo_err(t);
            continue;
        }
        int h = h0, guard = 0;
        do {
            detect_edge(t, h, stamp, keep, k, found);
            h = t.he_twin[bd_prev(h)];
            if (bad_he(t, h) || ++guard > 4096) {
                topo_err(t);
                break;
            }
        } while (h != h0);
    }
    return found;
}

// The validation of the repair after overlap round k fused with the next
// detection (round knew): both walk the stars of the disks round k moved, so
// one walk checks each triangle's orientation and tests each edge; then the
// triangles flips rewrote (validation) and the diagonals they created
// (detection).  The last workgroup runs the repair's check, then the
// detection's (check = 1) and the final check (check = 2).  On a repair that
// fails its check the detection's marks are never read: the host continues
// with rounds of its own slots and stamps.
// Body: inv is the repair's invalid-triangle counter, or a workgroup's share
// of it in LDS; the stamp st is absolute.  Returns the overlapping edges this thread found (the caller adds them
// to K_OVL + knew).
template <int CAP = 1>
__device__ __forceinline__ int validate_detect_local_body(const Topo &t, int *inv, int k, int st, double keep,
                                                          int knew, int i0, int stride, Stage<CAP> *stage = nullptr) {
#pragma clang fp contract(off)
    const int nmoved = t.ctl[K_TOUCH + k];
    const int nvt = t.ctl[K_VT_N];
    const int nfl = t.ctl[K_FL_N];
    const int *moved = touched_of(t, k);
    int found = 0;
    for (int idx = i0; idx < nmoved + nvt + nfl; idx += stride) {
        if (idx >= nmoved + nvt) {
            const int e = t.fl[idx - nmoved - nvt];
            if (bad_he(t, e)) {
                topo_err(t);
                continue;
            }
            detect_edge(t, e, st, keep, knew, found, stage);
            continue;
        }
        if (idx >= nmoved) {
            const int tri = t.vt[idx - nmoved];
            if ((unsigned)tri >= (unsigned)t.T) {
                topo_err(t);
                continue;
            }
            validate_tri(t, tri, inv);
            continue;
        }
        const int v = moved[idx];
        const int h0 = t.vert_he[v];
        if (bad_he(t, h0)) {
            topo_err(t);
            continue;
        }
        int h = h0, guard = 0;
        do {
            validate_tri(t, h / 3, inv);
            detect_edge(t, h, st, keep, knew, found, stage);
            h = t.he_twin[bd_prev(h)];
            if (bad_he(t, h) || ++guard > 4096) {
                atomicAdd(inv, 1);
                topo_err(t);
                break;
            }
        } while (h != h0);
    }
    return found;
}

constexpr int kTouchStage = 2048;

__global__ void k_validate_detect_local(Topo t, int rep, int k, int last, int stamp, double keep, int knew,
                                        int check) {
    __shared__ int inv, nfound;
    __shared__ Stage<kTouchStage> st;
    if (stopped(t.ctl)) return;   // nothing in this launch writes the stop flags before its last workgroup
    if (threadIdx.x == 0) {
        inv = 0;
        nfound = 0;
    }
    stage_init(st);
    int found = validate_detect_local_body(t, &inv, k, stamp + t.base->vbase, keep, knew,
                                           xcd_block() * blockDim.x + threadIdx.x, gridDim.x * blockDim.x, &st);
    stage_flush(st, &t.ctl[K_TOUCH + knew], touched_of(t, knew));
    for (int off = 32; off > 0; off >>= 1) found += __shfl_xor(found, off);
    if (__lane_id() == 0 && found) atomicAdd(&nfound, found);
    const bool a1 = add_block_count(&t.ctl[K_INV + rep], &inv);
    const bool a2 = add_block_count(&t.ctl[K_OVL + knew], &nfound);
    if (last_workgroup(t.ctl, a1 || a2) && threadIdx.x == 0) {
        repair_check_body(t.ctl, rep, last);
        ovl_check_body(t.ctl, knew, stamp, t.base);
        if (check == 2) final_check_body(t.ctl, knew);
    }
}

__global__ void k_ovl_detect_local(Topo t, int stamp, double keep, int k, int kprev, int check) {
    __shared__ int nfound;
    if (stopped(t.ctl)) return;
    if (threadIdx.x == 0) nfound = 0;
    __syncthreads();
    int found = ovl_detect_local_body(t, stamp, keep, k, kprev, xcd_block() * blockDim.x + threadIdx.x,
                                      gridDim.x * blockDim.x);
    for (int off = 32; off > 0; off >>= 1) found += __shfl_xor(found, off);
    if (__lane_id() == 0 && found) atomicAdd(&nfound, found);
    const bool added = add_block_count(&t.ctl[K_OVL + k], &nfound);
    detect_checks(t, k, stamp, check, added);
}

// Overlap round k found nothing: the overlap loop of this step is done.  The
// flipped list restarts for the edges flipped after this detection.
__device__ __forceinline__ void ovl_check_body(int *ctl, int k, int stamp, const StepBase *base) {
    if (stopped(ctl)) return;
    ctl[K_FL_N] = 0;
    ctl[K_VT_N] = 0;
    ctl[K_FL_EPOCH] = stamp + base->vbase;
    if (ctl_read(ctl, K_TOPO) != 0) {
        ctl[K_REASON] = HALT_TOPOLOGY;
        ctl[K_STAGE] = k;
        ctl[K_HALT] = 1;
        return;
    }
    if (ctl_read(ctl, K_OVL + k) == 0)
        ctl[K_DONE] = 1;
    else
        ctl[K_OVL_ROUNDS] = k + 1;
}

// After the last budgeted round: overlaps remain, the host continues.
__device__ __forceinline__ void final_check_body(int *ctl, int k) {
    if (stopped(ctl)) return;
    ctl[K_REASON] = HALT_OVERLAP_BUDGET;
    ctl[K_STAGE] = k;
    ctl[K_HALT] = 1;
}

// Gather: for a queued disk, sum the Jacobi displacement over its star
// (Sec. 2.3 displacement along the unit vector, factor f), starting at the
// neighbour of smallest id so the summation order is independent of flip
// history; truncate the sum to cap_frac * r (Sec. 4.4); reflect at the walls
// (fold into the box when periodic).  The star is walked once: each
// neighbour's contribution is kept in registers (stars of up to kStarCache
// neighbours) and the sum is then folded in the canonical order with static
// indices; a larger star is walked a second time in that order.
constexpr int kStarCache = 10;

__device__ __forceinline__ void ovl_gather_body(const Topo &t, int k, double f, double cap_frac, double keep, int i0, int stride) {
#pragma clang fp contract(off)
    if (stopped(t.ctl)) return;
    const int ntouched = t.ctl[K_TOUCH + k];
    const int *touched = touched_of(t, k);
    for (int idx = i0; idx < ntouched; idx += stride) {
        const int v = touched[idx];
        const double2 pv = t.xy[v];
        const double xv = pv.x, yv = pv.y, rv = t.ru > 0.0 ? t.ru : t.rad[v];
        const double L = t.Lr[t.rep_of[v]];
        t.newpos[idx] = make_double2(xv, yv);
        const int h0 = t.vert_he[v];
        if (bad_he(t, h0)) {
            topo_err(t);
            continue;
        }
        // walk: neighbour ids and contributions (0 for a non-overlapping or non-disk neighbour)
        int nid[kStarCache];
        double cxs[kStarCache], cys[kStarCache];
        int best = h0, bestid = 0x7FFFFFFF, bestpos = 0, deg = 0;
        int h = h0;
        int guard = 0;
        bool broken = false;
#pragma unroll
        for (int q = 0; q < kStarCache; ++q) {
            nid[q] = -1;
            cxs[q] = 0.0;
            cys[q] = 0.0;
        }
        do {
            const int w = t.he_v[bd_next(h)];
            if (bad_v(t, w)) {
                broken = true;
                break;
            }
            if (w < t.inf && w < bestid) {
                bestid = w;
                best = h;
                bestpos = deg;
            }
            if (deg < kStarCache && w < t.n) {
                const double2 pw = t.xy[w];
                const double dx = sep_p(xv - pw.x, t.P), dy = sep_p(yv - pw.y, t.P);
                const double d = sqrt(dx * dx + dy * dy);
                const double contact = rv + (t.ru > 0.0 ? t.ru : t.rad[w]);
                double cx = 0.0, cy = 0.0;
                int id = -1;
                if (d < contact * keep) {
                    const double sc = f * (contact - d) / d;
                    cx = sc * dx;
                    cy = sc * dy;
                    id = w;
                }
#pragma unroll
                for (int q = 0; q < kStarCache; ++q)
                    if (q == deg) {
                        nid[q] = id;
                        cxs[q] = cx;
                        cys[q] = cy;
                    }
            }
            ++deg;
            h = t.he_twin[bd_prev(h)];
            if (bad_he(t, h) || ++guard > 4096) {
                broken = true;
                break;
            }
        } while (h != h0);
        if (broken) {
            topo_err(t);
            atomicAdd(&t.ctl[K_STAR], 1);
            continue;
        }
        // adjoint tape: entry of this disk in this round
        const bool rec = t.tev != nullptr;
        const int e = rec ? t.tent_base + t.ctl[K_TAPE_ENT] + idx : 0;
        const bool room = rec && e < t.tcap_ent;
        if (rec && !room) atomicOr(&t.ctl[K_TAPE_OVF], 1);
        int na = 0;
        double sx = 0.0, sy = 0.0;
        if (deg <= kStarCache) {
            // canonical order: positions bestpos .. deg-1, then 0 .. bestpos-1
#pragma unroll
            for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
                for (int q = 0; q < kStarCache; ++q) {
                    const bool in = pass == 0 ? (q >= bestpos && q < deg) : (q < bestpos);
                    if (in && nid[q] >= 0) {
                        sx += cxs[q];
                        sy += cys[q];
                        if (room && na < MAXACT) t.tenb[(size_t)e * MAXACT + na] = nid[q];
                        ++na;
                    }
                }
            }
        } else {
            h = best;
            do {
                int w = t.he_v[bd_next(h)];
                if (w < t.n) {
                    const double2 pw = t.xy[w];
                    double dx = sep_p(xv - pw.x, t.P), dy = sep_p(yv - pw.y, t.P);
                    double d = sqrt(dx * dx + dy * dy);
                    double contact = rv + (t.ru > 0.0 ? t.ru : t.rad[w]);
                    if (d < contact * keep) {
                        double sc = f * (contact - d) / d;
                        sx += sc * dx;
                        sy += sc * dy;
                        if (room && na < MAXACT) t.tenb[(size_t)e * MAXACT + na] = w;
                        ++na;
                    }
                }
                h = t.he_twin[bd_prev(h)];
            } while (h != best);
        }
        if (room) {
            if (na > MAXACT) atomicOr(&t.ctl[K_TAPE_OVF], 2);
            t.tev[e] = v;
            t.tecnt[e] = na < MAXACT ? na : MAXACT;
            t.teold[e] = make_double2(xv, yv);
            t.tedisp[e] = make_double2(sx, sy);
        }
        const double len = sqrt(sx * sx + sy * sy);
        const double cap = cap_frac * rv;
        if (len > cap) {
            double sc = cap / len;
            sx = sx * sc;
            sy = sy * sc;
            wave_count64(&t.acc[A_CAP_HITS], true);
        }
        if (room) {
            t.tewf[2 * (size_t)e] = bd_wall_slope(xv + sx, rv, L);
            t.tewf[2 * (size_t)e + 1] = bd_wall_slope(yv + sy, rv, L);
        }
        if (t.P > 0.0)
            t.newpos[idx] = make_double2(bd_wrap(xv + sx, t.P), bd_wrap(yv + sy, t.P));
        else
            t.newpos[idx] = make_double2(bd_wall(xv + sx, rv, L), bd_wall(yv + sy, rv, L));
    }
}

__global__ void k_ovl_gather(Topo t, int k, double f, double cap_frac, double keep) {
    ovl_gather_body(t, k, f, cap_frac, keep, xcd_block() * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

// Apply: write the new positions (keeping the old ones for a replay) and queue
// every edge of the moved disk's triangles (incident and link edges) as the
// worklist of round slot `slot`, the first round of the following repair.
template <int CAP = 1>
__device__ __forceinline__ void ovl_apply_body(const Topo &t, int k, int next_round, int slot, int i0, int stride,
                                               Stage<CAP> *st = nullptr) {
    if (stopped(t.ctl)) return;
    next_round += t.base->rbase;
    const int ntouched = t.ctl[K_TOUCH + k];
    if (t.tev != nullptr && i0 == 0) {
        // adjoint tape: close the round's entries (written by the gather)
        const int di = t.tdir_base + t.ctl[K_TAPE_DIR];
        if (di < t.tcap_dir)
            t.tdir[di] = make_int2(t.tent_base + t.ctl[K_TAPE_ENT], ntouched);
        else
            atomicOr(&t.ctl[K_TAPE_OVF], 1);
        t.ctl[K_TAPE_ENT] += ntouched;
        t.ctl[K_TAPE_DIR] += 1;
    }
    const int *touched = touched_of(t, k);
    for (int idx = i0; idx < ntouched; idx += stride) {
        const int v = touched[idx];
        const double2 np = t.newpos[idx];
        t.oldpos[idx] = t.xy[v];
        ((double *)t.x)[v] = np.x;
        ((double *)t.y)[v] = np.y;
        ((double2 *)t.xy)[v] = np;
        const int h0 = t.vert_he[v];
        if (bad_he(t, h0)) {
            topo_err(t);
            continue;
        }
        int h = h0, guard = 0;
        do {
            int tw = t.he_twin[h];
            int l = bd_next(h);
            int lt = t.he_twin[l];
            if (bad_he(t, tw) || bad_he(t, lt)) {
                topo_err(t);
                break;
            }
            push_edge(t, h < tw ? h : tw, next_round, slot, st);
            push_edge(t, l < lt ? l : lt, next_round, slot, st);
            h = t.he_twin[bd_prev(h)];
            if (bad_he(t, h)) {
                topo_err(t);
                break;
            }
        } while (h != h0 && ++guard < 4096);
    }
}

constexpr int kApplyStage = 4096;

__global__ void k_ovl_apply(Topo t, int k, int next_round, int slot) {
    __shared__ Stage<kApplyStage> st;
    if (stopped(t.ctl)) return;
    stage_init(st);
    ovl_apply_body(t, k, next_round, slot, xcd_block() * blockDim.x + threadIdx.x, gridDim.x * blockDim.x, &st);
    stage_flush(st, &t.ctl[K_WL + slot], wl_of(t, slot));
}

// The overlap rounds after the first detection in one workgroup: each phase
// is the body of the corresponding kernel run with the workgroup's threads,
// and a barrier separates phases (workgroup-scope release/acquire, so every
// thread sees the previous phase's writes).  Halts follow the same rules.
constexpr int kTailBlock = 1024;

// In one workgroup, after a barrier: true when flip round `slot` has nothing
// left to do, before its evaluation (empty worklist) or after it (no
// candidate).  A round without a candidate queues no edge, so every later
// round of the repair would find an empty worklist as well: leaving the loop
// there gives the same result as running the remaining rounds.  The counters
// were last written by atomics before the barrier and are not written again
// before the decision, so every thread reads the same value.
__device__ __forceinline__ bool rounds_done(const Topo &t, int slot, bool evaluated) {
    return ctl_read(t.ctl, (evaluated ? K_CAND : K_WL) + slot) == 0;
}

__global__ __launch_bounds__(kTailBlock) void k_tail(Topo t, TailPlan p) {
    const int i0 = threadIdx.x, stride = blockDim.x;
#define TAIL_SYNC()                  \
    do {                             \
        __syncthreads();             \
        if (stopped(t.ctl)) return;  \
        __syncthreads();             \
    } while (0)
    TAIL_SYNC();
    for (int j = 0; j < p.nover; ++j) {
        const int k = p.k[j];
        ovl_gather_body(t, k, p.f, p.cap_frac, p.keep, i0, stride);
        TAIL_SYNC();
        ovl_apply_body(t, k, p.next_round[j], p.slot0[j], i0, stride);
        TAIL_SYNC();
        int last = -1;
        for (int r = 0; r < p.rounds[j]; ++r) {
            int slot = p.slot0[j] + r;
            if (slot >= MAXR) slot -= MAXR;
            const int round = p.next_round[j] + r;
            last = slot;
            if (rounds_done(t, slot, false)) break;
            flip_eval_list_body(t, round, slot, i0, stride);
            TAIL_SYNC();
            if (rounds_done(t, slot, true)) break;
            flip_apply_body(t, round, slot, i0, stride);
            TAIL_SYNC();
            flip_fix_body(t, round, slot, i0, stride);
            TAIL_SYNC();
        }
        // this repair's validation with the next round's detection, one walk
        // over the stars of the disks round k moved; then the repair's check
        // and the detection's, as the last workgroup of the fused launch does
        const int knew = p.k[j + 1];
        wave_sum_add(&t.ctl[K_OVL + knew],
                     validate_detect_local_body(t, &t.ctl[K_INV + p.rep[j]], k, p.stamp[j + 1] + t.base->vbase,
                                                p.keep, knew, i0, stride));
        __syncthreads();
        if (i0 == 0) {
            repair_check_body(t.ctl, p.rep[j], last);
            ovl_check_body(t.ctl, knew, p.stamp[j + 1], t.base);
            if (j + 1 == p.nover) final_check_body(t.ctl, knew);
        }
        TAIL_SYNC();
    }
#undef TAIL_SYNC
}

// Flip rounds [round0, round0 + rounds) of a repair in one workgroup, from
// slot slot0 on.  first_evaluated: the first round's evaluation already ran in
// a launch of many workgroups (the repair after the move scans every edge), so
// it starts with that round's apply; otherwise with the evaluation of the
// worklist in slot0.  The loop ends at the first round with nothing to do.
__global__ __launch_bounds__(kTailBlock) void k_repair_rounds(Topo t, int round0, int slot0, int rounds,
                                                              int first_evaluated) {
    const int i0 = threadIdx.x, stride = blockDim.x;
#define TAIL_SYNC()                  \
    do {                             \
        __syncthreads();             \
        if (stopped(t.ctl)) return;  \
        __syncthreads();             \
    } while (0)
    TAIL_SYNC();
    for (int r = 0; r < rounds; ++r) {
        int slot = slot0 + r;
        if (slot >= MAXR) slot -= MAXR;
        const int round = round0 + r;
        if (r > 0 || !first_evaluated) {
            if (rounds_done(t, slot, false)) break;
            flip_eval_list_body(t, round, slot, i0, stride);
            TAIL_SYNC();
        }
        if (rounds_done(t, slot, true)) break;
        flip_apply_body(t, round, slot, i0, stride);
        TAIL_SYNC();
        flip_fix_body(t, round, slot, i0, stride);
        TAIL_SYNC();
    }
#undef TAIL_SYNC
}

// Topology snapshot before a repair (skipped once the step has stopped, so the
// snapshot of the failing repair survives).
__global__ void k_snapshot(Topo t, int *snap_v, int *snap_twin, int *snap_vh, int nvh, int vec) {
    if (stopped(t.ctl)) return;
    const int H = 3 * t.T;
    const int H4 = vec ? H / 4 : 0, N4 = vec ? nvh / 4 : 0;   // 16-byte copies when aligned, then the tails
    const int stride = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < H4; i += stride) {
        reinterpret_cast<int4 *>(snap_v)[i] = reinterpret_cast<const int4 *>(t.he_v)[i];
        reinterpret_cast<int4 *>(snap_twin)[i] = reinterpret_cast<const int4 *>(t.he_twin)[i];
        if (i < N4) reinterpret_cast<int4 *>(snap_vh)[i] = reinterpret_cast<const int4 *>(t.vert_he)[i];
    }
    for (int i = 4 * H4 + blockIdx.x * blockDim.x + threadIdx.x; i < H; i += stride) {
        snap_v[i] = t.he_v[i];
        snap_twin[i] = t.he_twin[i];
    }
    for (int i = 4 * N4 + blockIdx.x * blockDim.x + threadIdx.x; i < nvh; i += stride) snap_vh[i] = t.vert_he[i];
}

__global__ void k_scatter_oldpos(Topo t, int k, double *xa, double *ya) {
    const int ntouched = t.ctl[K_TOUCH + k];
    const int *touched = touched_of(t, k);
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < ntouched; idx += gridDim.x * blockDim.x) {
        const int v = touched[idx];
        xa[v] = t.oldpos[idx].x;
        ya[v] = t.oldpos[idx].y;
    }
}

// Sub-step i of k of a replayed move from (xa, ya) to (xb, yb); in a periodic
// box (P > 0) along the nearest-image displacement, folded into [0, P).
__global__ void k_interp(int n, int i, int k, const double *xa, const double *ya, const double *xb,
                         const double *yb, double *x, double *y, double2 *xy, double P) {
#pragma clang fp contract(off)
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    double nx, ny;
    if (i == k) {
        nx = xb[v];
        ny = yb[v];
    } else if (P > 0.0) {
        const double s = (double)i / (double)k;
        nx = bd_wrap(xa[v] + s * bd_min_image(xb[v] - xa[v], P), P);
        ny = bd_wrap(ya[v] + s * bd_min_image(yb[v] - ya[v], P), P);
    } else {
        const double s = (double)i / (double)k;
        nx = xa[v] + s * (xb[v] - xa[v]);
        ny = ya[v] + s * (yb[v] - ya[v]);
    }
    x[v] = nx;
    y[v] = ny;
    xy[v] = make_double2(nx, ny);
}

inline int grid_for(long items, int cap = kMaxGrid) {
    long b = (items + 255) / 256;
    if (b < 1) b = 1;
    return (int)(b < cap ? b : cap);
}

// Workgroups of the worklist-driven launches: most of them find a short or
// empty list, and an empty launch costs more the more workgroups it has, so
// the grid grows with the problem (lists grow with it), from 16 to 128.
inline int list_grid(const Sim &s) {
    const int g = s.n / 1024;
    return g < 16 ? 16 : (g > kListGridMax ? kListGridMax : g);
}

}  // namespace

void launch_flip_eval_full(Sim &s, int round, int slot, int reversal) {
    round -= s.rbase;
    Topo t = topo_of(s);
    hipLaunchKernelGGL(k_flip_eval_full, dim3(grid_for((long)(s.T + 3) / 4 * 1024 / kEvalBlock, kEvalGrid)), dim3(kEvalBlock), 0, s.stream, t, round,
                       slot, reversal);
}

void launch_flip_eval_list(Sim &s, int round, int slot) {
    round -= s.rbase;
    Topo t = topo_of(s);
    hipLaunchKernelGGL(k_flip_eval_list, dim3(list_grid(s)), dim3(256), 0, s.stream, t, round, slot);
}

void launch_flip_apply(Sim &s, int round, int slot) {
    round -= s.rbase;
    Topo t = topo_of(s);
    hipLaunchKernelGGL(k_flip_apply, dim3(list_grid(s)), dim3(256), 0, s.stream, t, round, slot);
}

void launch_flip_fix(Sim &s, int round, int slot) {
    round -= s.rbase;
    Topo t = topo_of(s);
    hipLaunchKernelGGL(k_flip_fix, dim3(list_grid(s)), dim3(256), 0, s.stream, t, round, slot);
}

void launch_validate(Sim &s, int rep, int last) {
    Topo t = topo_of(s);
    hipLaunchKernelGGL(k_validate, dim3(grid_for((s.T + 3) / 4)), dim3(kScanBlock), 0, s.stream, t, rep, last);
}

void launch_validate_local(Sim &s, int rep, int k, int last) {
    Topo t = topo_of(s);
    hipLaunchKernelGGL(k_validate_local, dim3(list_grid(s)), dim3(256), 0, s.stream, t, rep, k, last);
}

void launch_ovl_detect(Sim &s, int vstamp, int k, int check, int vrep, int vlast) {
    vstamp -= s.vbase;
    Topo t = topo_of(s);
    hipLaunchKernelGGL(k_ovl_detect, dim3(grid_for((s.T + 3) / 4)), dim3(kDetBlock), 0, s.stream, t, vstamp,
                       1.0 - s.p.contact_tol, k, check, vrep, vlast);
}

void launch_validate_detect_local(Sim &s, int rep, int k, int last, int vstamp, int knew, int check) {
    vstamp -= s.vbase;
    Topo t = topo_of(s);
    hipLaunchKernelGGL(k_validate_detect_local, dim3(list_grid(s)), dim3(256), 0, s.stream, t, rep, k, last, vstamp,
                       1.0 - s.p.contact_tol, knew, check);
}

void launch_ovl_detect_local(Sim &s, int vstamp, int k, int kprev, int check) {
    vstamp -= s.vbase;
    Topo t = topo_of(s);
    hipLaunchKernelGGL(k_ovl_detect_local, dim3(list_grid(s)), dim3(256), 0, s.stream, t, vstamp,
                       1.0 - s.p.contact_tol, k, kprev, check);
}

void launch_ovl_gather(Sim &s, int k) {
    Topo t = topo_of(s);
    hipLaunchKernelGGL(k_ovl_gather, dim3(list_grid(s)), dim3(256), 0, s.stream, t, k, s.p.overlap_factor,
                       s.p.cap_frac, 1.0 - s.p.contact_tol);
}

void launch_ovl_apply(Sim &s, int k, int next_round, int slot) {
    next_round -= s.rbase;
    Topo t = topo_of(s);
    hipLaunchKernelGGL(k_ovl_apply, dim3(list_grid(s)), dim3(256), 0, s.stream, t, k, next_round, slot);
}

void launch_tail(Sim &s, const TailPlan &plan) {
    Topo t = topo_of(s);
    hipLaunchKernelGGL(k_tail, dim3(1), dim3(kTailBlock), 0, s.stream, t, plan);
}

void launch_repair_rounds(Sim &s, int round0, int slot0, int rounds, bool first_evaluated) {
    Topo t = topo_of(s);
    hipLaunchKernelGGL(k_repair_rounds, dim3(1), dim3(kTailBlock), 0, s.stream, t, round0 - s.rbase, slot0, rounds,
                       first_evaluated ? 1 : 0);
}

void launch_snapshot(Sim &s) {
    Topo t = topo_of(s);
    const void *p[] = {s.he_v, s.he_twin, s.vert_he, s.snap_v, s.snap_twin, s.snap_vh};
    int vec = 1;
    for (const void *q : p) vec &= ((uintptr_t)q % 16 == 0) ? 1 : 0;
    hipLaunchKernelGGL(k_snapshot, dim3(grid_for(s.H / 4, kScanGrid)), dim3(256), 0, s.stream, t, s.snap_v,
                       s.snap_twin, s.snap_vh, s.nv + s.R, vec);
}

void launch_scatter_oldpos(Sim &s, int k) {
    Topo t = topo_of(s);
    hipLaunchKernelGGL(k_scatter_oldpos, dim3(grid_for(s.n)), dim3(256), 0, s.stream, t, k, s.xa, s.ya);
}

void launch_interp(Sim &s, int i, int k) {
    hipLaunchKernelGGL(k_interp, dim3((s.n + 255) / 256), dim3(256), 0, s.stream, s.n, i, k, s.xa, s.ya, s.xb,
                       s.yb, s.x, s.y, s.xy, s.period);
}

}  // namespace bd
