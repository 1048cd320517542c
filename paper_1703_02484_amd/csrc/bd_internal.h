// Internal state of a simulation handle and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/bd.h"

namespace bd {

// Device control block (int32 ctl[]): flags and per-slot work counts.  A step
// is enqueued as a budgeted sequence of rounds; every round uses its own count
// slots, so no count is reset or read back between launches.
constexpr int MAXR = 160;     // flip-round slots (even: worklists alternate by slot parity)
constexpr int MAXREP = 48;    // repair slots
constexpr int MAXO = 48;      // overlap-round slots
enum Ctl {
    K_HALT = 0,        // nonzero: stop; the host finishes the step
    K_REASON = 1,      // HaltReason
    K_STAGE = 2,       // repair slot (or overlap round) where the step halted
    K_DONE = 3,        // the overlap loop found no overlapping edge
    K_TOPO = 4,        // an index read from the triangulation was out of range
    K_STAR = 5,        // a vertex star walk exceeded its bound
    K_OVL_ROUNDS = 6,  // overlap rounds that moved disks in the budgeted sequence
    K_LAST = 7,        // last round slot of the repair that halted
    K_NL_REBUILD = 8,  // a disk moved more than skin/2 since the neighbour lists were built
    K_NL_OVERFLOW = 9, // largest neighbour count when it exceeded the list capacity
    K_FQUEUE = 10,     // next tile of the persistent all-pairs force launch
    K_TAPE_ENT = 11,   // adjoint tape: entries recorded by the overlap rounds of this step
    K_TAPE_DIR = 12,   // adjoint tape: overlap rounds recorded in this step
    K_TAPE_OVF = 13,   // adjoint tape: 1 = capacity exceeded, 2 = a disk had more than MAXACT partners
    K_FL_N = 14,       // edges flipped since the last overlap detection (list length)
    K_FL_EPOCH = 15,   // stamp of the last overlap detection (dedupes the flipped lists)
    K_VT_N = 16,       // triangles rewritten by flips since the last overlap detection (list length)
    K_TICKET = 17,     // workgroups finished in the current launch (last-workgroup checks; back to 0 after)
    K_NL_BUILT = 18,   // the neighbour lists were rebuilt on the device at the start of this step
    K_NL_STALE = 19,   // list overlap detection: a disk moved so far since the build that a pair may be missing
    K_REV = 20,        // Delaunay edges reversed by this step's move, counted when a reversal halves the step
    K_CAND = 21,                     // [MAXR] flip candidates of round slot j
    K_WL = K_CAND + MAXR,            // [MAXR] worklist length read by round slot j
    K_INVQ = K_WL + MAXR,            // [MAXR] evaluated quads holding an inverted triangle
    K_INV = K_INVQ + MAXR,           // [MAXREP] invalid triangles after repair j
    K_TOUCH = K_INV + MAXREP,        // [MAXO] disks queued by overlap round k
    K_OVL = K_TOUCH + MAXO,          // [MAXO] overlapping edges found by overlap round k
    N_CTL = K_OVL + MAXO
};
enum HaltReason {
    HALT_REPAIR_BUDGET = 1,
    HALT_INVALID = 2,
    HALT_TOPOLOGY = 3,
    HALT_OVERLAP_BUDGET = 4,
    HALT_NL_CAPACITY = 5,  // a rebuild inside a queued step found more neighbours than the lists hold
    HALT_NL_STALE = 6,     // list overlap detection: the lists may miss a pair (rebuild, then continue)
    HALT_REVERSAL = 7      // the move reversed a Delaunay edge: the host redoes the step in halves
};

enum Acc {
    A_FLIPS = 0,
    A_INV_FLIPS = 1,
    A_REVERSALS = 2,
    A_NOISE_CLAMPS = 3,
    A_CAP_HITS = 4,
    A_OVL_EDGES = 5,
    // the noise clamps of the update (a few thousand per step on 1M disks) go to A_CLAMP_SLOTS
    // counters on separate 128-byte lines, chosen by workgroup: updates of one address from every
    // CU serialise; the host adds the slots
    A_CLAMP_BASE = 16,
    A_CLAMP_SLOTS = 64,
    A_CLAMP_STRIDE = 16,
    N_ACC = A_CLAMP_BASE + A_CLAMP_SLOTS * A_CLAMP_STRIDE
};

// Workgroups are dealt to the 8 XCDs of the device round-robin (XCD = block id mod
// 8) and every XCD has its own L2.  This workgroup index gives the workgroups of
// one XCD a contiguous range of the grid (a bijection of [0, gridDim.x)), so
// neighbouring items -- triangles and disks that share vertices and neighbours
// in the library's Hilbert order -- are read through one L2 instead of eight.
#ifdef __HIPCC__
__device__ __forceinline__ int xcd_block() {
    constexpr int kXcd = 8;
    const int b = (int)blockIdx.x, nb = (int)gridDim.x;
    const int q = nb / kXcd, r = nb % kXcd, x = b % kXcd;
    return x * q + (x < r ? x : r) + b / kXcd;
}
#endif

// One workgroup of the all-pairs force: sorted i range [i0, i1) (at most
// 256 * per_lane) against the sorted j range [js, je) of one species of the same
// system; partial sums go to part[pbase + i].
struct Tile {
    int i0, i1, js, je;
    long long pbase;
    long long work;   // (i1 - i0) * (je - js), for ordering
};

// Symmetric form of the all-pairs force: chunks A = [i0, i1) and B = [j0, j1)
// of one system (A before B, or A itself), each pair evaluated once and both
// sides written: part[pbase_i + i] (i in A, sum over B) and part[pbase_j + j]
// (j in B, sum over A; not for A itself).
constexpr int kSymChunk = 1024;   // longest chunk of the symmetric form (256 per_lane, per_lane 2 or 4)
struct SymTile {
    int i0, i1, j0, j1;
    long long pbase_i, pbase_j;
};

// Per-step values that kernels read from device memory, so that a captured
// step can be replayed: the noise counter and the bases of the flip-round and
// overlap-round stamps (kernels receive stamps relative to these bases).
// In graph mode several steps are queued at once: a step that halts (or
// needs new neighbour lists) sets `stop`, and the steps queued after it do
// nothing, so the host finishes that step and resumes exactly there.
struct StepBase {
    long long step;
    int rbase, vbase;
    int stop;        // 0 run; 1 the step batch_idx halted; 2 the ring is full
    int batch_idx;   // steps of the current batch completed on the device
    int nl_req;      // the skin test of the last step asks for new neighbour lists
    int nl_now;      // this step rebuilds them before its force (copied from nl_req when it begins)
};
constexpr int kRing = 64;            // most steps queued at once in graph mode
constexpr size_t kMaxGraphs = 16;    // captured step graphs kept per handle (one per budget setting)

constexpr int MAXACT = 16;    // overlapping partners recorded per disk and round (adjoint tape)

// Tape of one replayed segment of steps for the adjoint sweep: the positions
// before every step, the wall slopes of every move, and for every overlap
// round the disks it moved with their positions before the round, their
// uncapped Jacobi sums, wall slopes and overlapping partners.
struct Tape {
    bool on = false;
    int step_idx = 0;                      // step inside the segment being recorded
    int ent_base = 0, dir_base = 0;        // entries / rounds recorded before this step
    int cap_steps = 0, cap_ent = 0, cap_dir = 0;
    double *px = nullptr, *py = nullptr;   // [cap_steps][n]
    signed char *emwf = nullptr;           // [cap_steps][2n]
    int *ev = nullptr;                     // [cap_ent] disk of each entry
    double2 *eold = nullptr;               // [cap_ent] position before the round
    double2 *edisp = nullptr;              // [cap_ent] uncapped Jacobi sum
    signed char *ewf = nullptr;            // [2 cap_ent] wall slopes of the round's move
    int *ecnt = nullptr;                   // [cap_ent] overlapping partners
    int *enb = nullptr;                    // [cap_ent][MAXACT] their ids, in summation order
    int2 *dir = nullptr;                   // [cap_dir] (first entry, count) of each round
    void *phi = nullptr;                   // [cap_steps][part_cap] force partial sums of each step, or
                                           // null (then the sweep recomputes them)
    std::vector<int> step_dir_end;         // rounds recorded up to the end of each step
};

// Round budgets of the captured step, adapted to what recent steps needed.
struct Budgets {
    int em = 5;         // flip rounds of the repair after the move
    int overlaps = 3;   // overlap rounds
    int ovl[MAXO];      // flip rounds of the repair after overlap round j
    Budgets() {
        for (int &b : ovl) b = 4;
    }
};

// Device copy of the state at one step (adjoint checkpoints).
struct Checkpoint {
    double *x = nullptr, *y = nullptr, *xo = nullptr, *yo = nullptr, *th = nullptr, *tho = nullptr;
    int *he_v = nullptr, *he_twin = nullptr, *vert_he = nullptr;
    int64_t step = 0;
    bd_stats st{};
    unsigned long long acc[N_ACC] = {};
    Budgets budgets;
};

struct AdjState {
    bool ready = false;                    // a forward pass with checkpoints has been run
    int64_t t0 = 0, nsteps = 0;
    int every = 0;
    std::vector<Checkpoint> ck;            // at t0, t0 + every, ..., then the final state
    Tape tape;
    double2 *lam = nullptr, *nu = nullptr; // adjoint of the positions; round scratch
    double *bx = nullptr, *by = nullptr;   // positions before a round, by disk id
    double4 *pj4 = nullptr;                // sorted (x, y, lambda) of one step
    double2 *gpart = nullptr;              // [part_cap] per-chunk adjoint force contributions
    double *dk_rows = nullptr;             // [n][S] one step's dL/dK row of each particle
    double *dk_blk = nullptr;              // [blocks][S*S] partial sums of dL/dK
    double *dk = nullptr;                  // [S*S]
    int dk_blocks = 0;
};

// Per-system constants read by the update kernel.
struct RepInfo {
    int off, n;            // disks [off, off + n) in caller order and in sorted order
    int nch, cfirst;       // chunks of this system and the first one's index in chunk_spec
    long long poff;        // partial sums of chunk c, sorted index k: part[poff + c n + (k - off)]
    double L;              // box side
    unsigned long long seed;
};

struct Sim {
    int R = 1;          // independent systems held by this handle
    int n = 0;          // particles of all systems (vertex ids 0..n-1)
    int m = 0;          // fixed frame points outside the walls (vertex ids n..n+m-1)
    int nv = 0;         // finite vertices n + m
    int S = 1;          // species
    int T = 0;          // triangles incl. ghosts: 2 nv - 2
    int H = 0;          // half-edges: 3T
    int inf = 0;        // first infinite vertex id (= nv); system r has nv + r
    std::vector<int> off_h, foff_h, toff_h;   // per system: first disk, first frame point (rel. n), first triangle
    std::vector<double> L_h;
    std::vector<unsigned long long> seed_h;
    RepInfo *reps = nullptr;
    int *rep_of = nullptr;           // system of each disk
    double *Lr = nullptr;            // box side of each system
    bd_params p{};
    bd_force_params fp{};
    std::vector<double> K;           // S*S
    int64_t step = 0;
    bool fp32 = false;
    int kind_fast = 1;               // 1: inverse-square all pairs (q = 2, no cutoff)

    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    int device = 0;
    // device allocator installed with bd_set_allocator when the handle was created (null: hipMalloc)
    void *(*user_alloc)(size_t, void *, void *) = nullptr;
    void (*user_free)(void *, void *, void *) = nullptr;
    void *user_ctx = nullptr;

    // particle state, in the library's order: inside each system the disks
    // follow the Hilbert curve over the box (neighbours in space are
    // neighbours in memory); perm maps it back to the caller's order
    double *x = nullptr, *y = nullptr, *xo = nullptr, *yo = nullptr;
    // (x, y) of every vertex as one 16-byte pair, equal to x, y after every writer: the kernels that
    // gather the positions of other disks (triangle scans, star walks, list passes) load one pair
    double2 *xy = nullptr;
    double *th = nullptr, *tho = nullptr, *rad = nullptr;
    int *sp = nullptr;
    int *sp_sorted = nullptr;        // species in sorted order
    std::vector<int> perm_h;         // library index -> caller index
    int *perm = nullptr;             // device copy of perm_h
    int *key_id = nullptr;           // caller index inside the disk's system (noise key)
    // force stage
    int *sorted_id = nullptr;        // sorted index -> library index (species-sorted)
    int *pos_of = nullptr;           // library index -> sorted index
    void *pj = nullptr;              // float2 / double2 [n], sorted order
    void *part = nullptr;            // [nchunks][n] float2 / double2 partial sums
    Tile *tiles = nullptr;           // force tiles, longest first (symmetric form: the adjoint's tiles)
    int ntiles = 0;
    SymTile *stiles = nullptr;       // symmetric form: chunk pairs, then each chunk with itself
    int nstiles = 0;
    long long stiles_cap = 0;
    int *chunk_spec = nullptr;       // species of each chunk
    long long part_cap = 0;          // elements allocated for part
    long long tiles_cap = 0;         // tiles allocated
    int chunk_len = 0;               // j per chunk (last chunk of a species may be shorter)
    int per_lane = 4;                // i per lane: a tile holds 256 * per_lane particles
    int persistent = 0;              // launch form: 0 workgroup per tile, 1 fixed grid pulling tiles from a queue,
                                     // 2 symmetric chunk pairs (SymTile)
    int force_grid = 0;              // workgroups of the persistent launch
    int tuned = 0;                   // 1: tiling chosen by timing, 2: from the tuning cache, 0: fixed rule
    double tuned_ms = 0.0;           // force time of the chosen configuration when tuned, else 0
    std::vector<int> bstart_h;       // per system, per species: first sorted index (R x (S+1))
    double *Kd = nullptr;
    double *fout = nullptr;          // [2n] forces in caller order (bd_forces)
    // short-range path: Verlet lists on a cell grid (cutoff > 0)
    bool use_nl = false;
    bool need_rebuild = true;
    int nl_cap = 32, nl_nc = 1, nl_ncell = 1;
    int *nl = nullptr, *nl_cnt = nullptr;
    int *nl_cand = nullptr;          // disks of a one-workgroup list round
    int nl_phase = 1;                // list overlap rounds launched as full passes before the one-workgroup rest
    int *cell_of = nullptr, *cell_count = nullptr, *cell_start = nullptr, *cell_fill = nullptr, *cell_items = nullptr;
    double *xbuild = nullptr, *ybuild = nullptr;
    double2 *fsr = nullptr;          // short-range forces, caller order
    int ovl_method = 0;              // 0: overlap rounds over Delaunay edges; 1: over the neighbour lists
    double period = 0.0;             // > 0: periodic box of this side (minimum-image separations), else walls
    double rad_uni = 0.0;            // > 0: every disk has this radius
    double nl_margin = 0.0;          // lists hold every pair closer than contact while no disk moved farther
                                     // than this since the build: (cutoff + skin - 2 r_max) / 2
    int *scan_bsum = nullptr;        // per-block totals of the cell-count scan
    // triangulation (half-edge SoA, ghosts included)
    int *he_v = nullptr, *he_twin = nullptr, *vert_he = nullptr;
    unsigned long long *claim = nullptr;
    int *tri_stamp = nullptr, *moved = nullptr, *edge_stamp = nullptr, *vstamp = nullptr;
    int *wl[2] = {nullptr, nullptr};   // worklists; round slot j reads wl[j & 1]
    int2 *cand = nullptr;
    int *cand_won = nullptr;
    int *touched = nullptr;          // [2][n] disks queued by an overlap round, by round parity
    int *det_stamp = nullptr;        // [H] edge tested by the current local overlap detection
    int *fl_stamp = nullptr;         // [H] edge recorded in the flipped list in the current epoch
    int *fl = nullptr;               // [H/2 + 64] edges flipped since the last overlap detection
    int *vt_stamp = nullptr;         // [T] triangle recorded in the rewritten list in the current epoch
    int *vt = nullptr;               // [T + 64] triangles rewritten by flips since the last overlap detection
    double2 *newpos = nullptr;
    double2 *oldpos = nullptr;       // positions of touched disks before an overlap round
    // repair fallback: topology snapshot and the move it must replay
    int *snap_v = nullptr, *snap_twin = nullptr, *snap_vh = nullptr;
    double *xa = nullptr, *ya = nullptr, *xb = nullptr, *yb = nullptr;
    double *xs = nullptr, *ys = nullptr, *ths = nullptr;   // start of a step redone in halves (allocated on first use)
    int round_id = 0;                // flip-round stamp (absolute)
    int vround = 0;                  // overlap-round stamp (absolute)
    StepBase *dbase = nullptr;       // device copy of the bases below
    StepBase *hbase = nullptr;       // pinned staging for it
    int rbase = 0, vbase = 0;        // bases currently on the device; launches pass stamp - base
    // captured steps (one graph triple per round-budget setting)
    bool use_graph = false;
    int batch_hint = kRing;          // graph steps queued per batch (adapts to the steps between stops)
    int tail_mode = -1;              // overlap rounds after the first detection: 0 launch per phase,
                                     // 1 one workgroup, 2 the large first rounds launched per phase and the
                                     // rest in one workgroup, -1 chosen from the problem size
    int multi_em = 2;                // mode 2: flip rounds of the move's repair launched on many workgroups
    int multi_ovl = 1;               // mode 2: the same for the repair after an overlap round
    int ovl_phase = 1;               // mode 2: overlap rounds launched per phase before the one-workgroup tail
                                     // (1 + the leading later rounds that recently queued many disks)
    int touch_hi[MAXO] = {};         // most disks queued by overlap round j in the current window of steps
    int touch_prev[MAXO] = {};       // the same over the previous window
    int touch_steps = 0;             // steps in the current window
    struct StepGraph {
        hipGraphExec_t pre = nullptr, force = nullptr, post = nullptr;
        int r_used = 0, v_used = 0;
        int c_slot = 0, c_rep = 0, c_oround = 0;
        std::vector<int> orounds, rep_first;
    };
    std::vector<std::pair<std::vector<int>, StepGraph>> graphs;
    int *ring = nullptr;             // [kRing][N_CTL] control block of each queued step
    int *hring = nullptr;            // pinned mirror
    // control block and accumulators
    int *ctl = nullptr;
    unsigned long long *acc = nullptr;
    int *hctl = nullptr;             // pinned mirror of ctl
    unsigned long long *hacc = nullptr;
    // round budgets of the enqueued step (adapted to recent steps)
    Budgets budget;
    int slack_em = 0, slack_over = 0;   // steps in a row that needed less than each budget
    int slack_ovl[MAXO] = {};

    AdjState adj;

    // host-side stats
    bd_stats st{};
    std::string last_error;

    // measurement
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    double timed_ms = 0.0;
    int64_t timed_launches = 0;
};

// ---- kernel launchers (k_*.hip) ------------------------------------------
void launch_cast(Sim &s);
void launch_step_begin(Sim &s);                       // clear the control block unless the batch stopped
void launch_step_begin_cast(Sim &s);                  // both of the above in one launch (all-pairs path)
void launch_step_end(Sim &s, int r_used, int v_used); // record the control block, advance or stop
void launch_force(Sim &s);
int force_max_grid(Sim &s, int per_lane);            // resident workgroups of the persistent launch
// level > 0: sub-interval `index` of the 2^level halves of the step after edge reversals (Sec. 4.3)
void launch_em(Sim &s, int level = 0, unsigned index = 0);
void launch_reduce_forces(Sim &s);
// short-range path (k_verlet.hip)
int verlet_scan_blocks(int ncells);
void launch_verlet_build(Sim &s);
void launch_verlet_build_requested(Sim &s);   // the same kernels, each doing nothing unless the step asks (graph mode)
void launch_force_nl(Sim &s);
// xy[0, m) = (x, y)[0, m): after a copy into x, y
void launch_pack_xy(Sim &s, int m);
void launch_skin_check(Sim &s);
// overlap rounds over the neighbour lists (Sec. 5 short-range variant, no triangulation): round slot k
void launch_ovl_nl_gather(Sim &s, int k);
void launch_ovl_nl_apply(Sim &s, int k, bool final_check);
// the later overlap rounds over the lists in one workgroup, each over the disks the round before moved and
// their listed neighbours
struct NlTailPlan {
    int nr;          // rounds in the launch
    int k[MAXO];     // their round slots
    int kprev;       // slot of the round before the first
    int stamp0;      // stamp of the first round's marks (relative; one per round)
    int final_last;  // the last round is the budget's last (overlaps left halt the step)
};
void launch_nl_tail(Sim &s, const NlTailPlan &p);
// triangulation (slot: round slot in ctl; rep: repair slot)
// reversal: 0 no test; 1 count reversed edges (Sec. 4.3); 2 count them and flag the step (K_REV) for halving
void launch_flip_eval_full(Sim &s, int round, int slot, int reversal);
void launch_flip_eval_list(Sim &s, int round, int slot);
void launch_flip_apply(Sim &s, int round, int slot);
void launch_flip_fix(Sim &s, int round, int slot);
void launch_validate(Sim &s, int rep, int last = -1);   // last >= 0: also the repair check
// validation after the repair that follows overlap round k: triangles at the disks round k moved and
// triangles rewritten by flips since round k's detection
void launch_validate_local(Sim &s, int rep, int k, int last = -1);
void launch_snapshot(Sim &s);
// overlap correction (k: overlap-round slot)
// check: 0 none, 1 the overlap check of round k, 2 that and the final check
// vrep >= 0: the same pass validates every triangle for repair vrep (last round slot vlast) and checks it first
void launch_ovl_detect(Sim &s, int vstamp, int k, int check = 0, int vrep = -1, int vlast = -1);
// validation after overlap round k's repair fused with round knew's detection (stars walked once)
void launch_validate_detect_local(Sim &s, int rep, int k, int last, int vstamp, int knew, int check);
// detection after round kprev: only edges at disks moved by round kprev and edges flipped since
void launch_ovl_detect_local(Sim &s, int vstamp, int k, int kprev, int check = 0);
void launch_ovl_gather(Sim &s, int k);
void launch_ovl_apply(Sim &s, int k, int next_round, int slot);
// kinetic fallback helpers
void launch_scatter_oldpos(Sim &s, int k);            // xa[v] = old position for disks touched in round k
void launch_interp(Sim &s, int i, int k);             // x = xa + (i/k)(xb - xa); exactly xb when i == k

// The overlap rounds of a step after the first detection, run by one
// workgroup (phases separated by workgroup barriers instead of launches);
// the same rounds, slots and stamps as the launch-per-phase sequence.
constexpr int MAXTAIL = 24;
struct TailPlan {
    int nover;                     // budgeted overlap rounds
    int rounds[MAXTAIL];           // flip rounds of the repair after round j
    int k[MAXTAIL + 1];            // overlap-round slot of round j; k[nover] is the final detection
    int stamp[MAXTAIL + 1];        // detection stamps (relative; round 0's detection ran before)
    int next_round[MAXTAIL];       // first flip round of the repair after round j (relative)
    int slot0[MAXTAIL];            // its first round slot
    int rep[MAXTAIL];              // its repair slot
    double f, cap_frac, keep;
};
void launch_tail(Sim &s, const TailPlan &plan);
// rounds [round0, round0 + rounds) of a repair in one workgroup (first_evaluated: round0's evaluation ran
// already, in a launch of many workgroups)
void launch_repair_rounds(Sim &s, int round0, int slot0, int rounds, bool first_evaluated = true);

// adjoint sweep (k_adjoint.hip)
void launch_adj_round(Sim &s, int first_entry, int count);     // one recorded overlap round, reversed
void launch_adj_step(Sim &s, int t);                           // move of recorded step t, reversed
void launch_adj_dk_final(Sim &s);

// ---- host triangulation (host_dt.cpp) --------------------------------------
// Delaunay triangulation of (x[i], y[i]) with infinite vertex n, as half-edge
// arrays of 3(2n-2) entries.  Returns 0, or -1 when all points are collinear
// or two coincide.
uint64_t hilbert_index(uint32_t x, uint32_t y, int bits);
int host_delaunay(int n, const double *x, const double *y, std::vector<int> &he_v, std::vector<int> &he_twin);
// Delaunay triangulation of the flat torus [0, L)^2 (periodic box): 2n triangles over ids 0..n-1.
int host_torus_delaunay(int n, const double *x, const double *y, double L, std::vector<int> &he_v,
                        std::vector<int> &he_twin);

// Fixed frame points closing the triangulation outside the walls of [0, L]^2.
void frame_points(double L, double rmax, std::vector<double> &fx, std::vector<double> &fy);

}  // namespace bd

struct bd_sim {
    bd::Sim s;
};
