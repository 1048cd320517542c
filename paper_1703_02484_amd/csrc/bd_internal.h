// Internal state of a simulation handle and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/bd.h"

namespace bd {

// Device int32 counters (ctr[]) and uint64 accumulators (acc[]).
enum Ctr {
    C_CAND = 0,
    C_WL_NEXT = 1,
    C_TOUCHED = 2,
    C_OVL_EDGES = 3,
    C_INVALID = 4,
    C_STAR_OVF = 5,
    C_TOPO_ERR = 6,   // an index read from the triangulation was out of range
    C_INVERTED = 7,   // evaluated quads holding an inverted or flat finite triangle
    N_CTR = 16
};
enum Acc {
    A_FLIPS = 0,
    A_INV_FLIPS = 1,
    A_REVERSALS = 2,
    A_NOISE_CLAMPS = 3,
    A_CAP_HITS = 4,
    A_OVL_EDGES = 5,
    N_ACC = 8
};

// One chunk of the all-pairs j loop: sorted j range [js, je) of species spec.
struct Chunk {
    int js, je, spec, pad;
};

struct Sim {
    int n = 0;          // particles (vertex ids 0..n-1)
    int m = 0;          // fixed frame points outside the walls (vertex ids n..n+m-1)
    int nv = 0;         // finite vertices n + m
    int S = 1;          // species
    int T = 0;          // triangles incl. ghosts: 2 nv - 2
    int H = 0;          // half-edges: 3T
    int inf = 0;        // infinite vertex id (= nv)
    bd_params p{};
    bd_force_params fp{};
    std::vector<double> K;           // S*S
    int64_t step = 0;
    bool fp32 = false;
    int kind_fast = 1;               // 1: inverse-square all pairs (q = 2, no cutoff)

    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    int device = 0;

    // particle state (caller order)
    double *x = nullptr, *y = nullptr, *xo = nullptr, *yo = nullptr;
    double *th = nullptr, *tho = nullptr, *rad = nullptr;
    int *sp = nullptr;
    // force stage
    int *sorted_id = nullptr;        // sorted index -> caller id (species-sorted)
    int *pos_of = nullptr;           // caller id -> sorted index
    void *pj = nullptr;              // float2 / double2 [n], sorted order
    void *part = nullptr;            // [nchunks][n] float2 / double2 partial sums
    std::vector<Chunk> chunks_h;
    Chunk *chunks = nullptr;
    int nchunks = 0;
    int iblock = 0;                  // i per workgroup in the force kernel
    double *Kd = nullptr;
    double *fout = nullptr;          // [2n] forces in caller order (bd_forces)
    // triangulation (half-edge SoA, ghosts included)
    int *he_v = nullptr, *he_twin = nullptr, *vert_he = nullptr;
    unsigned long long *claim = nullptr;
    int *tri_stamp = nullptr, *moved = nullptr, *edge_stamp = nullptr, *vstamp = nullptr;
    int *wl[2] = {nullptr, nullptr};
    int wl_cur = 0;
    int2 *cand = nullptr;
    int *cand_won = nullptr;
    int *touched = nullptr;
    double2 *newpos = nullptr;
    double2 *oldpos = nullptr;       // positions of touched disks before an overlap round
    // repair fallback: topology snapshot and the move it must replay
    int *snap_v = nullptr, *snap_twin = nullptr, *snap_vh = nullptr;
    double *xa = nullptr, *ya = nullptr, *xb = nullptr, *yb = nullptr;
    int round_id = 0;                // flip-round stamp
    int vround = 0;                  // overlap-round stamp
    // counters
    int *ctr = nullptr;
    unsigned long long *acc = nullptr;
    int *hctr = nullptr;             // pinned mirror of ctr
    unsigned long long *hacc = nullptr;

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
void launch_force(Sim &s);
void launch_em(Sim &s);
void launch_reduce_forces(Sim &s);
// triangulation
void launch_flip_eval_full(Sim &s, int round, bool reversal);
void launch_flip_eval_list(Sim &s, int round, int count);
void launch_flip_apply(Sim &s, int round, int ncand);
void launch_flip_fix(Sim &s, int round, int ncand);
void launch_validate(Sim &s);
// overlap correction
void launch_ovl_detect(Sim &s, int vstamp);
void launch_ovl_gather(Sim &s, int ntouched);
void launch_ovl_apply(Sim &s, int ntouched, int next_round);
// kinetic fallback helpers
void launch_scatter_oldpos(Sim &s, int ntouched);   // xa[v] = oldpos for touched v
void launch_interp(Sim &s, int i, int k);            // x = xa + (i/k)(xb - xa); exactly xb when i == k

// ---- host triangulation (host_dt.cpp) --------------------------------------
// Delaunay triangulation of (x[i], y[i]) with infinite vertex n, as half-edge
// arrays of 3(2n-2) entries.  Returns 0, or -1 when all points are collinear
// or two coincide.
int host_delaunay(int n, const double *x, const double *y, std::vector<int> &he_v, std::vector<int> &he_twin);

// Fixed frame points closing the triangulation outside the walls of [0, L]^2.
void frame_points(double L, double rmax, std::vector<double> &fx, std::vector<double> &fy);

}  // namespace bd

struct bd_sim {
    bd::Sim s;
};
