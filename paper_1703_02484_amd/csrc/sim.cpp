// Host runtime of a simulation handle and the C ABI of include/bd.h.
//
// One time step (Algorithm 1, with the overlap loop of Sec. 4.4):
//   cast positions -> all-pairs force -> fused Euler-Maruyama update
//   -> flip repair of the triangulation (first round scans every edge and
//      also counts reversed edges, later rounds only the worklist)
//   -> overlap rounds: detect on Delaunay edges, Jacobi gather over vertex
//      stars, apply, flip repair of the touched stars; until none overlaps.
// Control returns to the host only for the small counters that size the next
// launch; a repair that cannot finish on the device falls back to a host
// rebuild of the Delaunay triangulation at that exact point of the step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "bd_internal.h"
#include "geom.h"

namespace bd {
namespace {

__global__ void k_fill_int(int *p, int count, int value) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

struct DeviceError {
    hipError_t e;
    const char *what;
};

inline void check(hipError_t e, const char *what) {
    if (e != hipSuccess) throw DeviceError{e, what};
}

template <typename T>
T *dalloc(size_t count) {
    void *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) throw std::bad_alloc();
    return (T *)p;
}

void fill_int(Sim &s, int *p, int count, int value) {
    hipLaunchKernelGGL(k_fill_int, dim3((count + 255) / 256), dim3(256), 0, s.stream, p, count, value);
}

void read_ctl(Sim &s) {
    check(hipMemcpyAsync(s.hctl, s.ctl, sizeof(int) * N_CTL, hipMemcpyDeviceToHost, s.stream), "control copy");
    check(hipStreamSynchronize(s.stream), "stream sync");
}

// Zeroes one control entry (device work, ordered on the stream).
void zero_ctl(Sim &s, int idx) { fill_int(s, s.ctl + idx, 1, 0); }

void upload_topology(Sim &s, const std::vector<int> &he_v, const std::vector<int> &he_twin) {
    std::vector<int> vh(s.nv + 1, -1);
    for (int h = 0; h < s.H; ++h) vh[he_v[h]] = h;
    check(hipMemcpyAsync(s.he_v, he_v.data(), sizeof(int) * s.H, hipMemcpyHostToDevice, s.stream), "he_v");
    check(hipMemcpyAsync(s.he_twin, he_twin.data(), sizeof(int) * s.H, hipMemcpyHostToDevice, s.stream), "twin");
    check(hipMemcpyAsync(s.vert_he, vh.data(), sizeof(int) * (s.nv + 1), hipMemcpyHostToDevice, s.stream), "vh");
    check(hipStreamSynchronize(s.stream), "topology upload");
}

// Host rebuild of DT(current positions).  Returns BD_OK or BD_ERR_TRIANGULATION.
int host_rebuild(Sim &s) {
    std::vector<double> hx(s.nv), hy(s.nv);
    check(hipMemcpyAsync(hx.data(), s.x, sizeof(double) * s.nv, hipMemcpyDeviceToHost, s.stream), "x");
    check(hipMemcpyAsync(hy.data(), s.y, sizeof(double) * s.nv, hipMemcpyDeviceToHost, s.stream), "y");
    check(hipStreamSynchronize(s.stream), "rebuild download");
    std::vector<int> hv, ht;
    if (host_delaunay(s.nv, hx.data(), hy.data(), hv, ht) != 0) {
        s.last_error = "host Delaunay rebuild failed (coincident positions)";
        return BD_ERR_TRIANGULATION;
    }
    upload_topology(s, hv, ht);
    ++s.st.host_rebuilds;
    return BD_OK;
}

// Slot cursor of one step: round slots, repair slots and overlap-round slots
// are handed out in order and wrap around (the host zeroes a slot before it
// reuses one).
struct Cursor {
    int slot = 0, rep = 0, oround = 0;
    int take_slot() {
        int v = slot;
        slot = slot + 1 == MAXR ? 0 : slot + 1;
        return v;
    }
    int take_rep() {
        int v = rep;
        rep = rep + 1 == MAXREP ? 0 : rep + 1;
        return v;
    }
    int take_oround() {
        int v = oround;
        oround = oround + 1 == MAXO ? 0 : oround + 1;
        return v;
    }
};

inline int next_slot(int slot) { return slot + 1 == MAXR ? 0 : slot + 1; }

// ------------------------------------------------------------------ budgeted sequence
// Enqueues one repair of `rounds` flip rounds with no host read-back: a
// topology snapshot, the rounds, the validation and the check that halts the
// step when the budget was too small or a triangle stayed inverted.
void enqueue_repair(Sim &s, Cursor &c, bool full, bool reversal, int rounds, std::vector<int> *first_slots) {
    launch_snapshot(s);
    const int rep = c.take_rep();
    if (first_slots) first_slots->push_back(c.slot);
    int last = -1;
    for (int j = 0; j < rounds; ++j) {
        const int r = ++s.round_id;
        const int slot = c.take_slot();
        if (j == 0 && full)
            launch_flip_eval_full(s, r, slot, reversal);
        else
            launch_flip_eval_list(s, r, slot);
        launch_flip_apply(s, r, slot);
        launch_flip_fix(s, r, slot);
        last = slot;
    }
    launch_validate(s, rep);
    launch_repair_check(s, rep, last);
}

// ------------------------------------------------------------------ host-driven path
// Flip rounds with one read-back per round (used to finish a step whose
// budget ran out, for bd_set_positions and for the kinetic replay).  The
// first round reads the worklist of slot c.slot unless `full`.  When `snap` is
// given and the first evaluation meets an inverted triangle, the topology is
// copied aside before any flip.  Returns true for a valid triangulation with
// no edge left to flip.
bool host_flip_rounds(Sim &s, Cursor &c, bool full, bool reversal, bool *snap) {
    if (snap) *snap = false;
    const int budget = s.p.max_flip_rounds > 0 ? s.p.max_flip_rounds : 200;
    bool done = false;
    for (int it = 0; it < budget; ++it) {
        const int r = ++s.round_id;
        const int slot = c.take_slot();
        zero_ctl(s, K_CAND + slot);
        zero_ctl(s, K_INVQ + slot);
        zero_ctl(s, K_WL + next_slot(slot));
        if (full)
            launch_flip_eval_full(s, r, slot, reversal && it == 0);
        else
            launch_flip_eval_list(s, r, slot);
        read_ctl(s);
        ++s.st.flip_rounds_total;
        if (s.hctl[K_TOPO] != 0) return false;
        if (it == 0 && snap && s.hctl[K_INVQ + slot] > 0) {
            launch_snapshot(s);
            *snap = true;
        }
        if (s.hctl[K_CAND + slot] == 0) {
            done = true;
            c.slot = slot;   // reuse the empty slot
            break;
        }
        launch_flip_apply(s, r, slot);
        launch_flip_fix(s, r, slot);
        full = false;
    }
    if (!done) return false;
    const int rep = c.take_rep();
    zero_ctl(s, K_INV + rep);
    launch_validate(s, rep);
    read_ctl(s);
    return s.hctl[K_INV + rep] == 0 && s.hctl[K_TOPO] == 0;
}

// Where the positions before the move that is being repaired are kept.
enum class MoveFrom { Previous, Touched };

// Replays the move from the snapshot in k equal sub-steps (k = 2, 4, ..., 64),
// each repaired by the Sec. 4.3 + Lawson rule, ending exactly at the target;
// a host rebuild is the last resort.  The Delaunay triangulation of the
// target is unique, so the path does not change the result.
int kinetic_replay(Sim &s, Cursor &c, MoveFrom from, int oround) {
    const size_t bytes = sizeof(double) * s.n;
    check(hipMemcpyAsync(s.xb, s.x, bytes, hipMemcpyDeviceToDevice, s.stream), "xb");
    check(hipMemcpyAsync(s.yb, s.y, bytes, hipMemcpyDeviceToDevice, s.stream), "yb");
    if (from == MoveFrom::Previous) {
        check(hipMemcpyAsync(s.xa, s.xo, bytes, hipMemcpyDeviceToDevice, s.stream), "xa");
        check(hipMemcpyAsync(s.ya, s.yo, bytes, hipMemcpyDeviceToDevice, s.stream), "ya");
    } else {
        check(hipMemcpyAsync(s.xa, s.x, bytes, hipMemcpyDeviceToDevice, s.stream), "xa");
        check(hipMemcpyAsync(s.ya, s.y, bytes, hipMemcpyDeviceToDevice, s.stream), "ya");
        launch_scatter_oldpos(s, oround);
    }
    for (int k = 2; k <= 64; k *= 2) {
        check(hipMemcpyAsync(s.he_v, s.snap_v, sizeof(int) * s.H, hipMemcpyDeviceToDevice, s.stream), "restore");
        check(hipMemcpyAsync(s.he_twin, s.snap_twin, sizeof(int) * s.H, hipMemcpyDeviceToDevice, s.stream),
              "restore");
        check(hipMemcpyAsync(s.vert_he, s.snap_vh, sizeof(int) * (s.nv + 1), hipMemcpyDeviceToDevice, s.stream),
              "restore");
        bool ok = true;
        for (int i = 1; i <= k && ok; ++i) {
            launch_interp(s, i, k);
            ok = host_flip_rounds(s, c, true, false, nullptr);
        }
        if (ok) {
            ++s.st.kinetic_repairs;
            return BD_OK;
        }
    }
    check(hipMemcpyAsync(s.x, s.xb, bytes, hipMemcpyDeviceToDevice, s.stream), "x");
    check(hipMemcpyAsync(s.y, s.yb, bytes, hipMemcpyDeviceToDevice, s.stream), "y");
    return host_rebuild(s);
}

// Restores DT(x) after a move, host-driven: the paper's repair
// (inverted-triangle flips, Sec. 4.3, and Lawson flips, Sec. 4.1) first; a
// disk that crossed more than one edge (Sec. 4.3, two-flip figure) makes it
// fail, and the move is replayed from the snapshot in sub-steps.
int host_repair(Sim &s, Cursor &c, bool full, bool reversal, MoveFrom from, int oround) {
    bool snapped = false;
    if (host_flip_rounds(s, c, full, reversal, &snapped)) return BD_OK;
    if (!snapped || s.hctl[K_TOPO] != 0) {
        zero_ctl(s, K_TOPO);
        return host_rebuild(s);
    }
    return kinetic_replay(s, c, from, oround);
}

void rollback(Sim &s) {
    check(hipMemcpyAsync(s.x, s.xo, sizeof(double) * s.n, hipMemcpyDeviceToDevice, s.stream), "rollback x");
    check(hipMemcpyAsync(s.y, s.yo, sizeof(double) * s.n, hipMemcpyDeviceToDevice, s.stream), "rollback y");
    check(hipMemcpyAsync(s.th, s.tho, sizeof(double) * s.n, hipMemcpyDeviceToDevice, s.stream), "rollback th");
    fill_int(s, s.ctl, N_CTL, 0);
    s.need_rebuild = true;
    host_rebuild(s);
}

// Rebuilds the Verlet lists from the current positions (one read-back to
// check the list capacity; grows it once if a disk has too many neighbours).
void verlet_rebuild(Sim &s) {
    for (int attempt = 0; attempt < 2; ++attempt) {
        fill_int(s, s.cell_count, s.nl_ncell + 1, 0);
        fill_int(s, s.cell_fill, s.nl_ncell, 0);
        zero_ctl(s, K_NL_OVERFLOW);
        launch_verlet_build(s);
        read_ctl(s);
        const int need = s.hctl[K_NL_OVERFLOW];
        if (need == 0) {
            ++s.st.verlet_rebuilds;
            s.need_rebuild = false;
            return;
        }
        if (need > 96 || s.nl_cap >= 96) throw DeviceError{hipErrorInvalidValue, "neighbour list capacity (96) exceeded"};
        check(hipFree(s.nl), "free nl");
        s.nl = nullptr;
        s.nl_cap = 96;
        s.nl = dalloc<int>((size_t)s.nl_cap * s.n);
    }
}

void compute_forces(Sim &s) {
    if (s.use_nl && s.need_rebuild) verlet_rebuild(s);
    if (!s.use_nl) launch_cast(s);
    hipEvent_t a = nullptr, b = nullptr;
    if (s.timing) {
        check(hipEventCreate(&a), "event");
        check(hipEventCreate(&b), "event");
        check(hipEventRecord(a, s.stream), "event record");
    }
    if (s.use_nl)
        launch_force_nl(s);
    else
        launch_force(s);
    if (s.timing) {
        check(hipEventRecord(b, s.stream), "event record");
        s.ev.emplace_back(a, b);
    }
}

// Skin test for the next step's lists (short-range path only).
void skin_check(Sim &s, bool read_back) {
    if (!s.use_nl) return;
    zero_ctl(s, K_NL_REBUILD);
    launch_skin_check(s);
    if (read_back) {
        read_ctl(s);
        s.need_rebuild = s.hctl[K_NL_REBUILD] != 0;
    }
}

// Host-driven overlap rounds from overlap round index `done_rounds` on; returns
// BD_OK with *rounds_out updated, or an error code (state rolled back).
int host_overlap_loop(Sim &s, Cursor &c, int &rounds) {
    const int max_rounds = s.p.max_overlap_rounds > 0 ? s.p.max_overlap_rounds : 10000;
    for (;;) {
        const int k = c.take_oround();
        zero_ctl(s, K_TOUCH + k);
        zero_ctl(s, K_OVL + k);
        launch_ovl_detect(s, ++s.vround, k);
        read_ctl(s);
        if (s.hctl[K_TOPO] != 0) {
            s.last_error = "triangulation index out of range during overlap detection";
            return BD_ERR_TRIANGULATION;
        }
        const int nedges = s.hctl[K_OVL + k];
        if (nedges == 0) return BD_OK;
        if (rounds >= max_rounds) {
            s.last_error = "overlap correction did not converge within max_overlap_rounds";
            return BD_ERR_NO_CONVERGENCE;
        }
        ++rounds;
        s.st.overlap_edges_total += nedges;
        launch_ovl_gather(s, k);
        const int slot = c.slot;
        zero_ctl(s, K_WL + slot);
        launch_ovl_apply(s, k, s.round_id + 1, slot);
        read_ctl(s);
        if (s.hctl[K_STAR] != 0 || s.hctl[K_TOPO] != 0) {
            s.last_error = "vertex star walk failed (corrupt triangulation)";
            return BD_ERR_TRIANGULATION;
        }
        int rc = host_repair(s, c, false, false, MoveFrom::Touched, k);
        if (rc != BD_OK) return rc;
    }
}

// One step of Algorithm 1.  The whole step is enqueued as a budgeted sequence
// (force, update, repair rounds, overlap rounds each with its repair) and the
// control block is read back once; if a budget ran out or a repair failed,
// the host finishes the step from exactly that point.
int one_step(Sim &s) {
    Cursor c;
    fill_int(s, s.ctl, N_CTL, 0);
    compute_forces(s);
    launch_em(s);
    std::vector<int> rep_first;   // first round slot of each enqueued repair
    enqueue_repair(s, c, true, true, s.budget_em_rounds, &rep_first);
    std::vector<int> orounds;
    for (int j = 0; j < s.budget_overlaps; ++j) {
        const int k = c.take_oround();
        orounds.push_back(k);
        launch_ovl_detect(s, ++s.vround, k);
        launch_ovl_check(s, k);
        launch_ovl_gather(s, k);
        launch_ovl_apply(s, k, s.round_id + 1, c.slot);
        enqueue_repair(s, c, false, false, s.budget_ovl_rounds, &rep_first);
    }
    {
        const int k = c.take_oround();
        orounds.push_back(k);
        launch_ovl_detect(s, ++s.vround, k);
        launch_ovl_check(s, k);
        launch_final_check(s, k);
    }
    skin_check(s, false);
    read_ctl(s);
    const int *h = s.hctl;
    s.need_rebuild = s.use_nl && h[K_NL_REBUILD] != 0;
    // bookkeeping of the budgeted part: overlap rounds that moved disks
    int rounds = h[K_OVL_ROUNDS];
    if (h[K_HALT]) {
        if (h[K_REASON] == HALT_OVERLAP_BUDGET) rounds = s.budget_overlaps;
        if (h[K_REASON] == HALT_REPAIR_BUDGET || h[K_REASON] == HALT_INVALID) rounds = h[K_STAGE];
    }
    for (int j = 0; j < rounds; ++j) s.st.overlap_edges_total += h[K_OVL + orounds[j]];
    for (int j = 0; j < c.slot; ++j) s.st.flip_rounds_total += h[K_CAND + j] > 0 ? 1 : 0;
    int rc = BD_OK;
    if (h[K_HALT]) {
        const int reason = h[K_REASON], stage = h[K_STAGE], last = h[K_LAST];
        if (reason == HALT_TOPOLOGY) {
            s.last_error = "triangulation index out of range";
            rollback(s);
            return BD_ERR_TRIANGULATION;
        }
        // continue host-driven after the halting point
        fill_int(s, s.ctl + K_HALT, 1, 0);
        fill_int(s, s.ctl + K_DONE, 1, 0);
        Cursor hc;
        hc.slot = c.slot;
        hc.rep = c.rep;
        hc.oround = c.oround;
        if (reason == HALT_REPAIR_BUDGET || reason == HALT_INVALID) {
            // repair slot `stage`: 0 is the repair after the update, j >= 1 the one after overlap round j-1
            const MoveFrom from = stage == 0 ? MoveFrom::Previous : MoveFrom::Touched;
            const int k = stage == 0 ? 0 : orounds[stage - 1];
            if (reason == HALT_REPAIR_BUDGET) {
                hc.slot = next_slot(last);   // its worklist holds the edges still to evaluate
                bool snapped = false;
                if (!host_flip_rounds(s, hc, false, false, &snapped)) rc = kinetic_replay(s, hc, from, k);
            } else {
                rc = kinetic_replay(s, hc, from, k);
            }
        }
        if (rc == BD_OK) rc = host_overlap_loop(s, hc, rounds);
        if (rc != BD_OK) {
            rollback(s);
            s.need_rebuild = true;
            return rc;
        }
        skin_check(s, true);   // positions moved after the budgeted sequence's test
    }
    // adapt the budgets to the rounds this step needed: grow at once when a
    // budget ran out, shrink by one when it was larger than needed
    auto used_rounds = [&](int rep, int budget) {
        for (int j = 0; j < budget; ++j)
            if (h[K_CAND + rep_first[rep] + j] == 0) return j + 1;
        return budget + 2;
    };
    auto adapt = [](int &budget, int used) {
        if (used >= budget)
            budget = std::min(8, used + 1);
        else if (used + 1 < budget)
            budget = std::max(2, budget - 1);
    };
    const int hreason = h[K_HALT] ? h[K_REASON] : 0;
    // repair slot that stopped the budgeted sequence (none for an overlap budget halt)
    const int halt_rep = (hreason == HALT_REPAIR_BUDGET || hreason == HALT_INVALID) ? h[K_STAGE] : 1 << 30;
    if (halt_rep > 0)
        adapt(s.budget_em_rounds, used_rounds(0, s.budget_em_rounds));
    else if (hreason == HALT_REPAIR_BUDGET)
        adapt(s.budget_em_rounds, s.budget_em_rounds + 2);
    int ovl_used = 0;
    for (int r = 1; r < (int)rep_first.size() && r <= rounds && r < halt_rep; ++r)
        ovl_used = std::max(ovl_used, used_rounds(r, s.budget_ovl_rounds));
    if (hreason == HALT_REPAIR_BUDGET && halt_rep > 0) ovl_used = s.budget_ovl_rounds + 2;
    if (ovl_used > 0) adapt(s.budget_ovl_rounds, ovl_used);
    s.budget_overlaps = std::max(2, std::min(8, rounds + 1));
    s.st.overlap_rounds_total += rounds;
    if (rounds > s.st.overlap_rounds_max) s.st.overlap_rounds_max = rounds;
    ++s.st.steps;
    ++s.step;
    return BD_OK;
}

void setup_chunks(Sim &s, const std::vector<int> &block_start) {
    const int per_block = 256 * 4;
    const int nib = (s.n + per_block - 1) / per_block;
    const int target_blocks = 2048;
    int want = std::max(1, (target_blocks + nib - 1) / nib);
    s.chunks_h.clear();
    for (int b = 0; b < s.S; ++b) {
        const int js = block_start[b], je = block_start[b + 1], cnt = je - js;
        if (cnt <= 0) continue;
        int nc = (int)std::llround((double)want * cnt / s.n);
        nc = std::max(1, std::min(nc, std::max(1, cnt / 64)));
        int len = (cnt + nc - 1) / nc;
        len = (len + 7) / 8 * 8;
        for (int j = js; j < je; j += len) s.chunks_h.push_back(Chunk{j, std::min(je, j + len), b, 0});
    }
    s.nchunks = (int)s.chunks_h.size();
}

void free_all(Sim &s) {
    void *ptrs[] = {s.x, s.y, s.xo, s.yo, s.th, s.tho, s.rad, s.sp, s.sorted_id, s.pos_of, s.pj, s.part,
                    s.chunks, s.Kd, s.fout, s.he_v, s.he_twin, s.vert_he, s.claim, s.tri_stamp, s.moved,
                    s.edge_stamp, s.vstamp, s.wl[0], s.wl[1], s.cand, s.cand_won, s.touched, s.newpos, s.oldpos,
                    s.snap_v, s.snap_twin, s.snap_vh, s.xa, s.ya, s.xb, s.yb, s.ctl, s.acc, s.nl, s.nl_cnt,
                    s.cell_of, s.cell_count, s.cell_start, s.cell_fill, s.cell_items, s.xbuild, s.ybuild, s.fsr,
                    s.scan_tmp};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (s.hctl) (void)hipHostFree(s.hctl);
    if (s.hacc) (void)hipHostFree(s.hacc);
    for (auto &e : s.ev) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    s.ev.clear();
    if (s.own_stream) (void)hipStreamDestroy(s.own_stream);
}

bool finite(double v) { return std::isfinite(v); }

int validate_args(int n, const double *xy, const double *radii, const int32_t *species, const double *theta,
                  const bd_force_params *fp, const bd_params *p, std::string &err) {
    if (!xy || !radii || !species || !fp || !p) return err = "NULL argument", BD_ERR_INVALID_ARG;
    if (n < 3) return err = "n must be at least 3", BD_ERR_INVALID_ARG;
    if (fp->S < 1 || fp->S > BD_MAX_SPECIES || !fp->K) return err = "S out of range or K NULL", BD_ERR_INVALID_ARG;
    if (fp->kind != BD_FORCE_POWER && fp->kind != BD_FORCE_SCREENED) return err = "unknown force kind", BD_ERR_INVALID_ARG;
    for (int k = 0; k < fp->S * fp->S; ++k)
        if (!finite(fp->K[k])) return err = "K has a non-finite entry", BD_ERR_INVALID_ARG;
    if (!finite(fp->q) || !finite(fp->A) || !finite(fp->lambda) || !finite(fp->cutoff) || !finite(fp->skin))
        return err = "non-finite force parameter", BD_ERR_INVALID_ARG;
    if (fp->kind == BD_FORCE_SCREENED && !(fp->lambda > 0)) return err = "lambda must be > 0", BD_ERR_INVALID_ARG;
    if (fp->cutoff > 0 && !(fp->skin >= 0)) return err = "skin must be >= 0", BD_ERR_INVALID_ARG;
    const double vals[] = {p->L, p->D, p->dt, p->v0, p->Dr, p->overlap_factor, p->cap_frac, p->noise_clip,
                           p->contact_tol};
    for (double v : vals)
        if (!finite(v)) return err = "non-finite step parameter", BD_ERR_INVALID_ARG;
    if (!(p->L > 0) || p->D < 0 || !(p->dt > 0) || p->Dr < 0 || !(p->overlap_factor > 0) || !(p->cap_frac > 0) ||
        !(p->noise_clip > 0) || p->contact_tol < 0 || p->contact_tol > 1e-3)
        return err = "step parameter out of range", BD_ERR_INVALID_ARG;
    if (p->force_precision != BD_PREC_FP32 && p->force_precision != BD_PREC_FP64)
        return err = "unknown force precision", BD_ERR_INVALID_ARG;
    if (p->reserved != 0) return err = "reserved field must be 0", BD_ERR_INVALID_ARG;
    for (int i = 0; i < n; ++i) {
        double r = radii[i], x = xy[2 * i], y = xy[2 * i + 1];
        if (!finite(r) || !(r > 0) || !finite(x) || !finite(y)) return err = "bad radius or position", BD_ERR_INVALID_ARG;
        if (species[i] < 0 || species[i] >= fp->S) return err = "species out of range", BD_ERR_INVALID_ARG;
        if (theta && !finite(theta[i])) return err = "non-finite theta", BD_ERR_INVALID_ARG;
        if (x < r || x > p->L - r || y < r || y > p->L - r) return err = "disk outside the walls", BD_ERR_BAD_INPUT;
    }
    // overlap check on a cell grid (cell side >= the largest contact distance)
    double rmax = 0;
    for (int i = 0; i < n; ++i) rmax = std::max(rmax, radii[i]);
    const double cell = 2 * rmax;
    long nc = std::max(1L, std::min(32768L, (long)std::floor(p->L / cell)));
    const double inv = nc / p->L;
    std::vector<int> head((size_t)nc * nc, -1), nxt(n, -1);
    auto cidx = [&](double v) { long c = (long)(v * inv); return c < 0 ? 0 : (c >= nc ? nc - 1 : c); };
    for (int i = 0; i < n; ++i) {
        long cx = cidx(xy[2 * i]), cy = cidx(xy[2 * i + 1]);
        for (long gy = std::max(0L, cy - 1); gy <= std::min(nc - 1, cy + 1); ++gy)
            for (long gx = std::max(0L, cx - 1); gx <= std::min(nc - 1, cx + 1); ++gx)
                for (int j = head[gy * nc + gx]; j >= 0; j = nxt[j]) {
                    double dx = xy[2 * i] - xy[2 * j], dy = xy[2 * i + 1] - xy[2 * j + 1];
                    if (std::sqrt(dx * dx + dy * dy) < radii[i] + radii[j])
                        return err = "initial disks overlap", BD_ERR_BAD_INPUT;
                }
        nxt[i] = head[cy * nc + cx];
        head[cy * nc + cx] = i;
    }
    return BD_OK;
}

int init_impl(Sim &s, int n, const double *xy, const double *radii, const int32_t *species, const double *theta,
              const bd_force_params *fp, const bd_params *p) {
    double rmax = 0.0;
    for (int i = 0; i < n; ++i) rmax = std::max(rmax, radii[i]);
    std::vector<double> fx, fy;
    frame_points(p->L, rmax, fx, fy);
    s.n = n;
    s.m = (int)fx.size();
    s.nv = n + s.m;
    s.S = fp->S;
    s.T = 2 * s.nv - 2;
    s.H = 3 * s.T;
    s.inf = s.nv;
    s.p = *p;
    s.fp = *fp;
    s.K.assign(fp->K, fp->K + fp->S * fp->S);
    s.fp.K = s.K.data();
    s.step = p->step0;
    s.fp32 = p->force_precision == BD_PREC_FP32;
    s.kind_fast = (fp->kind == BD_FORCE_POWER && fp->q == 2.0 && !(fp->cutoff > 0)) ? 1 : 0;
    s.use_nl = fp->cutoff > 0;
    check(hipGetDevice(&s.device), "hipGetDevice");
    check(hipStreamCreateWithFlags(&s.own_stream, hipStreamNonBlocking), "stream");
    s.stream = s.own_stream;

    // finite vertices: the disks, then the frame, then one padding entry for the infinite vertex
    const int nv = s.nv;
    std::vector<double> hx(nv + 1, 0.0), hy(nv + 1, 0.0), hth(n, 0.0), hrad(nv + 1, 0.0);
    for (int i = 0; i < n; ++i) {
        hx[i] = xy[2 * i];
        hy[i] = xy[2 * i + 1];
        hrad[i] = radii[i];
        if (theta) hth[i] = theta[i];
    }
    for (int k = 0; k < s.m; ++k) {
        hx[n + k] = fx[k];
        hy[n + k] = fy[k];
    }
    // species-sorted permutation (stable: ids ascending inside a species)
    std::vector<int> sorted(n), pos(n), block_start(s.S + 1, 0);
    for (int i = 0; i < n; ++i) ++block_start[species[i] + 1];
    for (int b = 0; b < s.S; ++b) block_start[b + 1] += block_start[b];
    {
        std::vector<int> fillp(block_start.begin(), block_start.end() - 1);
        for (int i = 0; i < n; ++i) {
            int k = fillp[species[i]]++;
            sorted[k] = i;
            pos[i] = k;
        }
    }
    setup_chunks(s, block_start);

    s.x = dalloc<double>(nv + 1);
    s.y = dalloc<double>(nv + 1);
    s.xo = dalloc<double>(nv + 1);
    s.yo = dalloc<double>(nv + 1);
    s.th = dalloc<double>(n);
    s.tho = dalloc<double>(n);
    s.rad = dalloc<double>(nv + 1);
    s.sp = dalloc<int>(n);
    s.sorted_id = dalloc<int>(n);
    s.pos_of = dalloc<int>(n);
    const size_t vec = s.fp32 ? sizeof(float2) : sizeof(double2);
    s.pj = dalloc<char>(vec * n);
    s.part = dalloc<char>(vec * n * (size_t)s.nchunks);
    s.chunks = dalloc<Chunk>(s.nchunks);
    s.Kd = dalloc<double>(s.S * s.S);
    s.fout = dalloc<double>(2 * (size_t)n);
    s.he_v = dalloc<int>(s.H);
    s.he_twin = dalloc<int>(s.H);
    s.vert_he = dalloc<int>(nv + 1);
    s.claim = dalloc<unsigned long long>(s.T);
    s.tri_stamp = dalloc<int>(s.T);
    s.moved = dalloc<int>(s.H);
    s.edge_stamp = dalloc<int>(s.H);
    s.vstamp = dalloc<int>(n + 1);
    s.wl[0] = dalloc<int>(s.H);
    s.wl[1] = dalloc<int>(s.H);
    s.cand = dalloc<int2>(s.H / 2 + 64);
    s.cand_won = dalloc<int>(s.H / 2 + 64);
    s.touched = dalloc<int>(n);
    s.newpos = dalloc<double2>(n);
    s.oldpos = dalloc<double2>(n);
    s.snap_v = dalloc<int>(s.H);
    s.snap_twin = dalloc<int>(s.H);
    s.snap_vh = dalloc<int>(nv + 1);
    s.xa = dalloc<double>(n);
    s.ya = dalloc<double>(n);
    s.xb = dalloc<double>(n);
    s.yb = dalloc<double>(n);
    s.ctl = dalloc<int>(N_CTL);
    if (s.use_nl) {
        const double rl = fp->cutoff + fp->skin;
        s.nl_nc = std::max(1, std::min(46000, (int)std::floor(p->L / rl)));
        s.nl_ncell = s.nl_nc * s.nl_nc;
        s.cell_count = dalloc<int>(s.nl_ncell + 1);
        s.cell_start = dalloc<int>(s.nl_ncell + 1);
        s.cell_fill = dalloc<int>(s.nl_ncell);
        s.cell_of = dalloc<int>(n);
        s.cell_items = dalloc<int>(n);
        s.nl = dalloc<int>((size_t)s.nl_cap * n);
        s.nl_cnt = dalloc<int>(n);
        s.xbuild = dalloc<double>(n);
        s.ybuild = dalloc<double>(n);
        s.fsr = dalloc<double2>(n);
        s.scan_bytes = verlet_scan_bytes(s.nl_ncell);
        s.scan_tmp = dalloc<char>(s.scan_bytes);
    }
    s.acc = dalloc<unsigned long long>(N_ACC);
    if (hipHostMalloc((void **)&s.hctl, sizeof(int) * N_CTL, hipHostMallocDefault) != hipSuccess) throw std::bad_alloc();
    if (hipHostMalloc((void **)&s.hacc, sizeof(unsigned long long) * N_ACC, hipHostMallocDefault) != hipSuccess)
        throw std::bad_alloc();

    check(hipMemcpyAsync(s.x, hx.data(), sizeof(double) * (nv + 1), hipMemcpyHostToDevice, s.stream), "x");
    check(hipMemcpyAsync(s.y, hy.data(), sizeof(double) * (nv + 1), hipMemcpyHostToDevice, s.stream), "y");
    check(hipMemcpyAsync(s.xo, hx.data(), sizeof(double) * (nv + 1), hipMemcpyHostToDevice, s.stream), "xo");
    check(hipMemcpyAsync(s.yo, hy.data(), sizeof(double) * (nv + 1), hipMemcpyHostToDevice, s.stream), "yo");
    check(hipMemcpyAsync(s.th, hth.data(), sizeof(double) * n, hipMemcpyHostToDevice, s.stream), "th");
    check(hipMemcpyAsync(s.tho, hth.data(), sizeof(double) * n, hipMemcpyHostToDevice, s.stream), "tho");
    check(hipMemcpyAsync(s.rad, hrad.data(), sizeof(double) * (nv + 1), hipMemcpyHostToDevice, s.stream), "rad");
    check(hipMemcpyAsync(s.sp, species, sizeof(int) * n, hipMemcpyHostToDevice, s.stream), "sp");
    check(hipMemcpyAsync(s.sorted_id, sorted.data(), sizeof(int) * n, hipMemcpyHostToDevice, s.stream), "sorted");
    check(hipMemcpyAsync(s.pos_of, pos.data(), sizeof(int) * n, hipMemcpyHostToDevice, s.stream), "pos");
    check(hipMemcpyAsync(s.chunks, s.chunks_h.data(), sizeof(Chunk) * s.nchunks, hipMemcpyHostToDevice, s.stream),
          "chunks");
    check(hipMemcpyAsync(s.Kd, s.K.data(), sizeof(double) * s.S * s.S, hipMemcpyHostToDevice, s.stream), "K");
    check(hipMemsetAsync(s.claim, 0, sizeof(unsigned long long) * s.T, s.stream), "claim");
    check(hipMemsetAsync(s.tri_stamp, 0, sizeof(int) * s.T, s.stream), "tri_stamp");
    check(hipMemsetAsync(s.edge_stamp, 0, sizeof(int) * s.H, s.stream), "edge_stamp");
    check(hipMemsetAsync(s.vstamp, 0, sizeof(int) * (n + 1), s.stream), "vstamp");
    check(hipMemsetAsync(s.acc, 0, sizeof(unsigned long long) * N_ACC, s.stream), "acc");
    check(hipMemsetAsync(s.ctl, 0, sizeof(int) * N_CTL, s.stream), "ctl");

    std::vector<int> hv, ht;
    if (host_delaunay(nv, hx.data(), hy.data(), hv, ht) != 0) {
        s.last_error = "initial Delaunay triangulation failed (coincident positions)";
        return BD_ERR_TRIANGULATION;
    }
    upload_topology(s, hv, ht);
    if (s.use_nl) verlet_rebuild(s);
    return BD_OK;
}

const char *err_name(int code) {
    switch (code) {
        case BD_OK: return "BD_OK";
        case BD_ERR_INVALID_ARG: return "BD_ERR_INVALID_ARG";
        case BD_ERR_BAD_INPUT: return "BD_ERR_BAD_INPUT";
        case BD_ERR_NO_CONVERGENCE: return "BD_ERR_NO_CONVERGENCE";
        case BD_ERR_TRIANGULATION: return "BD_ERR_TRIANGULATION";
        case BD_ERR_DEVICE: return "BD_ERR_DEVICE";
        case BD_ERR_OOM: return "BD_ERR_OOM";
        default: return "BD_ERR_UNKNOWN";
    }
}

template <typename F>
int guarded(Sim &s, F &&f) {
    try {
        return f();
    } catch (const DeviceError &e) {
        s.last_error = std::string(e.what) + ": " + hipGetErrorString(e.e);
        return BD_ERR_DEVICE;
    } catch (const std::bad_alloc &) {
        s.last_error = "out of memory";
        return BD_ERR_OOM;
    } catch (...) {
        s.last_error = "unexpected exception";
        return BD_ERR_DEVICE;
    }
}

}  // namespace
}  // namespace bd

using bd::Sim;

extern "C" {

const char *bd_strerror(int code) { return bd::err_name(code); }

const char *bd_last_error(const bd_sim *sim) { return sim ? sim->s.last_error.c_str() : ""; }

void bd_params_default(bd_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->D = 1.0;
    p->dt = 1e-4;
    p->overlap_factor = 1.0;
    p->cap_frac = 0.5;
    p->noise_clip = 3.0;
    p->contact_tol = 1e-9;
    p->max_overlap_rounds = 10000;
    p->max_flip_rounds = 200;
    p->force_precision = BD_PREC_FP64;
}

int bd_init(bd_sim **out, int32_t n, const double *xy, const double *radii, const int32_t *species,
            const double *theta, const bd_force_params *fp, const bd_params *p) {
    if (!out) return BD_ERR_INVALID_ARG;
    *out = nullptr;
    std::string err;
    int rc = bd::validate_args(n, xy, radii, species, theta, fp, p, err);
    if (rc != BD_OK) {
        std::fprintf(stderr, "bd_init: %s\n", err.c_str());
        return rc;
    }
    bd_sim *h = new (std::nothrow) bd_sim();
    if (!h) return BD_ERR_OOM;
    rc = bd::guarded(h->s, [&] { return bd::init_impl(h->s, n, xy, radii, species, theta, fp, p); });
    if (rc != BD_OK) {
        std::fprintf(stderr, "bd_init: %s\n", h->s.last_error.c_str());
        bd::free_all(h->s);
        delete h;
        return rc;
    }
    *out = h;
    return BD_OK;
}

int bd_step(bd_sim *sim, int64_t nsteps) {
    if (!sim || nsteps < 0) return BD_ERR_INVALID_ARG;
    Sim &s = sim->s;
    return bd::guarded(s, [&] {
        for (int64_t k = 0; k < nsteps; ++k) {
            int rc = bd::one_step(s);
            if (rc != BD_OK) return rc;
        }
        return (int)BD_OK;
    });
}

int bd_forces(bd_sim *sim, double *f_out) {
    if (!sim || !f_out) return BD_ERR_INVALID_ARG;
    Sim &s = sim->s;
    return bd::guarded(s, [&] {
        bd::compute_forces(s);
        if (s.use_nl) {
            bd::check(hipMemcpyAsync(f_out, s.fsr, sizeof(double) * 2 * s.n, hipMemcpyDeviceToHost, s.stream),
                      "forces copy");
        } else {
            bd::launch_reduce_forces(s);
            bd::check(hipMemcpyAsync(f_out, s.fout, sizeof(double) * 2 * s.n, hipMemcpyDeviceToHost, s.stream),
                      "forces copy");
        }
        bd::check(hipStreamSynchronize(s.stream), "sync");
        return (int)BD_OK;
    });
}

int bd_get_state(bd_sim *sim, double *xy_out, double *theta_out, int64_t *step_out, bd_stats *stats_out) {
    if (!sim) return BD_ERR_INVALID_ARG;
    Sim &s = sim->s;
    return bd::guarded(s, [&] {
        std::vector<double> hx(s.n), hy(s.n);
        if (xy_out) {
            bd::check(hipMemcpyAsync(hx.data(), s.x, sizeof(double) * s.n, hipMemcpyDeviceToHost, s.stream), "x");
            bd::check(hipMemcpyAsync(hy.data(), s.y, sizeof(double) * s.n, hipMemcpyDeviceToHost, s.stream), "y");
        }
        if (theta_out)
            bd::check(hipMemcpyAsync(theta_out, s.th, sizeof(double) * s.n, hipMemcpyDeviceToHost, s.stream), "th");
        bd::check(hipMemcpyAsync(s.hacc, s.acc, sizeof(unsigned long long) * bd::N_ACC, hipMemcpyDeviceToHost,
                                 s.stream),
                  "acc");
        bd::check(hipStreamSynchronize(s.stream), "sync");
        if (xy_out)
            for (int i = 0; i < s.n; ++i) {
                xy_out[2 * i] = hx[i];
                xy_out[2 * i + 1] = hy[i];
            }
        if (step_out) *step_out = s.step;
        if (stats_out) {
            bd_stats st = s.st;
            st.flips_total = (int64_t)s.hacc[bd::A_FLIPS];
            st.inversion_flips = (int64_t)s.hacc[bd::A_INV_FLIPS];
            st.reversals = (int64_t)s.hacc[bd::A_REVERSALS];
            st.noise_clamps = (int64_t)s.hacc[bd::A_NOISE_CLAMPS];
            st.cap_hits = (int64_t)s.hacc[bd::A_CAP_HITS];
            *stats_out = st;
        }
        return (int)BD_OK;
    });
}

int bd_get_triangulation(bd_sim *sim, int32_t *tri_out, int32_t cap, int32_t *ntri_out) {
    if (!sim || !tri_out || !ntri_out) return BD_ERR_INVALID_ARG;
    Sim &s = sim->s;
    return bd::guarded(s, [&] {
        std::vector<int> hv(s.H);
        bd::check(hipMemcpyAsync(hv.data(), s.he_v, sizeof(int) * s.H, hipMemcpyDeviceToHost, s.stream), "he_v");
        bd::check(hipStreamSynchronize(s.stream), "sync");
        int cnt = 0;
        for (int t = 0; t < s.T; ++t) {
            int a = hv[3 * t], b = hv[3 * t + 1], c = hv[3 * t + 2];
            if (a == s.inf || b == s.inf || c == s.inf) continue;
            if (cnt >= cap) {
                s.last_error = "triangle buffer too small";
                return (int)BD_ERR_INVALID_ARG;
            }
            tri_out[3 * cnt] = a;
            tri_out[3 * cnt + 1] = b;
            tri_out[3 * cnt + 2] = c;
            ++cnt;
        }
        *ntri_out = cnt;
        return (int)BD_OK;
    });
}

int bd_get_frame(bd_sim *sim, double *xy_out, int32_t cap, int32_t *m_out) {
    if (!sim || !m_out) return BD_ERR_INVALID_ARG;
    Sim &s = sim->s;
    *m_out = s.m;
    if (!xy_out) return BD_OK;
    if (cap < s.m) {
        s.last_error = "frame buffer too small";
        return BD_ERR_INVALID_ARG;
    }
    return bd::guarded(s, [&] {
        std::vector<double> hx(s.m), hy(s.m);
        bd::check(hipMemcpyAsync(hx.data(), s.x + s.n, sizeof(double) * s.m, hipMemcpyDeviceToHost, s.stream), "x");
        bd::check(hipMemcpyAsync(hy.data(), s.y + s.n, sizeof(double) * s.m, hipMemcpyDeviceToHost, s.stream), "y");
        bd::check(hipStreamSynchronize(s.stream), "sync");
        for (int k = 0; k < s.m; ++k) {
            xy_out[2 * k] = hx[k];
            xy_out[2 * k + 1] = hy[k];
        }
        return (int)BD_OK;
    });
}

int bd_set_positions(bd_sim *sim, const double *xy) {
    if (!sim || !xy) return BD_ERR_INVALID_ARG;
    Sim &s = sim->s;
    return bd::guarded(s, [&] {
        std::vector<double> hx(s.n), hy(s.n), hr(s.n);
        bd::check(hipMemcpyAsync(hr.data(), s.rad, sizeof(double) * s.n, hipMemcpyDeviceToHost, s.stream), "rad");
        bd::check(hipStreamSynchronize(s.stream), "sync");
        for (int i = 0; i < s.n; ++i) {
            hx[i] = xy[2 * i];
            hy[i] = xy[2 * i + 1];
            if (!std::isfinite(hx[i]) || !std::isfinite(hy[i]) || hx[i] < hr[i] || hx[i] > s.p.L - hr[i] ||
                hy[i] < hr[i] || hy[i] > s.p.L - hr[i]) {
                s.last_error = "position outside the walls or not finite";
                return (int)BD_ERR_BAD_INPUT;
            }
        }
        bd::check(hipMemcpyAsync(s.xo, s.x, sizeof(double) * s.n, hipMemcpyDeviceToDevice, s.stream), "xo");
        bd::check(hipMemcpyAsync(s.yo, s.y, sizeof(double) * s.n, hipMemcpyDeviceToDevice, s.stream), "yo");
        bd::check(hipMemcpyAsync(s.x, hx.data(), sizeof(double) * s.n, hipMemcpyHostToDevice, s.stream), "x");
        bd::check(hipMemcpyAsync(s.y, hy.data(), sizeof(double) * s.n, hipMemcpyHostToDevice, s.stream), "y");
        bd::fill_int(s, s.ctl, bd::N_CTL, 0);
        s.need_rebuild = true;
        bd::Cursor c;
        return bd::host_repair(s, c, true, false, bd::MoveFrom::Previous, 0);
    });
}

int bd_set_stream(bd_sim *sim, void *hip_stream) {
    if (!sim) return BD_ERR_INVALID_ARG;
    Sim &s = sim->s;
    return bd::guarded(s, [&] {
        bd::check(hipStreamSynchronize(s.stream), "sync");
        s.stream = hip_stream ? (hipStream_t)hip_stream : s.own_stream;
        return (int)BD_OK;
    });
}

int bd_enable_kernel_timing(bd_sim *sim, int enable) {
    if (!sim) return BD_ERR_INVALID_ARG;
    Sim &s = sim->s;
    return bd::guarded(s, [&] {
        bd::check(hipStreamSynchronize(s.stream), "sync");
        for (auto &e : s.ev) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        s.ev.clear();
        s.timed_ms = 0.0;
        s.timed_launches = 0;
        s.timing = enable != 0;
        return (int)BD_OK;
    });
}

int bd_kernel_time(bd_sim *sim, double *force_ms, int64_t *force_launches) {
    if (!sim) return BD_ERR_INVALID_ARG;
    Sim &s = sim->s;
    return bd::guarded(s, [&] {
        bd::check(hipStreamSynchronize(s.stream), "sync");
        for (auto &e : s.ev) {
            float ms = 0.f;
            bd::check(hipEventElapsedTime(&ms, e.first, e.second), "elapsed");
            s.timed_ms += ms;
            ++s.timed_launches;
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        s.ev.clear();
        if (force_ms) *force_ms = s.timed_ms;
        if (force_launches) *force_launches = s.timed_launches;
        return (int)BD_OK;
    });
}

void bd_destroy(bd_sim *sim) {
    if (!sim) return;
    (void)hipStreamSynchronize(sim->s.stream);
    bd::free_all(sim->s);
    delete sim;
}

}  // extern "C"
