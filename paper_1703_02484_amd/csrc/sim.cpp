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
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "bd_internal.h"
#include "geom.h"

namespace bd {
namespace {

// library order -> caller order (perm: library index -> caller index)
// The positions are read from the packed copy, so every state a caller sees has been through it.
__global__ void k_to_caller(int n, const int *__restrict__ perm, const double2 *__restrict__ pos,
                            const double *__restrict__ th, double *__restrict__ xy, double *__restrict__ th_out) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) {
        const size_t i = (size_t)perm[k];
        if (xy) {
            xy[2 * i] = pos[k].x;
            xy[2 * i + 1] = pos[k].y;
        }
        if (th_out) th_out[i] = th[k];
    }
}

__global__ void k_scatter2(int n, const int *__restrict__ perm, const double2 *__restrict__ in,
                           double2 *__restrict__ out) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[perm[k]] = in[k];
}

__global__ void k_gather2(int n, const int *__restrict__ perm, const double2 *__restrict__ in,
                          double2 *__restrict__ out) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = in[perm[k]];
}

__global__ void k_fill_int(int *p, int count, int value) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

struct DeviceError {
    hipError_t e;
    const char *what;
};

// A request the library cannot serve (reported as BD_ERR_INVALID_ARG).
struct UnsupportedError {
    const char *what;
};

inline void check(hipError_t e, const char *what) {
    if (e != hipSuccess) throw DeviceError{e, what};
}

// Device memory comes from hipMalloc or from the allocator installed with
// bd_set_allocator when the handle was created (the handle keeps using the
// one it started with).  The handle being served is thread-local while a call
// runs, so the helpers below need no handle argument.
struct Allocator {
    void *(*alloc)(size_t, void *, void *) = nullptr;
    void (*free)(void *, void *, void *) = nullptr;
    void *ctx = nullptr;
};
std::mutex g_alloc_mu;
Allocator g_alloc;
thread_local Sim *tl_sim = nullptr;

struct UseSim {   // marks the handle served by this thread for the duration of a call
    Sim *prev;
    explicit UseSim(Sim &s) : prev(tl_sim) { tl_sim = &s; }
    ~UseSim() { tl_sim = prev; }
};

void *raw_alloc(size_t bytes) {
    Sim *s = tl_sim;
    if (s && s->user_alloc) {
        void *p = s->user_alloc(bytes, (void *)s->stream, s->user_ctx);
        if (!p) throw std::bad_alloc();
        return p;
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) throw std::bad_alloc();
    return p;
}

void dfree(void *p) {
    if (!p) return;
    Sim *s = tl_sim;
    if (s && s->user_free)
        s->user_free(p, (void *)s->stream, s->user_ctx);
    else
        (void)hipFree(p);
}

template <typename T>
T *dalloc(size_t count) {
    if (count == 0) count = 1;
    return (T *)raw_alloc(count * sizeof(T));
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
    std::vector<int> vh(s.nv + s.R, -1);
    for (int h = 0; h < s.H; ++h) vh[he_v[h]] = h;
    check(hipMemcpyAsync(s.he_v, he_v.data(), sizeof(int) * s.H, hipMemcpyHostToDevice, s.stream), "he_v");
    check(hipMemcpyAsync(s.he_twin, he_twin.data(), sizeof(int) * s.H, hipMemcpyHostToDevice, s.stream), "twin");
    check(hipMemcpyAsync(s.vert_he, vh.data(), sizeof(int) * (s.nv + s.R), hipMemcpyHostToDevice, s.stream), "vh");
    check(hipStreamSynchronize(s.stream), "topology upload");
}

// Delaunay triangulation of every system from host positions (global vertex
// ids: disks, then frame points, then the infinite vertices).  System r owns
// triangles [toff_r, toff_{r+1}); systems are independent, so they are
// triangulated in parallel.  Returns 0, or -1 if one of them failed.
int host_dt_all(Sim &s, const double *hx, const double *hy, std::vector<int> &hv, std::vector<int> &ht) {
    hv.assign(s.H, -1);
    ht.assign(s.H, -1);
    std::atomic<int> next{0}, failed{0};
    auto work = [&] {
        std::vector<double> lx, ly;
        std::vector<int> lv, lt;
        for (int r = next++; r < s.R; r = next++) {
            const int d0 = s.off_h[r], nr = s.off_h[r + 1] - d0;
            const int f0 = s.n + s.foff_h[r], mr = s.foff_h[r + 1] - s.foff_h[r];
            const int vr = nr + mr;
            lx.resize(vr);
            ly.resize(vr);
            for (int i = 0; i < nr; ++i) {
                lx[i] = hx[d0 + i];
                ly[i] = hy[d0 + i];
            }
            for (int k = 0; k < mr; ++k) {
                lx[nr + k] = hx[f0 + k];
                ly[nr + k] = hy[f0 + k];
            }
            const int hb = 3 * s.toff_h[r], hr = 3 * (s.toff_h[r + 1] - s.toff_h[r]);
            const int rc = s.period > 0.0 ? host_torus_delaunay(nr, lx.data(), ly.data(), s.L_h[r], lv, lt)
                                          : host_delaunay(vr, lx.data(), ly.data(), lv, lt);
            if (rc != 0 || (int)lv.size() != hr) {
                failed = 1;
                continue;
            }
            for (int h = 0; h < hr; ++h) {
                const int v = lv[h];
                hv[hb + h] = v < nr ? d0 + v : (v < vr ? f0 + (v - nr) : s.inf + r);
                ht[hb + h] = hb + lt[h];
            }
        }
    };
    const int nth = std::max(1, std::min({s.R, 16, (int)std::thread::hardware_concurrency()}));
    std::vector<std::thread> pool;
    for (int t = 1; t < nth; ++t) pool.emplace_back(work);
    work();
    for (auto &t : pool) t.join();
    return failed ? -1 : 0;
}

// Host rebuild of DT(current positions).  Returns BD_OK or BD_ERR_TRIANGULATION.
int host_rebuild(Sim &s) {
    std::vector<double> hx(s.nv), hy(s.nv);
    check(hipMemcpyAsync(hx.data(), s.x, sizeof(double) * s.nv, hipMemcpyDeviceToHost, s.stream), "x");
    check(hipMemcpyAsync(hy.data(), s.y, sizeof(double) * s.nv, hipMemcpyDeviceToHost, s.stream), "y");
    check(hipStreamSynchronize(s.stream), "rebuild download");
    std::vector<int> hv, ht;
    if (host_dt_all(s, hx.data(), hy.data(), hv, ht) != 0) {
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

bool tail_fused(const Sim &s);
int tail_mode_of(const Sim &s);
void update_ovl_phase(Sim &s, const int *h, const std::vector<int> &orounds, int rounds);

// Evaluation mode of the first flip round after a move: count reversed edges, and with halving
// enabled also flag the step so that its repair check halts it.
inline int rev_mode(const Sim &s) { return s.p.max_dt_halvings > 0 ? 2 : 1; }

// ------------------------------------------------------------------ budgeted sequence
// Enqueues one repair of `rounds` flip rounds with no host read-back: a
// topology snapshot, the rounds, the validation and the check that halts the
// step when the budget was too small or a triangle stayed inverted.
// The overlap detection that follows a repair, run in the same launch as the
// repair's validation (same triangles or stars): round slot, stamp, check.
struct FusedDetect {
    int k, stamp, check;
};

void enqueue_repair(Sim &s, Cursor &c, bool full, bool reversal, int rounds, std::vector<int> *first_slots,
                    int oround = -1, const FusedDetect *fd = nullptr, int multi = 1 << 30) {
    // The repair after the move keeps the triangulation of the step's start
    // positions: a later repair of the same step that fails replays the
    // whole move from there (the Delaunay triangulation of the end positions
    // is unique), so the repairs after overlap rounds need no copy of their own.
    if (full) launch_snapshot(s);
    const int rep = c.take_rep();
    if (first_slots) first_slots->push_back(c.slot);
    int last = -1;
    if (full && rounds >= 1 && tail_fused(s)) {
        // the first evaluation scans every edge; the rest of the rounds run in one workgroup
        const int r0 = ++s.round_id;
        const int slot0 = c.take_slot();
        launch_flip_eval_full(s, r0, slot0, reversal ? rev_mode(s) : 0);
        last = slot0;
        for (int j = 1; j < rounds; ++j) {
            ++s.round_id;
            last = c.take_slot();
        }
        launch_repair_rounds(s, r0, slot0, rounds);
        if (fd)
            launch_ovl_detect(s, fd->stamp, fd->k, fd->check, rep, last);
        else
            launch_validate(s, rep, last);
        return;
    }
    // the first `multi` rounds (the long worklists) on many workgroups, the rest in one workgroup
    // launch that stops at the first round with nothing to do
    const int m = std::min(rounds, std::max(1, multi));
    for (int j = 0; j < m; ++j) {
        const int r = ++s.round_id;
        const int slot = c.take_slot();
        if (j == 0 && full)
            launch_flip_eval_full(s, r, slot, reversal ? rev_mode(s) : 0);
        else
            launch_flip_eval_list(s, r, slot);
        launch_flip_apply(s, r, slot);
        launch_flip_fix(s, r, slot);
        last = slot;
    }
    if (m < rounds) {
        const int r0 = s.round_id + 1, slot0 = c.slot;
        for (int j = m; j < rounds; ++j) {
            ++s.round_id;
            last = c.take_slot();
        }
        launch_repair_rounds(s, r0, slot0, rounds - m, false);
    }
    if (fd && oround >= 0)
        launch_validate_detect_local(s, rep, oround, last, fd->stamp, fd->k, fd->check);
    else if (fd)
        launch_ovl_detect(s, fd->stamp, fd->k, fd->check, rep, last);
    else if (oround >= 0)
        launch_validate_local(s, rep, oround, last);
    else
        launch_validate(s, rep, last);
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
            launch_flip_eval_full(s, r, slot, reversal && it == 0 ? rev_mode(s) : 0);
        else
            launch_flip_eval_list(s, r, slot);
        read_ctl(s);
        if (s.hctl[K_CAND + slot] > 0) ++s.st.flip_rounds_total;   // rounds that found an edge to flip
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
        check(hipMemcpyAsync(s.vert_he, s.snap_vh, sizeof(int) * (s.nv + s.R), hipMemcpyDeviceToDevice, s.stream),
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
    launch_pack_xy(s, s.n);
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
    launch_pack_xy(s, s.n);
    check(hipMemcpyAsync(s.th, s.tho, sizeof(double) * s.n, hipMemcpyDeviceToDevice, s.stream), "rollback th");
    fill_int(s, s.ctl, N_CTL, 0);
    s.need_rebuild = true;
    if (s.ovl_method == 0) host_rebuild(s);
}

void drop_graphs(Sim &s) {
    for (auto &e : s.graphs) {
        if (e.second.pre) (void)hipGraphExecDestroy(e.second.pre);
        if (e.second.force) (void)hipGraphExecDestroy(e.second.force);
        if (e.second.post) (void)hipGraphExecDestroy(e.second.post);
    }
    s.graphs.clear();
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
        if (need > 96 || s.nl_cap >= 96)
            throw UnsupportedError{"more than 96 disks within cutoff + skin of one disk (neighbour list capacity)"};
        dfree(s.nl);
        s.nl = nullptr;
        drop_graphs(s);   // captured steps hold the old list pointer
        s.nl_cap = 96;
        s.nl = dalloc<int>((size_t)s.nl_cap * s.n);
    }
}

void timed(Sim &s, const std::function<void()> &work);

void compute_forces(Sim &s) {
    if (s.use_nl && s.need_rebuild) verlet_rebuild(s);
    if (!s.use_nl) launch_cast(s);
    timed(s, [&] {
        if (s.use_nl)
            launch_force_nl(s);
        else
            launch_force(s);
    });
}

// Skin test for the next step's lists (short-range path only).  Inside an
// enqueued step (read_back false) the flag is still clear from the step's start.
void skin_check(Sim &s, bool read_back) {
    if (!s.use_nl) return;
    if (read_back) zero_ctl(s, K_NL_REBUILD);
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

// Host-driven overlap rounds of the list method (Sec. 5 variant) from round
// index `rounds` on; a detection that finds the lists possibly incomplete
// rebuilds them and is repeated.
int host_overlap_loop_nl(Sim &s, Cursor &c, int &rounds) {
    const int max_rounds = s.p.max_overlap_rounds > 0 ? s.p.max_overlap_rounds : 10000;
    for (int stale = 0;;) {
        const int k = c.take_oround();
        zero_ctl(s, K_TOUCH + k);
        zero_ctl(s, K_OVL + k);
        zero_ctl(s, K_NL_STALE);
        launch_ovl_nl_gather(s, k);
        read_ctl(s);
        if (s.hctl[K_NL_STALE] != 0) {
            if (++stale > 1) {   // right after a rebuild every disk sits at its build position
                s.last_error = "neighbour lists stale right after a rebuild";
                return BD_ERR_DEVICE;
            }
            verlet_rebuild(s);
            continue;
        }
        stale = 0;
        const int npairs = s.hctl[K_OVL + k];
        if (npairs == 0) return BD_OK;
        if (rounds >= max_rounds) {
            s.last_error = "overlap correction did not converge within max_overlap_rounds";
            return BD_ERR_NO_CONVERGENCE;
        }
        ++rounds;
        s.st.overlap_edges_total += npairs;
        launch_ovl_nl_apply(s, k, false);
    }
}

// Puts the step counter and the stamp bases of the coming step in device
// memory (stream-ordered); later launches pass stamps relative to them.
void write_base(Sim &s) {
    s.hbase->step = s.step;
    s.hbase->rbase = s.round_id;
    s.hbase->vbase = s.vround;
    s.hbase->stop = 0;
    s.hbase->batch_idx = 0;
    s.hbase->nl_req = 0;   // the host rebuilds lists that are due before it queues steps
    s.hbase->nl_now = 0;
    check(hipMemcpyAsync(s.dbase, s.hbase, sizeof(StepBase), hipMemcpyHostToDevice, s.stream), "step base");
    s.rbase = s.round_id;
    s.vbase = s.vround;
}

// Overlap rounds enqueued per step: the adaptive budget, never more than the
// caller's round cap (the host loop enforces the cap beyond that) nor more
// than the step's flip-round slots hold.
int overlaps_budget(const Sim &s) {
    const int cap = s.p.max_overlap_rounds > 0 ? s.p.max_overlap_rounds : 10000;
    const int nover = std::min(s.budget.overlaps, cap);
    int slots = s.budget.em;
    for (int j = 0; j < nover; ++j) {
        if (slots + s.budget.ovl[j] > MAXR) return j;
        slots += s.budget.ovl[j];
    }
    return nover;
}

// How the overlap rounds after the first detection are launched (bd_set_tail_mode).
int tail_mode_of(const Sim &s) {
    // Library choice: one workgroup for handles of at most 16,384 disks, measured per step with
    // graph replay on 16,384 disks 10-21 % faster than launching every phase (the lists of the
    // later rounds hold tens of items and a launch costs more than a barrier) and within 2 % of
    // mode 2 from 4,096 to 16,384 disks.  Larger handles: the first rounds of each repair and the
    // overlap rounds that queue many disks launched per phase, the rest in one workgroup (mode 2),
    // measured 6-18 % faster than mode 1 on 32,768 disks, 0.96 vs 1.11 ms per step (mode 0) on
    // 65,536 and 0.64 vs 0.84 ms on 1M (all in one workgroup: 1.25 ms and 13.6 ms; the large
    // phases are latency chains over thousands of items that spread better over many CUs).
    constexpr int kTailMaxDisks = 16384;
    if (s.tail_mode != -1) return s.tail_mode;
    return s.n <= kTailMaxDisks ? 1 : 2;
}

// Mode 2: overlap rounds launched per phase before the one-workgroup tail.  Rounds 0, 1, ... are,
// up to the first round whose detection queued at most kTailItems disks (half of what the tail's
// workgroup of 1024 threads takes in one pass of each phase) in the current and the previous
// window of kTouchWindow steps; that round and the later ones run in the tail.  Measured per step
// with graph replay: 512 and 128 within 1 % of each other on 65,536 and 1M disks and on 16,384
// disks with the contact factor; 2048 is 25-40 % slower on the first two.
void update_ovl_phase(Sim &s, const int *h, const std::vector<int> &orounds, int rounds) {
    constexpr int kTouchWindow = 64, kTailItems = 512;
    for (int j = 0; j < rounds && j < (int)orounds.size() && j < MAXO; ++j)
        s.touch_hi[j] = std::max(s.touch_hi[j], h[K_TOUCH + orounds[j]]);
    if (++s.touch_steps >= kTouchWindow) {
        std::copy(s.touch_hi, s.touch_hi + MAXO, s.touch_prev);
        std::fill(s.touch_hi, s.touch_hi + MAXO, 0);
        s.touch_steps = 0;
    }
    int phase = 0;
    while (phase < MAXO && std::max(s.touch_hi[phase], s.touch_prev[phase]) > kTailItems) ++phase;
    s.ovl_phase = phase;
}

// Whether the overlap rounds after the first detection run in one workgroup.
bool tail_fused(const Sim &s) { return tail_mode_of(s) == 1; }

// The budgeted part of a step after the update: repair rounds, then overlap
// rounds each with its repair, the final overlap check, the skin test.
void enqueue_rounds(Sim &s, Cursor &c, std::vector<int> &orounds, std::vector<int> &rep_first) {
    const int nover = overlaps_budget(s);
    const int mode = tail_mode_of(s);
    if (mode != 1 || nover > MAXTAIL || nover == 0) {
        // Each detection runs in the launch that validates the repair before it: the first one
        // scans every triangle (after the repair of the move), later ones the stars of the disks
        // the previous round moved and the diagonals flipped since; the launch's last workgroup
        // runs the repair's check, then the round's (and after the last budgeted round the final one).
        // Mode 2: each repair launches its first rounds on many workgroups and the rest in one, and
        // after the first ovl_phase overlap rounds the others run in one workgroup (k_tail).
        const bool hybrid = mode == 2;
        const int per_phase =
            hybrid ? std::min(nover, std::max({0, s.ovl_phase, nover - MAXTAIL})) : nover;   // the tail holds MAXTAIL
        int k = c.take_oround();
        orounds.push_back(k);
        FusedDetect fd{k, ++s.vround, nover == 0 ? 2 : 1};
        enqueue_repair(s, c, true, true, s.budget.em, &rep_first, -1, &fd, hybrid ? s.multi_em : 1 << 30);
        for (int j = 0; j < per_phase; ++j) {
            launch_ovl_gather(s, k);
            launch_ovl_apply(s, k, s.round_id + 1, c.slot);
            const int knext = c.take_oround();
            orounds.push_back(knext);
            FusedDetect fn{knext, ++s.vround, j + 1 == nover ? 2 : 1};
            enqueue_repair(s, c, false, false, s.budget.ovl[j], &rep_first, k, &fn,
                           hybrid ? s.multi_ovl : 1 << 30);
            k = knext;
        }
        if (per_phase < nover) {
            // the remaining rounds in one workgroup; the detection for the first of them (slot k)
            // ran with the last repair's validation
            TailPlan plan{};
            plan.nover = nover - per_phase;
            plan.f = s.p.overlap_factor;
            plan.cap_frac = s.p.cap_frac;
            plan.keep = 1.0 - s.p.contact_tol;
            for (int jj = 0; jj < plan.nover; ++jj) {
                if (jj > 0) {
                    k = c.take_oround();
                    orounds.push_back(k);
                    plan.stamp[jj] = ++s.vround - s.vbase;
                } else {
                    plan.stamp[0] = 0;
                }
                plan.k[jj] = k;
                plan.next_round[jj] = s.round_id + 1 - s.rbase;
                plan.slot0[jj] = c.slot;
                plan.rep[jj] = c.take_rep();
                rep_first.push_back(c.slot);
                plan.rounds[jj] = s.budget.ovl[per_phase + jj];
                for (int r = 0; r < plan.rounds[jj]; ++r) {
                    ++s.round_id;
                    c.take_slot();
                }
            }
            k = c.take_oround();
            orounds.push_back(k);
            plan.k[plan.nover] = k;
            plan.stamp[plan.nover] = ++s.vround - s.vbase;
            launch_tail(s, plan);
        }
        skin_check(s, false);
        return;
    }
    enqueue_repair(s, c, true, true, s.budget.em, &rep_first);
    // the first detection after the move scans every edge, later ones only
    // what round k-1 changed; the detection's last workgroup runs the round's
    // check (and after the last budgeted round the final check)
    auto detect = [&](int k, int check) {
        const int stamp = ++s.vround;
        if (orounds.size() == 1)
            launch_ovl_detect(s, stamp, k, check);
        else
            launch_ovl_detect_local(s, stamp, k, orounds[orounds.size() - 2], check);
    };
    // rounds after the first detection in one workgroup (same slots, stamps and round ids)
    TailPlan plan{};
    plan.nover = nover;
    plan.f = s.p.overlap_factor;
    plan.cap_frac = s.p.cap_frac;
    plan.keep = 1.0 - s.p.contact_tol;
    for (int j = 0; j < nover; ++j) {
        const int k = c.take_oround();
        orounds.push_back(k);
        plan.k[j] = k;
        if (j == 0) {
            detect(k, 1);
            plan.stamp[0] = 0;
        } else {
            plan.stamp[j] = ++s.vround - s.vbase;
        }
        plan.next_round[j] = s.round_id + 1 - s.rbase;
        plan.slot0[j] = c.slot;
        plan.rep[j] = c.take_rep();
        rep_first.push_back(c.slot);
        plan.rounds[j] = s.budget.ovl[j];
        for (int r = 0; r < plan.rounds[j]; ++r) {
            ++s.round_id;
            c.take_slot();
        }
    }
    const int k = c.take_oround();
    orounds.push_back(k);
    plan.k[nover] = k;
    plan.stamp[nover] = ++s.vround - s.vbase;
    launch_tail(s, plan);
    skin_check(s, false);
}

// The budgeted overlap rounds of the list method: gather and apply per round,
// then a last detection that halts the step if overlaps remain; the skin test.
void enqueue_rounds_nl(Sim &s, Cursor &c, std::vector<int> &orounds) {
    const int cap = s.p.max_overlap_rounds > 0 ? s.p.max_overlap_rounds : 10000;
    const int nover = std::min({s.budget.overlaps, cap, MAXO - 1});
    // rounds 0 .. nfull-1 as full passes over every disk (round 0 after the move always), the rest in one
    // workgroup over the disks near those the round before moved: launch form 0 every round as a full
    // pass, 1 every round after the first in one workgroup, 2 the rounds that recently moved many disks
    // as full passes (same results in every form)
    const int mode = tail_mode_of(s);
    const int phase = mode == 0 ? nover + 1 : (mode == 1 ? 1 : s.nl_phase);
    const int nfull = std::min(nover + 1, std::max(1, phase));
    for (int j = 0; j < nfull; ++j) {
        const int k = c.take_oround();
        orounds.push_back(k);
        launch_ovl_nl_gather(s, k);
        launch_ovl_nl_apply(s, k, j == nover);
    }
    if (nfull <= nover) {
        NlTailPlan p{};
        p.nr = nover + 1 - nfull;
        p.kprev = orounds.back();
        for (int r = 0; r < p.nr; ++r) {
            p.k[r] = c.take_oround();
            orounds.push_back(p.k[r]);
        }
        p.stamp0 = s.vround + 1 - s.vbase;
        s.vround += p.nr;
        p.final_last = 1;
        launch_nl_tail(s, p);
    }
    skin_check(s, false);
}

// List overlap rounds launched as full passes: round j >= 1 joins the one-workgroup rest once the round
// before it recently moved at most kNlTailItems disks (over the current and the previous window of
// kTouchWindow steps); its disks are then those and their listed neighbours, a few times as many.
// (The window is the one update_ovl_phase keeps: a handle runs one overlap method.)  Limits of 128 to 1024
// measured within 1 % on 1M disks; 2048 and above let rounds that moved thousands of disks into the one
// workgroup, which then takes longer than a pass over every disk.
void update_nl_phase(Sim &s, const int *h, const std::vector<int> &orounds, int rounds) {
    constexpr int kTouchWindow = 64, kNlTailItems = 512;
    for (int j = 0; j < rounds && j < (int)orounds.size() && j < MAXO; ++j)
        s.touch_hi[j] = std::max(s.touch_hi[j], h[K_TOUCH + orounds[j]]);
    if (++s.touch_steps >= kTouchWindow) {
        std::copy(s.touch_hi, s.touch_hi + MAXO, s.touch_prev);
        std::fill(s.touch_hi, s.touch_hi + MAXO, 0);
        s.touch_steps = 0;
    }
    int phase = 1;
    while (phase < MAXO && std::max(s.touch_hi[phase - 1], s.touch_prev[phase - 1]) > kNlTailItems) ++phase;
    s.nl_phase = phase;
}

hipGraphExec_t capture(Sim &s, const std::function<void()> &enqueue) {
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
    check(hipStreamBeginCapture(s.stream, hipStreamCaptureModeRelaxed), "begin capture");
    enqueue();
    check(hipStreamEndCapture(s.stream, &g), "end capture");
    hipError_t rc = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    check(rc, "graph instantiate");
    return e;
}

// The captured step for the current round budgets (captured on first use):
// [clear counters, cast] [force] [update, budgeted rounds, checks].  Stamps
// inside are relative to the bases of the step being replayed.
Sim::StepGraph &step_graph(Sim &s) {
    const int nover = s.ovl_method == 1 ? s.budget.overlaps : overlaps_budget(s);
    std::vector<int> key = {s.budget.em, nover, tail_mode_of(s), s.multi_em, s.multi_ovl, s.ovl_phase, s.nl_phase};
    for (int j = 0; j < nover; ++j) key.push_back(s.budget.ovl[j]);
    for (auto &e : s.graphs)
        if (e.first == key) return e.second;
    if (s.graphs.size() >= kMaxGraphs) {   // the least recently captured goes (nothing of it is in flight)
        Sim::StepGraph &old = s.graphs.front().second;
        (void)hipGraphExecDestroy(old.pre);
        (void)hipGraphExecDestroy(old.force);
        (void)hipGraphExecDestroy(old.post);
        s.graphs.erase(s.graphs.begin());
    }
    Sim::StepGraph g;
    // stamps inside the graph count from the base of the step it is replayed for
    const int r0 = s.round_id, v0 = s.vround;
    const int rbase_live = s.rbase, vbase_live = s.vbase;
    s.rbase = r0;
    s.vbase = v0;
    g.pre = capture(s, [&] {
        if (s.use_nl) {
            launch_step_begin(s);
            launch_verlet_build_requested(s);
        } else {
            launch_step_begin_cast(s);
        }
    });
    g.force = capture(s, [&] {
        if (s.use_nl)
            launch_force_nl(s);
        else
            launch_force(s);
    });
    Cursor c;
    g.post = capture(s, [&] {
        launch_em(s);
        if (s.ovl_method == 1)
            enqueue_rounds_nl(s, c, g.orounds);
        else
            enqueue_rounds(s, c, g.orounds, g.rep_first);
        launch_step_end(s, s.round_id - r0, s.vround - v0);
    });
    g.r_used = s.round_id - r0;
    g.v_used = s.vround - v0;
    g.c_slot = c.slot;
    g.c_rep = c.rep;
    g.c_oround = c.oround;
    s.round_id = r0;   // capturing ran nothing
    s.vround = v0;
    s.rbase = rbase_live;
    s.vbase = vbase_live;
    s.graphs.emplace_back(key, std::move(g));
    return s.graphs.back().second;
}

void timed(Sim &s, const std::function<void()> &work) {
    hipEvent_t a = nullptr, b = nullptr;
    if (s.timing) {
        check(hipEventCreate(&a), "event");
        check(hipEventCreate(&b), "event");
        check(hipEventRecord(a, s.stream), "event record");
    }
    work();
    if (s.timing) {
        check(hipEventRecord(b, s.stream), "event record");
        s.ev.emplace_back(a, b);
    }
}

struct StepPlan {
    Cursor c;
    std::vector<int> orounds, rep_first;   // overlap-round slot and first round slot of each repair
    Budgets b;                             // round budgets the step ran with
    int overlaps = 0;                      // overlap rounds enqueued
};

int finish_step(Sim &s, const int *h_in, const StepPlan &plan);

void copy_d(Sim &s, void *dst, const void *src, size_t bytes) {
    check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s.stream), "device copy");
}

// Positions and angles back to those before the last move (kept by the update kernel) and the
// triangulation back to its snapshot taken before that move's repair.
void undo_move(Sim &s) {
    const size_t dn = sizeof(double) * s.n;
    copy_d(s, s.x, s.xo, dn);
    copy_d(s, s.y, s.yo, dn);
    launch_pack_xy(s, s.n);
    copy_d(s, s.th, s.tho, dn);
    copy_d(s, s.he_v, s.snap_v, sizeof(int) * s.H);
    copy_d(s, s.he_twin, s.snap_twin, sizeof(int) * s.H);
    copy_d(s, s.vert_he, s.snap_vh, sizeof(int) * (s.nv + s.R));
}

// Interval (level, index) of a step whose move reversed a Delaunay edge
// (Sec. 4.3: discard the move and repeat with a smaller time step), run from
// the host: forces at the current positions, the move over dt / 2^level with
// the Brownian-bridge noise of this interval, the repair (its first round
// counts reversed edges), then the overlap loop.  A move that reverses an
// edge again is undone and split while level < max_dt_halvings.
int halved_interval(Sim &s, Cursor &c, int level, unsigned index, int &rounds) {
    if (s.use_nl) skin_check(s, true);   // the lists must hold at this interval's positions
    compute_forces(s);
    launch_em(s, level, index);
    launch_snapshot(s);
    zero_ctl(s, K_REV);
    int rc = host_repair(s, c, true, true, MoveFrom::Previous, 0);
    if (rc != BD_OK) return rc;
    read_ctl(s);
    if (s.hctl[K_REV] != 0 && level < s.p.max_dt_halvings) {
        ++s.st.dt_halvings;
        undo_move(s);
        rc = halved_interval(s, c, level + 1, 2 * index, rounds);
        if (rc != BD_OK) return rc;
        return halved_interval(s, c, level + 1, 2 * index + 1, rounds);
    }
    return host_overlap_loop(s, c, rounds);
}

// A step halted because its move reversed a Delaunay edge: undo the move and
// redo the step as two halves.  On error the state returns to the step's start.
int redo_step_in_halves(Sim &s, Cursor &c, int &rounds) {
    write_base(s);   // clears a graph batch's stop flag, which would keep the update and force kernels idle
    undo_move(s);
    const size_t dn = sizeof(double) * s.n;
    if (!s.xs) {
        s.xs = dalloc<double>(s.n);
        s.ys = dalloc<double>(s.n);
        s.ths = dalloc<double>(s.n);
    }
    copy_d(s, s.xs, s.x, dn);
    copy_d(s, s.ys, s.y, dn);
    copy_d(s, s.ths, s.th, dn);
    ++s.st.dt_halvings;
    int rc = halved_interval(s, c, 1, 0, rounds);
    if (rc == BD_OK) rc = halved_interval(s, c, 1, 1, rounds);
    if (rc != BD_OK) {   // leave the rollback the step's start in xo, yo, tho
        copy_d(s, s.xo, s.xs, dn);
        copy_d(s, s.yo, s.ys, dn);
        copy_d(s, s.tho, s.ths, dn);
    }
    return rc;
}

// One step of Algorithm 1 launched kernel by kernel: the whole step is
// enqueued as a budgeted sequence (force, update, repair rounds, overlap
// rounds each with its repair) and the control block is read back once; if a
// budget ran out or a repair failed, the host finishes the step from exactly
// that point.
int one_step(Sim &s) {
    StepPlan plan;
    write_base(s);
    if (s.use_nl && s.need_rebuild) verlet_rebuild(s);
    fill_int(s, s.ctl, N_CTL, 0);
    if (s.adj.tape.on) {   // adjoint tape: positions before the step
        const Tape &tp = s.adj.tape;
        const size_t off = (size_t)tp.step_idx * s.n, bytes = sizeof(double) * s.n;
        check(hipMemcpyAsync(tp.px + off, s.x, bytes, hipMemcpyDeviceToDevice, s.stream), "tape x");
        check(hipMemcpyAsync(tp.py + off, s.y, bytes, hipMemcpyDeviceToDevice, s.stream), "tape y");
    }
    compute_forces(s);
    if (s.adj.tape.on && s.adj.tape.phi) {   // adjoint tape: the step's force partial sums
        const size_t bytes = (size_t)s.part_cap * (s.fp32 ? sizeof(float2) : sizeof(double2));
        check(hipMemcpyAsync((char *)s.adj.tape.phi + (size_t)s.adj.tape.step_idx * bytes, s.part, bytes,
                             hipMemcpyDeviceToDevice, s.stream),
              "tape phi");
    }
    launch_em(s);
    plan.b = s.budget;
    if (s.ovl_method == 1) {
        plan.overlaps = s.budget.overlaps;
        enqueue_rounds_nl(s, plan.c, plan.orounds);
    } else {
        plan.overlaps = overlaps_budget(s);
        enqueue_rounds(s, plan.c, plan.orounds, plan.rep_first);
    }
    read_ctl(s);
    return finish_step(s, s.hctl, plan);
}

// Graph mode: up to kRing steps are queued as graph replays; each records its
// control block and the first one that halts (or needs new neighbour lists)
// stops the rest.  The host then does the per-step bookkeeping in order,
// finishes a halted step exactly where it stopped, and queues the remainder.
int run_graph_steps(Sim &s, int64_t nsteps) {
    while (nsteps > 0) {
        if (s.use_nl && s.need_rebuild) verlet_rebuild(s);
        Sim::StepGraph &g = step_graph(s);
        // steps queued after one that stops still cost their launches: queue about as many
        // steps as recently ran between stops (neighbour-list rebuilds, budget growth)
        const int m = (int)std::min<int64_t>(nsteps, std::min(kRing, s.batch_hint));
        write_base(s);
        for (int k = 0; k < m; ++k) {
            check(hipGraphLaunch(g.pre, s.stream), "graph launch");
            timed(s, [&] { check(hipGraphLaunch(g.force, s.stream), "graph launch"); });
            check(hipGraphLaunch(g.post, s.stream), "graph launch");
        }
        StepBase hb;
        check(hipMemcpyAsync(&s.hbase->step, &s.dbase->step, sizeof(StepBase), hipMemcpyDeviceToHost, s.stream),
              "step base");
        check(hipStreamSynchronize(s.stream), "sync");
        hb = *s.hbase;
        const int done = hb.batch_idx;
        const int nrec = done + (hb.stop == 1 ? 1 : 0);
        // stops are rare (a halted step; list rebuilds happen inside the queued steps): after one,
        // queue as many steps as ran before it, then double back up to the ring size
        if (hb.stop == 1)
            s.batch_hint = std::max(4, nrec);
        else if (nrec == m)
            s.batch_hint = std::min(kRing, 2 * s.batch_hint);
        check(hipMemcpyAsync(s.hring, s.ring, sizeof(int) * N_CTL * nrec, hipMemcpyDeviceToHost, s.stream), "ring");
        check(hipStreamSynchronize(s.stream), "sync");
        StepPlan plan;
        plan.b = s.budget;
        plan.overlaps = s.ovl_method == 1 ? s.budget.overlaps : overlaps_budget(s);
        plan.c.slot = g.c_slot;
        plan.c.rep = g.c_rep;
        plan.c.oround = g.c_oround;
        plan.orounds = g.orounds;
        plan.rep_first = g.rep_first;
        const int r_used = g.r_used, v_used = g.v_used;   // g may move when budgets change below
        for (int j = 0; j < nrec; ++j) {
            // the device's stamp bases for this step, for any host-driven continuation
            s.rbase = s.round_id;
            s.vbase = s.vround;
            s.round_id += r_used;
            s.vround += v_used;
            const int *hj = s.hring + (size_t)j * N_CTL;
            int rc;
            if (hj[K_HALT] && hj[K_REASON] == HALT_NL_CAPACITY) {
                // the step stopped before its force: the lists grow (the captured steps go),
                // then the step runs again launch by launch
                verlet_rebuild(s);
                rc = one_step(s);
            } else {
                rc = finish_step(s, hj, plan);
            }
            if (rc != BD_OK) {
                write_base(s);
                return rc;
            }
        }
        nsteps -= nrec;
        write_base(s);   // clears the stop flag for later work on this handle
    }
    return BD_OK;
}

// Host side of a step whose budgeted part has run: bookkeeping, the
// continuation of a halted step, budget adaptation.  h_in is the step's
// control block as read back.
// finish_step for the list method: no repairs, only overlap rounds.
int finish_step_nl(Sim &s, const int *h_in, const StepPlan &plan);

int finish_step(Sim &s, const int *h_in, const StepPlan &plan) {
    if (s.ovl_method == 1) return finish_step_nl(s, h_in, plan);
    const std::vector<int> hv(h_in, h_in + N_CTL);
    const int *h = hv.data();
    const Cursor &c = plan.c;
    const std::vector<int> &orounds = plan.orounds;
    const std::vector<int> &rep_first = plan.rep_first;
    s.need_rebuild = s.use_nl && h[K_NL_REBUILD] != 0;
    if (h[K_NL_BUILT]) ++s.st.verlet_rebuilds;   // rebuilt on the device at the start of this step
    // bookkeeping of the budgeted part: overlap rounds that moved disks
    int rounds = h[K_OVL_ROUNDS];
    if (h[K_HALT]) {
        if (h[K_REASON] == HALT_OVERLAP_BUDGET) rounds = plan.overlaps;
        if (h[K_REASON] == HALT_REPAIR_BUDGET || h[K_REASON] == HALT_INVALID) rounds = h[K_STAGE];
    }
    for (int j = 0; j < rounds; ++j) s.st.overlap_edges_total += h[K_OVL + orounds[j]];
    for (int j = 0; j < c.slot; ++j) s.st.flip_rounds_total += h[K_CAND + j] > 0 ? 1 : 0;
    int rc = BD_OK;
    if (h[K_HALT] || h[K_TOPO]) {
        const int reason = h[K_TOPO] ? HALT_TOPOLOGY : h[K_REASON], stage = h[K_STAGE], last = h[K_LAST];
        if (reason == HALT_TOPOLOGY) {
            s.last_error = "triangulation index out of range";
            rollback(s);
            return BD_ERR_TRIANGULATION;
        }
        // continue host-driven after the halting point
        ++s.st.host_continued;
        fill_int(s, s.ctl + K_HALT, 1, 0);
        fill_int(s, s.ctl + K_DONE, 1, 0);
        Cursor hc;
        hc.slot = c.slot;
        hc.rep = c.rep;
        hc.oround = c.oround;
        if (reason == HALT_REVERSAL) {
            rc = redo_step_in_halves(s, hc, rounds);
            if (rc != BD_OK) {
                rollback(s);
                s.need_rebuild = true;
                return rc;
            }
            skin_check(s, true);
        } else if (reason == HALT_REPAIR_BUDGET || reason == HALT_INVALID) {
            // repair slot `stage`: 0 is the repair after the update, j >= 1 the one after overlap round j-1
            // a failure replays the step's whole move from the copy taken before its first repair
            if (reason == HALT_REPAIR_BUDGET) {
                hc.slot = next_slot(last);   // its worklist holds the edges still to evaluate
                if (!host_flip_rounds(s, hc, false, false, nullptr))
                    rc = kinetic_replay(s, hc, MoveFrom::Previous, 0);
            } else {
                rc = kinetic_replay(s, hc, MoveFrom::Previous, 0);
            }
        }
        if (reason != HALT_REVERSAL) {
            if (rc == BD_OK) rc = host_overlap_loop(s, hc, rounds);
            if (rc != BD_OK) {
                rollback(s);
                s.need_rebuild = true;
                return rc;
            }
            skin_check(s, true);   // positions moved after the budgeted sequence's test
        }
    }
    // adapt the budgets to the rounds this step needed: grow at once when a
    // budget ran out, shrink by one when it was larger than needed
    auto used_rounds = [&](int rep, int budget) {
        for (int j = 0; j < budget; ++j)
            if (h[K_CAND + rep_first[rep] + j] == 0) return j + 1;
        return budget + 2;
    };
    // grow at once when a budget ran out; shrink by one only after kShrinkAfter
    // steps in a row that needed less (a halted step costs far more than a few
    // extra no-op launches)
    constexpr int kShrinkAfter = 64;
    auto adapt = [&](int &budget, int used, int &slack, int most = 8) {
        if (used >= budget) {
            budget = std::min(most, used + 1);
            slack = 0;
        } else if (used + 1 < budget) {
            if (++slack >= kShrinkAfter) {
                budget = std::max(2, budget - 1);
                slack = 0;
            }
        } else {
            slack = 0;
        }
    };
    const int hreason = h[K_HALT] ? h[K_REASON] : 0;
    // repair slot that stopped the budgeted sequence (none for an overlap budget halt)
    const int halt_rep = (hreason == HALT_REPAIR_BUDGET || hreason == HALT_INVALID) ? h[K_STAGE] : 1 << 30;
    s.budget = plan.b;
    if (halt_rep > 0)
        adapt(s.budget.em, used_rounds(0, plan.b.em), s.slack_em);
    else if (hreason == HALT_REPAIR_BUDGET)
        adapt(s.budget.em, plan.b.em + 2, s.slack_em);
    // each overlap round's repair has its own budget: the later rounds move
    // fewer disks and need fewer flip rounds; one that did not run this step
    // counts as needing the least
    for (int j = 0; j < plan.overlaps; ++j) {
        const int r = j + 1;
        int used = 1;
        if (r == halt_rep && hreason == HALT_REPAIR_BUDGET)
            used = plan.b.ovl[j] + 2;
        else if (r < (int)rep_first.size() && r <= rounds && r < halt_rep)
            used = used_rounds(r, plan.b.ovl[j]);
        adapt(s.budget.ovl[j], used, s.slack_ovl[j]);
    }
    s.budget.overlaps = std::max(s.budget.overlaps, plan.overlaps);
    adapt(s.budget.overlaps, rounds, s.slack_over, MAXO / 2);   // contact-factor runs need ~20 rounds
    update_ovl_phase(s, h, plan.orounds, std::min(rounds, plan.overlaps));
    s.st.overlap_rounds_total += rounds;
    if (rounds > s.st.overlap_rounds_max) s.st.overlap_rounds_max = rounds;
    ++s.st.steps;
    ++s.step;
    return BD_OK;
}

int finish_step_nl(Sim &s, const int *h_in, const StepPlan &plan) {
    const std::vector<int> hv(h_in, h_in + N_CTL);
    const int *h = hv.data();
    s.need_rebuild = h[K_NL_REBUILD] != 0;
    if (h[K_NL_BUILT]) ++s.st.verlet_rebuilds;
    int rounds = h[K_OVL_ROUNDS];
    for (int j = 0; j < rounds; ++j) s.st.overlap_edges_total += h[K_OVL + plan.orounds[j]];
    update_nl_phase(s, h, plan.orounds, rounds);
    if (h[K_HALT]) {
        // overlaps left after the budgeted rounds, or lists that may miss a pair: the host continues
        ++s.st.host_continued;
        fill_int(s, s.ctl + K_HALT, 1, 0);
        fill_int(s, s.ctl + K_DONE, 1, 0);
        Cursor hc = plan.c;
        if (h[K_REASON] == HALT_NL_STALE) verlet_rebuild(s);
        int rc = host_overlap_loop_nl(s, hc, rounds);
        if (rc != BD_OK) {
            rollback(s);
            return rc;
        }
        skin_check(s, true);   // positions moved after the budgeted sequence's test
    }
    constexpr int kShrinkAfter = 64;
    int &budget = s.budget.overlaps;
    budget = plan.b.overlaps;
    if (rounds >= budget) {
        budget = std::min(MAXO / 2, rounds + 1);
        s.slack_over = 0;
    } else if (rounds + 1 < budget) {
        if (++s.slack_over >= kShrinkAfter) {
            budget = std::max(2, budget - 1);
            s.slack_over = 0;
        }
    } else {
        s.slack_over = 0;
    }
    s.st.overlap_rounds_total += rounds;
    if (rounds > s.st.overlap_rounds_max) s.st.overlap_rounds_max = rounds;
    ++s.st.steps;
    ++s.step;
    return BD_OK;
}

// ------------------------------------------------------------------ force tiling
// Chunks of one species range [js, je): nc = round(cnt / chunk) equal parts,
// lengths rounded up to a multiple of 8.  Depends only on the range and the
// chunk length, so a system is cut the same way alone or in a batch.
void cut_species(int js, int je, int chunk, std::vector<int2> &out, bool cap = false) {
    const int cnt = je - js;
    if (cnt <= 0) return;
    // cap: no part longer than chunk (a multiple of 8)
    int nc = cap ? (cnt + chunk - 1) / chunk : std::max(1, (int)std::llround((double)cnt / chunk));
    int len = (cnt + nc - 1) / nc;
    len = (len + 7) / 8 * 8;
    for (int j = js; j < je; j += len) out.push_back(make_int2(j, std::min(je, j + len)));
}

struct Tiling {
    std::vector<Tile> tiles;
    std::vector<SymTile> stiles;   // symmetric form only
    std::vector<int> chunk_spec;
    std::vector<RepInfo> reps;
    long long part_len = 0;
};

// sym: chunks of at most 256 per_lane and the symmetric form's tile list (every
// pair of chunks of a system once, then every chunk with itself); the
// ordinary tiles of the same chunks are kept for the adjoint sweep.
// Longest chunk of the symmetric form for a per_lane setting (2, 4: 4 wavefronts; 8: 2 wavefronts).
inline int sym_cap(int per_lane) { return per_lane == 8 ? 1024 : 256 * per_lane; }

Tiling make_tiling(const Sim &s, int chunk, int per_lane, bool sym = false) {
    Tiling t;
    t.reps.resize(s.R);
    const int ib_len = 256 * std::min(per_lane, 4);   // ordinary tiles (and the adjoint's) hold 2 or 4 per lane
    std::vector<int2> ch;
    for (int r = 0; r < s.R; ++r) {
        RepInfo &ri = t.reps[r];
        ri.off = s.off_h[r];
        ri.n = s.off_h[r + 1] - s.off_h[r];
        ri.cfirst = (int)t.chunk_spec.size();
        ri.poff = t.part_len;
        ri.L = s.L_h[r];
        ri.seed = s.seed_h[r];
        int nch = 0;
        std::vector<int2> all;   // this system's chunks in order
        for (int b = 0; b < s.S; ++b) {
            ch.clear();
            cut_species(s.bstart_h[r * (s.S + 1) + b], s.bstart_h[r * (s.S + 1) + b + 1],
                        sym ? sym_cap(per_lane) : chunk, ch, sym);
            for (const int2 &c : ch) {
                all.push_back(c);
                t.chunk_spec.push_back(b);
                for (int i0 = ri.off; i0 < ri.off + ri.n; i0 += ib_len) {
                    Tile tl;
                    tl.i0 = i0;
                    tl.i1 = std::min(ri.off + ri.n, i0 + ib_len);
                    tl.js = c.x;
                    tl.je = c.y;
                    tl.pbase = ri.poff + (long long)nch * ri.n - ri.off;
                    tl.work = (long long)(tl.i1 - tl.i0) * (tl.je - tl.js);
                    t.tiles.push_back(tl);
                }
                ++nch;
            }
        }
        ri.nch = nch;
        if (sym) {
            const long long base = ri.poff - ri.off;
            for (int a = 0; a < nch; ++a)
                for (int b = a; b < nch; ++b)
                    t.stiles.push_back(SymTile{all[a].x, all[a].y, all[b].x, all[b].y, base + (long long)b * ri.n,
                                               base + (long long)a * ri.n});
        }
        t.part_len += (long long)nch * ri.n;
    }
    std::stable_sort(t.tiles.begin(), t.tiles.end(), [](const Tile &a, const Tile &b) { return a.work > b.work; });
    std::stable_sort(t.stiles.begin(), t.stiles.end(), [](const SymTile &a, const SymTile &b) {
        return (long long)(a.i1 - a.i0) * (a.j1 - a.j0) > (long long)(b.i1 - b.i0) * (b.j1 - b.j0);
    });
    return t;
}

void upload_tiling(Sim &s, const Tiling &t, int chunk, int per_lane, int persistent) {
    // the force kernel writes part[pbase + i] for every tile: never launch a tiling the buffers cannot hold
    if ((long long)t.tiles.size() > s.tiles_cap || t.part_len > s.part_cap ||
        (long long)t.stiles.size() > s.stiles_cap || (persistent == 2) != !t.stiles.empty())
        throw DeviceError{hipErrorInvalidValue, "force tiling larger than its buffers"};
    for (const SymTile &st : t.stiles)   // the kernel holds at most sym_cap(per_lane) particles of each side
        if (st.i1 - st.i0 > sym_cap(per_lane) || st.j1 - st.j0 > sym_cap(per_lane) || st.i1 <= st.i0 ||
            st.j1 <= st.j0 || (per_lane != 2 && per_lane != 4 && per_lane != 8))
            throw DeviceError{hipErrorInvalidValue, "symmetric force tile out of shape"};
    if (!t.stiles.empty())
        check(hipMemcpyAsync(s.stiles, t.stiles.data(), sizeof(SymTile) * t.stiles.size(), hipMemcpyHostToDevice,
                             s.stream),
              "symmetric tiles");
    s.nstiles = (int)t.stiles.size();
    check(hipMemcpyAsync(s.tiles, t.tiles.data(), sizeof(Tile) * t.tiles.size(), hipMemcpyHostToDevice, s.stream),
          "tiles");
    check(hipMemcpyAsync(s.chunk_spec, t.chunk_spec.data(), sizeof(int) * t.chunk_spec.size(), hipMemcpyHostToDevice,
                         s.stream),
          "chunk_spec");
    check(hipMemcpyAsync(s.reps, t.reps.data(), sizeof(RepInfo) * s.R, hipMemcpyHostToDevice, s.stream), "reps");
    check(hipStreamSynchronize(s.stream), "tiling upload");
    s.ntiles = (int)t.tiles.size();
    s.chunk_len = chunk;
    s.per_lane = per_lane;
    s.persistent = persistent;
    s.force_grid = persistent == 2   ? s.nstiles
                   : persistent == 1 ? std::min(s.ntiles, force_max_grid(s, per_lane))
                                     : s.ntiles;
}

// Fixed rule: the smallest power-of-two chunk (>= 64) that keeps the launch
// at or below 2048 tiles.
int default_chunk(const Sim &s) {
    for (int c = 64;; c *= 2) {
        if (c >= 65536) return 65536;
        if ((long long)make_tiling(s, c, 4).tiles.size() <= 2048) return c;
    }
}

// ------------------------------------------------------------------ autotuner
// Candidate tilings (chunk length x i per lane x launch form) are timed on
// the handle's own positions; the fastest is kept.  Choices are cached per
// workload shape for the process, and in the JSON file named by the
// environment variable BD_TUNE_CACHE when it is set, so that handles of the
// same shape cut their sums the same way.
struct TuneChoice {
    int chunk, per_lane, persistent;
    double ms;
};
std::mutex g_tune_mu;
std::map<std::string, TuneChoice> g_tune;
bool g_tune_file_read = false;

std::string tune_key(const Sim &s) {
    unsigned long long h = 1469598103934665603ull;   // FNV-1a over the system shapes
    auto mix = [&](unsigned long long v) {
        for (int k = 0; k < 8; ++k) {
            h ^= (v >> (8 * k)) & 0xffu;
            h *= 1099511628211ull;
        }
    };
    for (int r = 0; r < s.R; ++r)
        for (int b = 0; b <= s.S; ++b) mix((unsigned long long)(s.bstart_h[r * (s.S + 1) + b] - s.off_h[r]));
    hipDeviceProp_t prop;
    std::string arch = hipGetDeviceProperties(&prop, s.device) == hipSuccess ? prop.gcnArchName : "unknown";
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s|%s|%s|S%d|R%d|n%d|%016llx", arch.c_str(), s.fp32 ? "fp32" : "fp64",
                  s.kind_fast ? "q2" : "general", s.S, s.R, s.n, h);
    return buf;
}

void read_tune_file() {
    g_tune_file_read = true;
    const char *path = std::getenv("BD_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof(line), f)) {
        char key[300];
        TuneChoice c;
        if (std::sscanf(line, " \"%299[^\"]\": [%d, %d, %d, %lf]", key, &c.chunk, &c.per_lane, &c.persistent, &c.ms) ==
            5)
            g_tune[key] = c;
    }
    std::fclose(f);
}

void write_tune_file() {
    const char *path = std::getenv("BD_TUNE_CACHE");
    if (!path || !*path) return;
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\n");
    size_t k = 0;
    for (const auto &e : g_tune)
        std::fprintf(f, "  \"%s\": [%d, %d, %d, %.6f]%s\n", e.first.c_str(), e.second.chunk, e.second.per_lane,
                     e.second.persistent, e.second.ms, ++k < g_tune.size() ? "," : "");
    std::fprintf(f, "}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

// Median time of the force launch plus the per-particle reduction of its
// partial sums (the update kernel's gather, which grows with the chunk count).
double time_force(Sim &s, int reps) {
    hipEvent_t a, b;
    check(hipEventCreate(&a), "event");
    check(hipEventCreate(&b), "event");
    launch_force(s);   // warm-up
    launch_reduce_forces(s);
    std::vector<float> t;
    for (int k = 0; k < reps; ++k) {
        check(hipEventRecord(a, s.stream), "event");
        launch_force(s);
        launch_reduce_forces(s);
        check(hipEventRecord(b, s.stream), "event");
        check(hipEventSynchronize(b), "event sync");
        float ms = 0.f;
        check(hipEventElapsedTime(&ms, a, b), "elapsed");
        t.push_back(ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

// Allocates tiles / part for the largest of the given tilings.
void alloc_force_buffers(Sim &s, long long max_tiles, long long max_part, long long max_stiles = 0) {
    const size_t vec = s.fp32 ? sizeof(float2) : sizeof(double2);
    dfree(s.tiles);
    dfree(s.part);
    dfree(s.stiles);
    s.tiles = nullptr;
    s.part = nullptr;
    s.stiles = nullptr;
    s.tiles = dalloc<Tile>((size_t)max_tiles);
    s.part = dalloc<char>(vec * (size_t)max_part);
    if (max_stiles > 0) s.stiles = dalloc<SymTile>((size_t)max_stiles);
    s.tiles_cap = max_tiles;
    s.part_cap = max_part;
    s.stiles_cap = max_stiles;
}

void setup_force(Sim &s) {
    const size_t vec = s.fp32 ? sizeof(float2) : sizeof(double2);
    s.reps = dalloc<RepInfo>(s.R);
    long long max_chunks = 0;
    for (int r = 0; r < s.R; ++r) max_chunks += (s.off_h[r + 1] - s.off_h[r]) / 8 + s.S;
    s.chunk_spec = dalloc<int>((size_t)max_chunks);
    if (s.use_nl) {   // short-range path: the all-pairs buffers stay minimal
        Tiling t = make_tiling(s, 65536, 4);
        alloc_force_buffers(s, (long long)t.tiles.size(), t.part_len);
        upload_tiling(s, t, 65536, 4, 0);
        return;
    }
    if (s.p.force_chunk > 0) {   // pinned: chunk length, particles per lane and launch form
        const int pl = s.p.force_per_lane == 2 ? 2 : 4;
        Tiling t = make_tiling(s, s.p.force_chunk, pl);
        alloc_force_buffers(s, (long long)t.tiles.size(), t.part_len);
        upload_tiling(s, t, s.p.force_chunk, pl, s.p.force_launch == 1 ? 1 : s.p.force_launch == 2 ? 3 : 0);
        return;
    }
    if (s.p.force_chunk < 0) {   // the symmetric form, pinned: -1 chunks of 1024 (4 per lane), -2 of 512, -3 1024 (8)
        const int pl = s.p.force_chunk == -1 ? 4 : s.p.force_chunk == -2 ? 2 : 8;
        Tiling t = make_tiling(s, sym_cap(pl), pl, true);
        alloc_force_buffers(s, (long long)t.tiles.size(), t.part_len, (long long)t.stiles.size());
        upload_tiling(s, t, sym_cap(pl), pl, 2);
        return;
    }
    long double pairs = 0;
    for (int r = 0; r < s.R; ++r) pairs += (long double)(s.off_h[r + 1] - s.off_h[r]) * (s.off_h[r + 1] - s.off_h[r]);
    const int dchunk = default_chunk(s);
    // a periodic box has its own (minimum-image) kernel in the one-workgroup-per-tile form: fixed rule
    if (pairs < (long double)(1 << 26) || s.period > 0.0) {
        Tiling t = make_tiling(s, dchunk, 4);
        alloc_force_buffers(s, (long long)t.tiles.size(), t.part_len);
        upload_tiling(s, t, dchunk, 4, 0);
        return;
    }
    const std::string key = tune_key(s);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (!g_tune_file_read) read_tune_file();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            const TuneChoice c = it->second;
            Tiling t = make_tiling(s, c.chunk, c.per_lane, c.persistent == 2);
            alloc_force_buffers(s, (long long)t.tiles.size(), t.part_len, (long long)t.stiles.size());
            upload_tiling(s, t, c.chunk, c.per_lane, c.persistent);
            s.tuned = 2;
            s.tuned_ms = c.ms;
            return;
        }
    }
    // candidates: chunk lengths around the fixed rule, both tile heights, both launch forms
    std::vector<int> chunks{dchunk};   // the fixed rule is always a candidate
    for (int c = std::max(256, dchunk / 8); c <= std::min(65536, dchunk * 4); c *= 2)
        if (c != dchunk) chunks.push_back(c);
    const long long part_limit = (2ll << 30) / (long long)vec;
    long long max_tiles = 0, max_part = 0;
    std::vector<std::pair<int, int>> cands;   // (chunk, per_lane)
    for (int c : chunks)
        for (int pl : {2, 4}) {
            Tiling t = make_tiling(s, c, pl);
            if (t.part_len > part_limit) continue;
            cands.emplace_back(c, pl);
            max_tiles = std::max(max_tiles, (long long)t.tiles.size());
            max_part = std::max(max_part, t.part_len);
        }
    if (cands.empty()) {
        Tiling t = make_tiling(s, dchunk, 4);
        alloc_force_buffers(s, (long long)t.tiles.size(), t.part_len);
        upload_tiling(s, t, dchunk, 4, 0);
        return;
    }
    // the symmetric form (inverse-square law): every pair of chunks once
    long long max_stiles = 0;
    std::vector<int> sym_pl;   // symmetric candidates: chunks of 512 (2 per lane) or 1024 (4 or 8 per lane)
    if (s.kind_fast)
        for (int pl : {2, 4, 8}) {
            Tiling t = make_tiling(s, sym_cap(pl), pl, true);
            if (t.part_len > part_limit) continue;
            sym_pl.push_back(pl);
            max_tiles = std::max(max_tiles, (long long)t.tiles.size());
            max_part = std::max(max_part, t.part_len);
            max_stiles = std::max(max_stiles, (long long)t.stiles.size());
        }
    alloc_force_buffers(s, max_tiles, max_part, max_stiles);
    launch_cast(s);
    // bring the clocks up before timing anything (with the first candidate, which the buffers hold)
    {
        Tiling t = make_tiling(s, cands[0].first, cands[0].second);
        upload_tiling(s, t, cands[0].first, cands[0].second, 0);
        hipEvent_t e0, e1;
        check(hipEventCreate(&e0), "event");
        check(hipEventCreate(&e1), "event");
        float ms = 0.f;
        for (int k = 0; k < 200 && ms < 50.f; ++k) {
            check(hipEventRecord(e0, s.stream), "event");
            for (int j = 0; j < 4; ++j) launch_force(s);
            check(hipEventRecord(e1, s.stream), "event");
            check(hipEventSynchronize(e1), "event sync");
            float dt = 0.f;
            check(hipEventElapsedTime(&dt, e0, e1), "elapsed");
            ms += dt;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    // first pass over every candidate, then the best few again
    std::vector<TuneChoice> scored;
    for (const auto &cp : cands) {
        Tiling t = make_tiling(s, cp.first, cp.second);
        for (int pers = 0; pers <= 1; ++pers) {
            upload_tiling(s, t, cp.first, cp.second, pers);
            scored.push_back(TuneChoice{cp.first, cp.second, pers, time_force(s, 5)});
        }
    }
    for (int pl : sym_pl) {
        upload_tiling(s, make_tiling(s, sym_cap(pl), pl, true), sym_cap(pl), pl, 2);
        scored.push_back(TuneChoice{sym_cap(pl), pl, 2, time_force(s, 5)});
    }
    std::sort(scored.begin(), scored.end(), [](const TuneChoice &x, const TuneChoice &y) { return x.ms < y.ms; });
    TuneChoice best{0, 0, 0, 1e30};
    for (size_t i = 0; i < scored.size() && i < 3; ++i) {
        const TuneChoice &c = scored[i];
        upload_tiling(s, make_tiling(s, c.chunk, c.per_lane, c.persistent == 2), c.chunk, c.per_lane, c.persistent);
        const double ms = time_force(s, 9);
        if (ms < best.ms) best = TuneChoice{c.chunk, c.per_lane, c.persistent, ms};
    }
    Tiling t = make_tiling(s, best.chunk, best.per_lane, best.persistent == 2);
    alloc_force_buffers(s, (long long)t.tiles.size(), t.part_len, (long long)t.stiles.size());
    upload_tiling(s, t, best.chunk, best.per_lane, best.persistent);
    s.tuned = 1;
    s.tuned_ms = best.ms;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best;
    write_tune_file();
}

void adj_free(Sim &s);

void free_all(Sim &s) {
    adj_free(s);
    void *ptrs[] = {s.x, s.y, s.xy, s.xo, s.yo, s.th, s.tho, s.rad, s.sp, s.sp_sorted, s.perm, s.key_id, s.sorted_id, s.pos_of, s.pj, s.part,
                    s.tiles, s.chunk_spec, s.reps, s.rep_of, s.Lr, s.Kd, s.fout, s.he_v, s.he_twin, s.vert_he,
                    s.claim, s.tri_stamp, s.moved, s.edge_stamp, s.vstamp, s.wl[0], s.wl[1], s.cand, s.cand_won,
                    s.touched, s.det_stamp, s.fl_stamp, s.fl, s.vt_stamp, s.vt, s.newpos, s.oldpos, s.snap_v, s.snap_twin,
                    s.snap_vh, s.xa, s.ya, s.xb, s.yb, s.ctl,
                    s.acc, s.nl, s.nl_cnt, s.nl_cand, s.cell_of, s.cell_count, s.cell_start, s.cell_fill, s.cell_items,
                    s.xbuild, s.ybuild, s.fsr, s.scan_bsum, s.stiles, s.xs, s.ys, s.ths};
    for (void *p : ptrs)
        dfree(p);
    drop_graphs(s);
    dfree(s.dbase);
    dfree(s.ring);
    if (s.hring) (void)hipHostFree(s.hring);
    if (s.hbase) (void)hipHostFree(s.hbase);
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

// Parameters shared by all systems of a handle (L is checked per system).
int validate_params(const bd_force_params *fp, const bd_params *p, std::string &err) {
    if (!fp || !p) return err = "NULL argument", BD_ERR_INVALID_ARG;
    if (fp->S < 1 || fp->S > BD_MAX_SPECIES || !fp->K) return err = "S out of range or K NULL", BD_ERR_INVALID_ARG;
    if (fp->kind != BD_FORCE_POWER && fp->kind != BD_FORCE_SCREENED)
        return err = "unknown force kind", BD_ERR_INVALID_ARG;
    for (int k = 0; k < fp->S * fp->S; ++k)
        if (!finite(fp->K[k])) return err = "K has a non-finite entry", BD_ERR_INVALID_ARG;
    if (!finite(fp->q) || !finite(fp->A) || !finite(fp->lambda) || !finite(fp->cutoff) || !finite(fp->skin))
        return err = "non-finite force parameter", BD_ERR_INVALID_ARG;
    if (fp->kind == BD_FORCE_SCREENED && !(fp->lambda > 0)) return err = "lambda must be > 0", BD_ERR_INVALID_ARG;
    if (fp->cutoff > 0 && !(fp->skin >= 0)) return err = "skin must be >= 0", BD_ERR_INVALID_ARG;
    const double vals[] = {p->D, p->dt, p->v0, p->Dr, p->overlap_factor, p->cap_frac, p->noise_clip, p->contact_tol};
    for (double v : vals)
        if (!finite(v)) return err = "non-finite step parameter", BD_ERR_INVALID_ARG;
    if (p->D < 0 || !(p->dt > 0) || p->Dr < 0 || !(p->overlap_factor > 0) || !(p->cap_frac > 0) ||
        !(p->noise_clip > 0) || p->contact_tol < 0 || p->contact_tol > 1e-3)
        return err = "step parameter out of range", BD_ERR_INVALID_ARG;
    if (p->force_precision != BD_PREC_FP32 && p->force_precision != BD_PREC_FP64)
        return err = "unknown force precision", BD_ERR_INVALID_ARG;
    if (p->force_chunk != 0 && (p->force_chunk < -3 || (p->force_chunk > 0 && p->force_chunk < 64) ||
                                p->force_chunk > 65536))
        return err = "force_chunk must be 0, -1, -2, -3 or in [64, 65536]", BD_ERR_INVALID_ARG;
    if (p->overlap_method != BD_OVERLAP_DELAUNAY && p->overlap_method != BD_OVERLAP_VERLET)
        return err = "unknown overlap method", BD_ERR_INVALID_ARG;
    if (p->overlap_method == BD_OVERLAP_VERLET && !(fp->cutoff > 0))
        return err = "the list overlap method needs short-range forces (cutoff > 0)", BD_ERR_INVALID_ARG;
    if (p->max_dt_halvings < 0 || p->max_dt_halvings > 12)
        return err = "max_dt_halvings must be in [0, 12]", BD_ERR_INVALID_ARG;
    if (p->max_dt_halvings > 0 && p->overlap_method != BD_OVERLAP_DELAUNAY)
        return err = "halving on edge reversal needs the Delaunay overlap method", BD_ERR_INVALID_ARG;
    if (p->force_per_lane != 0 && p->force_per_lane != 2 && p->force_per_lane != 4)
        return err = "force_per_lane must be 0, 2 or 4", BD_ERR_INVALID_ARG;
    if (p->force_launch < 0 || p->force_launch > 2) return err = "force_launch must be 0, 1 or 2", BD_ERR_INVALID_ARG;
    if (p->periodic != 0 && p->periodic != 1) return err = "periodic must be 0 or 1", BD_ERR_INVALID_ARG;
    if (p->periodic && !(fp->cutoff > 0) && (p->force_chunk < 0 || p->force_launch != 0))
        return err = "a periodic box evaluates all-pairs forces in the one-workgroup-per-tile form only "
                     "(force_chunk >= 0, force_launch 0)",
               BD_ERR_INVALID_ARG;
    if (p->force_launch == 2 && !(fp->kind == BD_FORCE_POWER && fp->q == 2.0 && !(fp->cutoff > 0)))
        return err = "force_launch 2 (j staged in LDS) needs the inverse-square law without cutoff",
               BD_ERR_INVALID_ARG;
    if (p->force_chunk < 0 && !(fp->kind == BD_FORCE_POWER && fp->q == 2.0 && !(fp->cutoff > 0)))
        return err = "force_chunk < 0 (symmetric form) needs the inverse-square law without cutoff",
               BD_ERR_INVALID_ARG;
    return BD_OK;
}

// One system: radii, species, positions inside [r, L - r], no overlap.
int validate_system(int n, const double *xy, const double *radii, const int32_t *species, const double *theta,
                    double L, int S, bool periodic, std::string &err) {
    if (n < 3) return err = "n must be at least 3", BD_ERR_INVALID_ARG;
    if (!finite(L) || !(L > 0)) return err = "box side must be finite and > 0", BD_ERR_INVALID_ARG;
    for (int i = 0; i < n; ++i) {
        double r = radii[i], x = xy[2 * i], y = xy[2 * i + 1];
        if (!finite(r) || !(r > 0) || !finite(x) || !finite(y))
            return err = "bad radius or position", BD_ERR_INVALID_ARG;
        if (species[i] < 0 || species[i] >= S) return err = "species out of range", BD_ERR_INVALID_ARG;
        if (theta && !finite(theta[i])) return err = "non-finite theta", BD_ERR_INVALID_ARG;
        if (periodic) {
            if (x < 0.0 || x >= L || y < 0.0 || y >= L) return err = "disk outside [0, L)^2", BD_ERR_BAD_INPUT;
        } else if (x < r || x > L - r || y < r || y > L - r) {
            return err = "disk outside the walls", BD_ERR_BAD_INPUT;
        }
    }
    // overlap check on a cell grid (cell side >= the largest contact distance)
    double rmax = 0;
    for (int i = 0; i < n; ++i) rmax = std::max(rmax, radii[i]);
    const double cell = 2 * rmax;
    long nc = std::max(1L, std::min(32768L, (long)std::floor(L / cell)));
    // periodic: separations by the nearest image; neighbouring cells wrap (with fewer than 3 cells a
    // row, every cell is a neighbour of every other: one cell holds all)
    if (periodic && nc < 3) nc = 1;
    const double inv = nc / L;
    std::vector<int> head((size_t)nc * nc, -1), nxt(n, -1);
    auto cidx = [&](double v) { long c = (long)(v * inv); return c < 0 ? 0 : (c >= nc ? nc - 1 : c); };
    const long span = nc == 1 ? 0 : 1;
    for (int i = 0; i < n; ++i) {
        long cx = cidx(xy[2 * i]), cy = cidx(xy[2 * i + 1]);
        for (long oy = -span; oy <= span; ++oy)
            for (long ox = -span; ox <= span; ++ox) {
                long gy = cy + oy, gx = cx + ox;
                if (periodic) {
                    gy = (gy + nc) % nc;
                    gx = (gx + nc) % nc;
                } else if (gy < 0 || gy >= nc || gx < 0 || gx >= nc) {
                    continue;
                }
                for (int j = head[gy * nc + gx]; j >= 0; j = nxt[j]) {
                    double dx = xy[2 * i] - xy[2 * j], dy = xy[2 * i + 1] - xy[2 * j + 1];
                    if (periodic) {
                        dx = bd_min_image(dx, L);
                        dy = bd_min_image(dy, L);
                    }
                    if (std::sqrt(dx * dx + dy * dy) < radii[i] + radii[j])
                        return err = "initial disks overlap", BD_ERR_BAD_INPUT;
                }
            }
        nxt[i] = head[cy * nc + cx];
        head[cy * nc + cx] = i;
    }
    return BD_OK;
}

int validate_batch(int R, const int32_t *n_per, const double *xy, const double *radii, const int32_t *species,
                   const double *theta, const double *L_per, const bd_force_params *fp, const bd_params *p,
                   std::string &err) {
    if (R < 1 || !n_per || !xy || !radii || !species || !L_per)
        return err = "NULL argument or R < 1", BD_ERR_INVALID_ARG;
    int rc = validate_params(fp, p, err);
    if (rc != BD_OK) return rc;
    if (R > 1 && fp->cutoff > 0) return err = "short-range forces need one system per handle", BD_ERR_INVALID_ARG;
    if (R > 1 && p->periodic) return err = "a periodic box needs one system per handle", BD_ERR_INVALID_ARG;
    long long total = 0;
    for (int r = 0; r < R; ++r) {
        if (n_per[r] < 3) return err = "every system needs at least 3 disks", BD_ERR_INVALID_ARG;
        total += n_per[r];
    }
    if (total > (1ll << 28)) return err = "too many disks in one handle", BD_ERR_INVALID_ARG;
    long long off = 0;
    for (int r = 0; r < R; ++r) {
        rc = validate_system(n_per[r], xy + 2 * off, radii + off, species + off, theta ? theta + off : nullptr,
                             L_per[r], fp->S, p->periodic != 0, err);
        if (rc != BD_OK) {
            if (R > 1) err = "system " + std::to_string(r) + ": " + err;
            return rc;
        }
        off += n_per[r];
    }
    return BD_OK;
}

int init_impl(Sim &s, int R, const int32_t *n_per, const double *xy, const double *radii, const int32_t *species,
              const double *theta, const double *L_per, const uint64_t *seed_per, const bd_force_params *fp,
              const bd_params *p) {
    s.R = R;
    s.off_h.assign(R + 1, 0);
    for (int r = 0; r < R; ++r) s.off_h[r + 1] = s.off_h[r] + n_per[r];
    const int n = s.off_h[R];
    s.L_h.assign(L_per, L_per + R);
    s.seed_h.assign(seed_per, seed_per + R);
    // Library order: inside each system the disks sorted along the Hilbert
    // curve over [0, L]^2 on a 2^16 grid (ties in caller order).  Every
    // gather of an edge's or a neighbour's endpoints then stays in a few cache
    // lines; the caller's order returns at every entry point that takes or
    // gives per-disk data, and the noise stays keyed by the caller's index.
    s.perm_h.resize(n);
    std::vector<int> key_h(n);
    for (int r = 0; r < R; ++r) {
        const int o = s.off_h[r], nr = n_per[r];
        const double scale = 65535.0 / L_per[r];
        std::vector<uint64_t> key(nr);
        for (int i = 0; i < nr; ++i) {
            const double cx = std::min(std::max(xy[2 * (size_t)(o + i)] * scale, 0.0), 65535.0);
            const double cy = std::min(std::max(xy[2 * (size_t)(o + i) + 1] * scale, 0.0), 65535.0);
            key[i] = hilbert_index((uint32_t)cx, (uint32_t)cy, 16);
        }
        int *pr = s.perm_h.data() + o;
        std::iota(pr, pr + nr, 0);
        std::stable_sort(pr, pr + nr, [&](int a, int b) { return key[a] < key[b]; });
        for (int k = 0; k < nr; ++k) {
            key_h[o + k] = pr[k];
            pr[k] += o;
        }
    }
    std::vector<double> xy_l(2 * (size_t)n), rad_l(n), th_l(theta ? n : 0);
    std::vector<int32_t> sp_l(n);
    for (int k = 0; k < n; ++k) {
        const int i = s.perm_h[k];
        xy_l[2 * (size_t)k] = xy[2 * (size_t)i];
        xy_l[2 * (size_t)k + 1] = xy[2 * (size_t)i + 1];
        rad_l[k] = radii[i];
        sp_l[k] = species[i];
        if (theta) th_l[k] = theta[i];
    }
    xy = xy_l.data();
    radii = rad_l.data();
    species = sp_l.data();
    if (theta) theta = th_l.data();
    // frame points of every system
    std::vector<std::vector<double>> fxs(R), fys(R);
    s.foff_h.assign(R + 1, 0);
    for (int r = 0; r < R; ++r) {
        double rmax = 0.0;
        for (int i = s.off_h[r]; i < s.off_h[r + 1]; ++i) rmax = std::max(rmax, radii[i]);
        if (!p->periodic) frame_points(L_per[r], rmax, fxs[r], fys[r]);   // a periodic box has no walls
        s.foff_h[r + 1] = s.foff_h[r] + (int)fxs[r].size();
    }
    s.n = n;
    s.m = s.foff_h[R];
    s.nv = n + s.m;
    s.S = fp->S;
    s.toff_h.assign(R + 1, 0);
    // planar: 2 (disks + frame) - 2 triangles with the infinite vertex; torus (periodic box): 2 n exactly
    for (int r = 0; r < R; ++r)
        s.toff_h[r + 1] = s.toff_h[r] + (p->periodic ? 2 * (s.off_h[r + 1] - s.off_h[r])
                                                     : 2 * (s.off_h[r + 1] - s.off_h[r] + s.foff_h[r + 1] -
                                                            s.foff_h[r]) - 2);
    s.T = s.toff_h[R];
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
    s.ovl_method = p->overlap_method;
    s.period = p->periodic ? L_per[0] : 0.0;
    check(hipGetDevice(&s.device), "hipGetDevice");
    check(hipStreamCreateWithFlags(&s.own_stream, hipStreamNonBlocking), "stream");
    s.stream = s.own_stream;

    // finite vertices: the disks, then the frames, then one padding entry per infinite vertex
    const int nv = s.nv, nva = nv + R;
    std::vector<double> hx(nva, 0.0), hy(nva, 0.0), hth(n, 0.0), hrad(nva, 0.0);
    std::vector<int> hrep(n);
    for (int i = 0; i < n; ++i) {
        hx[i] = xy[2 * i];
        hy[i] = xy[2 * i + 1];
        hrad[i] = radii[i];
        if (theta) hth[i] = theta[i];
    }
    s.rad_uni = n > 0 ? radii[0] : 0.0;
    for (int i = 1; i < n && s.rad_uni > 0.0; ++i)
        if (radii[i] != radii[0]) s.rad_uni = 0.0;
    for (int r = 0; r < R; ++r) {
        for (int i = s.off_h[r]; i < s.off_h[r + 1]; ++i) hrep[i] = r;
        for (int k = 0; k < (int)fxs[r].size(); ++k) {
            hx[n + s.foff_h[r] + k] = fxs[r][k];
            hy[n + s.foff_h[r] + k] = fys[r][k];
        }
    }
    // species-sorted permutation inside each system (stable: ids ascending inside a species)
    std::vector<int> sorted(n), pos(n);
    s.bstart_h.assign((size_t)R * (s.S + 1), 0);
    for (int r = 0; r < R; ++r) {
        int *bs = &s.bstart_h[(size_t)r * (s.S + 1)];
        std::vector<int> cnt(s.S + 1, 0);
        for (int i = s.off_h[r]; i < s.off_h[r + 1]; ++i) ++cnt[species[i] + 1];
        bs[0] = s.off_h[r];
        for (int b = 0; b < s.S; ++b) bs[b + 1] = bs[b] + cnt[b + 1];
        std::vector<int> fillp(bs, bs + s.S);
        for (int i = s.off_h[r]; i < s.off_h[r + 1]; ++i) {
            int k = fillp[species[i]]++;
            sorted[k] = i;
            pos[i] = k;
        }
    }

    s.x = dalloc<double>(nva);
    s.y = dalloc<double>(nva);
    s.xy = dalloc<double2>(nva);
    s.xo = dalloc<double>(nva);
    s.yo = dalloc<double>(nva);
    s.th = dalloc<double>(n);
    s.tho = dalloc<double>(n);
    s.rad = dalloc<double>(nva);
    s.sp = dalloc<int>(n);
    s.sp_sorted = dalloc<int>(n);
    s.perm = dalloc<int>(n);
    s.key_id = dalloc<int>(n);
    s.rep_of = dalloc<int>(n);
    s.Lr = dalloc<double>(R);
    s.sorted_id = dalloc<int>(n);
    s.pos_of = dalloc<int>(n);
    const size_t vec = s.fp32 ? sizeof(float2) : sizeof(double2);
    s.pj = dalloc<char>(vec * n);
    s.Kd = dalloc<double>(s.S * s.S);
    s.fout = dalloc<double>(2 * (size_t)n);
    s.he_v = dalloc<int>(s.H);
    s.he_twin = dalloc<int>(s.H);
    s.vert_he = dalloc<int>(nva);
    s.claim = dalloc<unsigned long long>(s.T);
    s.tri_stamp = dalloc<int>(s.T);
    s.moved = dalloc<int>(s.H);
    s.edge_stamp = dalloc<int>(s.H);
    s.vstamp = dalloc<int>(n + 1);
    s.wl[0] = dalloc<int>(s.H);
    s.wl[1] = dalloc<int>(s.H);
    s.cand = dalloc<int2>(s.H / 2 + 64);
    s.cand_won = dalloc<int>(s.H / 2 + 64);
    s.touched = dalloc<int>(2 * (size_t)n);
    s.det_stamp = dalloc<int>(s.H);
    s.fl_stamp = dalloc<int>(s.H);
    s.fl = dalloc<int>(s.H / 2 + 64);
    s.vt_stamp = dalloc<int>(s.T);
    s.vt = dalloc<int>(s.T + 64);
    s.newpos = dalloc<double2>(n);
    s.oldpos = dalloc<double2>(n);
    s.snap_v = dalloc<int>(s.H);
    s.snap_twin = dalloc<int>(s.H);
    s.snap_vh = dalloc<int>(nva);
    s.xa = dalloc<double>(n);
    s.ya = dalloc<double>(n);
    s.xb = dalloc<double>(n);
    s.yb = dalloc<double>(n);
    s.ctl = dalloc<int>(N_CTL);
    s.dbase = dalloc<StepBase>(1);
    s.ring = dalloc<int>((size_t)kRing * N_CTL);
    if (hipHostMalloc((void **)&s.hring, sizeof(int) * kRing * N_CTL, hipHostMallocDefault) != hipSuccess)
        throw std::bad_alloc();
    if (hipHostMalloc((void **)&s.hbase, sizeof(StepBase), hipHostMallocDefault) != hipSuccess) throw std::bad_alloc();
    if (s.use_nl) {
        const double rl = fp->cutoff + fp->skin;
        s.nl_nc = std::max(1, std::min(46000, (int)std::floor(L_per[0] / rl)));
        if (s.period > 0.0 && s.nl_nc < 3) {
            s.last_error = "a periodic box needs a side of at least 3 (cutoff + skin) for its cell grid";
            return BD_ERR_INVALID_ARG;
        }
        s.nl_ncell = s.nl_nc * s.nl_nc;
        s.cell_count = dalloc<int>(s.nl_ncell + 1);
        s.cell_start = dalloc<int>(s.nl_ncell + 1);
        s.cell_fill = dalloc<int>(s.nl_ncell);
        s.cell_of = dalloc<int>(n);
        s.cell_items = dalloc<int>(n);
        s.nl = dalloc<int>((size_t)s.nl_cap * n);
        s.nl_cnt = dalloc<int>(n);
        s.nl_cand = dalloc<int>(n);
        s.xbuild = dalloc<double>(n);
        s.ybuild = dalloc<double>(n);
        s.fsr = dalloc<double2>(n);
        s.scan_bsum = dalloc<int>(verlet_scan_blocks(s.nl_ncell));
    }
    s.acc = dalloc<unsigned long long>(N_ACC);
    if (hipHostMalloc((void **)&s.hctl, sizeof(int) * N_CTL, hipHostMallocDefault) != hipSuccess)
        throw std::bad_alloc();
    if (hipHostMalloc((void **)&s.hacc, sizeof(unsigned long long) * N_ACC, hipHostMallocDefault) != hipSuccess)
        throw std::bad_alloc();

    check(hipMemcpyAsync(s.x, hx.data(), sizeof(double) * nva, hipMemcpyHostToDevice, s.stream), "x");
    check(hipMemcpyAsync(s.y, hy.data(), sizeof(double) * nva, hipMemcpyHostToDevice, s.stream), "y");
    launch_pack_xy(s, nva);
    check(hipMemcpyAsync(s.xo, hx.data(), sizeof(double) * nva, hipMemcpyHostToDevice, s.stream), "xo");
    check(hipMemcpyAsync(s.yo, hy.data(), sizeof(double) * nva, hipMemcpyHostToDevice, s.stream), "yo");
    check(hipMemcpyAsync(s.th, hth.data(), sizeof(double) * n, hipMemcpyHostToDevice, s.stream), "th");
    check(hipMemcpyAsync(s.tho, hth.data(), sizeof(double) * n, hipMemcpyHostToDevice, s.stream), "tho");
    check(hipMemcpyAsync(s.rad, hrad.data(), sizeof(double) * nva, hipMemcpyHostToDevice, s.stream), "rad");
    check(hipMemcpyAsync(s.sp, species, sizeof(int) * n, hipMemcpyHostToDevice, s.stream), "sp");
    std::vector<int> sps(n);
    for (int k = 0; k < n; ++k) sps[k] = species[sorted[k]];
    check(hipMemcpyAsync(s.sp_sorted, sps.data(), sizeof(int) * n, hipMemcpyHostToDevice, s.stream), "sp_sorted");
    check(hipMemcpyAsync(s.perm, s.perm_h.data(), sizeof(int) * n, hipMemcpyHostToDevice, s.stream), "perm");
    check(hipMemcpyAsync(s.key_id, key_h.data(), sizeof(int) * n, hipMemcpyHostToDevice, s.stream), "key_id");
    check(hipMemcpyAsync(s.rep_of, hrep.data(), sizeof(int) * n, hipMemcpyHostToDevice, s.stream), "rep_of");
    check(hipMemcpyAsync(s.Lr, L_per, sizeof(double) * R, hipMemcpyHostToDevice, s.stream), "Lr");
    check(hipMemcpyAsync(s.sorted_id, sorted.data(), sizeof(int) * n, hipMemcpyHostToDevice, s.stream), "sorted");
    check(hipMemcpyAsync(s.pos_of, pos.data(), sizeof(int) * n, hipMemcpyHostToDevice, s.stream), "pos");
    check(hipMemcpyAsync(s.Kd, s.K.data(), sizeof(double) * s.S * s.S, hipMemcpyHostToDevice, s.stream), "K");
    check(hipMemsetAsync(s.claim, 0, sizeof(unsigned long long) * s.T, s.stream), "claim");
    check(hipMemsetAsync(s.tri_stamp, 0, sizeof(int) * s.T, s.stream), "tri_stamp");
    check(hipMemsetAsync(s.edge_stamp, 0, sizeof(int) * s.H, s.stream), "edge_stamp");
    check(hipMemsetAsync(s.det_stamp, 0, sizeof(int) * s.H, s.stream), "det_stamp");
    check(hipMemsetAsync(s.fl_stamp, 0xFF, sizeof(int) * s.H, s.stream), "fl_stamp");
    check(hipMemsetAsync(s.vt_stamp, 0xFF, sizeof(int) * s.T, s.stream), "vt_stamp");
    check(hipMemsetAsync(s.vstamp, 0, sizeof(int) * (n + 1), s.stream), "vstamp");
    check(hipMemsetAsync(s.acc, 0, sizeof(unsigned long long) * N_ACC, s.stream), "acc");
    check(hipMemsetAsync(s.ctl, 0, sizeof(int) * N_CTL, s.stream), "ctl");
    check(hipStreamSynchronize(s.stream), "init upload");
    write_base(s);

    setup_force(s);

    if (s.ovl_method == 0) {   // the list method keeps no triangulation
        std::vector<int> hv, ht;
        if (host_dt_all(s, hx.data(), hy.data(), hv, ht) != 0) {
            s.last_error = "initial Delaunay triangulation failed (coincident positions)";
            return BD_ERR_TRIANGULATION;
        }
        upload_topology(s, hv, ht);
    } else {
        double rmax = 0.0;
        for (int i = 0; i < n; ++i) rmax = std::max(rmax, radii[i]);
        s.nl_margin = 0.5 * (fp->cutoff + fp->skin - 2.0 * rmax);
        if (!(s.nl_margin > 0.0)) {
            s.last_error = "the list overlap method needs cutoff + skin larger than the largest contact distance";
            return BD_ERR_INVALID_ARG;
        }
    }
    if (s.use_nl) verlet_rebuild(s);
    return BD_OK;
}

// ------------------------------------------------------------------ adjoint
void ck_alloc(Sim &s, Checkpoint &c) {
    c.x = dalloc<double>(s.n);
    c.y = dalloc<double>(s.n);
    c.xo = dalloc<double>(s.n);
    c.yo = dalloc<double>(s.n);
    c.th = dalloc<double>(s.n);
    c.tho = dalloc<double>(s.n);
    c.he_v = dalloc<int>(s.H);
    c.he_twin = dalloc<int>(s.H);
    c.vert_he = dalloc<int>(s.nv + s.R);
}

void ck_free(Checkpoint &c) {
    void *ptrs[] = {c.x, c.y, c.xo, c.yo, c.th, c.tho, c.he_v, c.he_twin, c.vert_he};
    for (void *p : ptrs)
        dfree(p);
    c = Checkpoint();
}

void d2d(Sim &s, void *dst, const void *src, size_t bytes) {
    check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s.stream), "checkpoint copy");
}

void ck_save(Sim &s, Checkpoint &c) {
    const size_t dn = sizeof(double) * s.n;
    d2d(s, c.x, s.x, dn);
    d2d(s, c.y, s.y, dn);
    d2d(s, c.xo, s.xo, dn);
    d2d(s, c.yo, s.yo, dn);
    d2d(s, c.th, s.th, dn);
    d2d(s, c.tho, s.tho, dn);
    d2d(s, c.he_v, s.he_v, sizeof(int) * s.H);
    d2d(s, c.he_twin, s.he_twin, sizeof(int) * s.H);
    d2d(s, c.vert_he, s.vert_he, sizeof(int) * (s.nv + s.R));
    check(hipMemcpyAsync(c.acc, s.acc, sizeof(unsigned long long) * N_ACC, hipMemcpyDeviceToHost, s.stream), "acc");
    check(hipStreamSynchronize(s.stream), "checkpoint");
    c.step = s.step;
    c.st = s.st;
    c.budgets = s.budget;
}

void ck_restore(Sim &s, const Checkpoint &c) {
    const size_t dn = sizeof(double) * s.n;
    d2d(s, s.x, c.x, dn);
    d2d(s, s.y, c.y, dn);
    launch_pack_xy(s, s.n);
    d2d(s, s.xo, c.xo, dn);
    d2d(s, s.yo, c.yo, dn);
    d2d(s, s.th, c.th, dn);
    d2d(s, s.tho, c.tho, dn);
    d2d(s, s.he_v, c.he_v, sizeof(int) * s.H);
    d2d(s, s.he_twin, c.he_twin, sizeof(int) * s.H);
    d2d(s, s.vert_he, c.vert_he, sizeof(int) * (s.nv + s.R));
    check(hipMemcpyAsync(s.acc, c.acc, sizeof(unsigned long long) * N_ACC, hipMemcpyHostToDevice, s.stream), "acc");
    fill_int(s, s.ctl, N_CTL, 0);
    check(hipStreamSynchronize(s.stream), "restore");
    s.step = c.step;
    s.st = c.st;
    s.budget = c.budgets;
}

void tape_free(Tape &tp) {
    void *ptrs[] = {tp.px, tp.py, tp.emwf, tp.ev, tp.eold, tp.edisp, tp.ewf, tp.ecnt, tp.enb, tp.dir, tp.phi};
    for (void *p : ptrs)
        dfree(p);
    tp = Tape();
}

void tape_alloc_rounds(Tape &tp, int cap_ent, int cap_dir) {
    void *ptrs[] = {tp.ev, tp.eold, tp.edisp, tp.ewf, tp.ecnt, tp.enb, tp.dir};
    for (void *p : ptrs)
        dfree(p);
    tp.cap_ent = cap_ent;
    tp.cap_dir = cap_dir;
    tp.ev = dalloc<int>(cap_ent);
    tp.eold = dalloc<double2>(cap_ent);
    tp.edisp = dalloc<double2>(cap_ent);
    tp.ewf = dalloc<signed char>(2 * (size_t)cap_ent);
    tp.ecnt = dalloc<int>(cap_ent);
    tp.enb = dalloc<int>((size_t)cap_ent * MAXACT);
    tp.dir = dalloc<int2>(cap_dir);
}

void adj_free(Sim &s) {
    AdjState &a = s.adj;
    for (auto &c : a.ck) ck_free(c);
    tape_free(a.tape);
    void *ptrs[] = {a.lam, a.nu, a.bx, a.by, a.pj4, a.gpart, a.dk_rows, a.dk_blk, a.dk};
    for (void *p : ptrs)
        dfree(p);
    a = AdjState();
}

int adjoint_begin(Sim &s, int64_t nsteps, int every) {
    if (!s.kind_fast || s.use_nl) {
        s.last_error = "the adjoint covers the all-pairs inverse-square force only";
        return BD_ERR_INVALID_ARG;
    }
    if (s.p.max_dt_halvings > 0) {
        s.last_error = "the adjoint does not cover steps halved after an edge reversal";
        return BD_ERR_INVALID_ARG;
    }
    if (s.period > 0.0) {
        s.last_error = "the adjoint covers the box with walls only";
        return BD_ERR_INVALID_ARG;
    }
    adj_free(s);
    AdjState &a = s.adj;
    a.t0 = s.step;
    a.nsteps = nsteps;
    a.every = every;
    const int nseg = (int)((nsteps + every - 1) / every);
    a.ck.resize(nseg + 1);
    for (auto &c : a.ck) ck_alloc(s, c);
    for (int64_t t = 0; t < nsteps; ++t) {
        if (t % every == 0) ck_save(s, a.ck[t / every]);
        int rc = one_step(s);
        if (rc != BD_OK) {
            adj_free(s);
            return rc;
        }
    }
    ck_save(s, a.ck[nseg]);
    const int n = s.n;
    a.lam = dalloc<double2>(n);
    a.nu = dalloc<double2>(n);
    a.bx = dalloc<double>(n);
    a.by = dalloc<double>(n);
    a.pj4 = dalloc<double4>(n);
    a.gpart = dalloc<double2>((size_t)s.part_cap);
    a.dk_blocks = (n + 255) / 256;
    a.dk_rows = dalloc<double>((size_t)n * s.S);
    a.dk_blk = dalloc<double>((size_t)a.dk_blocks * s.S * s.S);
    a.dk = dalloc<double>(s.S * s.S);
    Tape &tp = a.tape;
    tp.cap_steps = every;
    tp.px = dalloc<double>((size_t)every * n);
    tp.py = dalloc<double>((size_t)every * n);
    tp.emwf = dalloc<signed char>((size_t)every * 2 * n);
    tape_alloc_rounds(tp, std::max(4096, 2 * n), std::max(256, 64 * every));
    // keep each step's force partial sums when they fit in 8 GiB (else the sweep recomputes them)
    const size_t phi_bytes = (size_t)every * s.part_cap * (s.fp32 ? sizeof(float2) : sizeof(double2));
    if (phi_bytes <= (8ull << 30)) {
        try {
            tp.phi = raw_alloc(phi_bytes);
        } catch (const std::bad_alloc &) {
            tp.phi = nullptr;
        }
    }
    a.ready = true;
    return BD_OK;
}

// Replays segment `seg` from its checkpoint with the tape on.  Returns BD_OK,
// or an error (state left at the segment's end).
int record_segment(Sim &s, int seg, int len) {
    AdjState &a = s.adj;
    Tape &tp = a.tape;
    for (int attempt = 0; attempt < 3; ++attempt) {
        ck_restore(s, a.ck[seg]);
        tp.on = true;
        tp.ent_base = 0;
        tp.dir_base = 0;
        tp.step_dir_end.assign(len, 0);
        bool grow = false;
        for (int t = 0; t < len; ++t) {
            tp.step_idx = t;
            int rc = one_step(s);
            if (rc != BD_OK) {
                tp.on = false;
                return rc;
            }
            read_ctl(s);
            const int *h = s.hctl;
            if (h[K_TAPE_OVF] & 2) {
                tp.on = false;
                s.last_error = "a disk overlapped more partners in one round than the adjoint tape records";
                return BD_ERR_INVALID_ARG;
            }
            if (h[K_TAPE_OVF]) grow = true;
            tp.ent_base += h[K_TAPE_ENT];
            tp.dir_base += h[K_TAPE_DIR];
            tp.step_dir_end[t] = tp.dir_base;
        }
        tp.on = false;
        if (!grow) return BD_OK;
        tape_alloc_rounds(tp, std::max(tp.cap_ent, 2 * tp.ent_base), std::max(tp.cap_dir, 2 * tp.dir_base));
    }
    s.last_error = "adjoint tape could not be sized";
    return BD_ERR_DEVICE;
}

int adjoint_backward(Sim &s, const double *gT, double *g0, double *gK, bool dev = false) {
    AdjState &a = s.adj;
    if (!a.ready) {
        s.last_error = "bd_adjoint_begin has not been run";
        return BD_ERR_INVALID_ARG;
    }
    Tape &tp = a.tape;
    const int nseg = (int)a.ck.size() - 1;
    const int nb = (s.n + 255) / 256;
    std::vector<double> hl;
    if (dev) {
        hipLaunchKernelGGL(k_gather2, dim3(nb), dim3(256), 0, s.stream, s.n, (const int *)s.perm, (const double2 *)gT,
                           a.lam);
    } else {
        hl.resize(2 * (size_t)s.n);
        for (int k = 0; k < s.n; ++k) {
            hl[2 * (size_t)k] = gT[2 * (size_t)s.perm_h[k]];
            hl[2 * (size_t)k + 1] = gT[2 * (size_t)s.perm_h[k] + 1];
        }
        check(hipMemcpyAsync(a.lam, hl.data(), sizeof(double2) * s.n, hipMemcpyHostToDevice, s.stream), "lambda");
    }
    check(hipMemsetAsync(a.dk_blk, 0, sizeof(double) * a.dk_blocks * s.S * s.S, s.stream), "dk");
    int rc = BD_OK;
    std::vector<int2> dir;
    for (int seg = nseg - 1; seg >= 0 && rc == BD_OK; --seg) {
        const int len = (int)std::min<int64_t>(a.every, a.nsteps - (int64_t)seg * a.every);
        rc = record_segment(s, seg, len);
        if (rc != BD_OK) break;
        dir.resize(tp.dir_base);
        if (tp.dir_base > 0)
            check(hipMemcpyAsync(dir.data(), tp.dir, sizeof(int2) * tp.dir_base, hipMemcpyDeviceToHost, s.stream),
                  "tape directory");
        check(hipStreamSynchronize(s.stream), "sync");
        for (int t = len - 1; t >= 0; --t) {
            const int r0 = t == 0 ? 0 : tp.step_dir_end[t - 1], r1 = tp.step_dir_end[t];
            for (int r = r1 - 1; r >= r0; --r) launch_adj_round(s, dir[r].x, dir[r].y);
            launch_adj_step(s, t);
        }
    }
    if (rc == BD_OK) {
        launch_adj_dk_final(s);
        const hipMemcpyKind out = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        if (g0 && dev)
            hipLaunchKernelGGL(k_scatter2, dim3(nb), dim3(256), 0, s.stream, s.n, (const int *)s.perm,
                               (const double2 *)a.lam, (double2 *)g0);
        if (g0 && !dev) {
            hl.resize(2 * (size_t)s.n);
            check(hipMemcpyAsync(hl.data(), a.lam, sizeof(double2) * s.n, out, s.stream), "grad x0");
        }
        if (gK) check(hipMemcpyAsync(gK, a.dk, sizeof(double) * s.S * s.S, out, s.stream), "grad K");
        check(hipStreamSynchronize(s.stream), "sync");
        if (g0 && !dev)
            for (int k = 0; k < s.n; ++k) {
                g0[2 * (size_t)s.perm_h[k]] = hl[2 * (size_t)k];
                g0[2 * (size_t)s.perm_h[k] + 1] = hl[2 * (size_t)k + 1];
            }
    }
    ck_restore(s, a.ck[nseg]);   // back to the end of the forward pass
    return rc;
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
    UseSim use(s);
    try {
        return f();
    } catch (const DeviceError &e) {
        s.last_error = std::string(e.what) + ": " + hipGetErrorString(e.e);
        return BD_ERR_DEVICE;
    } catch (const UnsupportedError &e) {
        s.last_error = e.what;
        return BD_ERR_INVALID_ARG;
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

int bd_batch_init(bd_sim **out, int32_t R, const int32_t *n_per, const double *xy, const double *radii,
                  const int32_t *species, const double *theta, const double *L_per, const uint64_t *seed_per,
                  const bd_force_params *fp, const bd_params *p) {
    if (!out) return BD_ERR_INVALID_ARG;
    *out = nullptr;
    std::string err;
    int rc = bd::validate_batch(R, n_per, xy, radii, species, theta, L_per, fp, p, err);
    if (rc == BD_OK && !seed_per) rc = BD_ERR_INVALID_ARG, err = "NULL seed_per";
    if (rc != BD_OK) {
        std::fprintf(stderr, "bd_batch_init: %s\n", err.c_str());
        return rc;
    }
    bd_sim *h = new (std::nothrow) bd_sim();
    if (!h) return BD_ERR_OOM;
    {
        std::lock_guard<std::mutex> lk(bd::g_alloc_mu);
        h->s.user_alloc = bd::g_alloc.alloc;
        h->s.user_free = bd::g_alloc.free;
        h->s.user_ctx = bd::g_alloc.ctx;
    }
    rc = bd::guarded(h->s, [&] {
        return bd::init_impl(h->s, R, n_per, xy, radii, species, theta, L_per, seed_per, fp, p);
    });
    if (rc != BD_OK) {
        std::fprintf(stderr, "bd_batch_init: %s\n", h->s.last_error.c_str());
        bd::UseSim use(h->s);
        bd::free_all(h->s);
        delete h;
        return rc;
    }
    *out = h;
    return BD_OK;
}

int bd_init(bd_sim **out, int32_t n, const double *xy, const double *radii, const int32_t *species,
            const double *theta, const bd_force_params *fp, const bd_params *p) {
    if (!out) return BD_ERR_INVALID_ARG;
    *out = nullptr;
    if (!p) {
        std::fprintf(stderr, "bd_init: NULL argument\n");
        return BD_ERR_INVALID_ARG;
    }
    const double L = p->L;
    const uint64_t seed = p->seed;
    return bd_batch_init(out, 1, &n, xy, radii, species, theta, &L, &seed, fp, p);
}

int bd_adjoint_begin(bd_sim *sim, int64_t nsteps, int32_t checkpoint_every) {
    if (!sim || nsteps < 1 || checkpoint_every < 1) return BD_ERR_INVALID_ARG;
    Sim &s = sim->s;
    return bd::guarded(s, [&] { return bd::adjoint_begin(s, nsteps, checkpoint_every); });
}

int bd_adjoint_backward(bd_sim *sim, const double *grad_xy, double *grad_xy0, double *grad_K) {
    if (!sim || !grad_xy) return BD_ERR_INVALID_ARG;
    Sim &s = sim->s;
    return bd::guarded(s, [&] { return bd::adjoint_backward(s, grad_xy, grad_xy0, grad_K); });
}

int bd_adjoint_backward_dev(bd_sim *sim, const double *grad_xy, double *grad_xy0, double *grad_K) {
    if (!sim || !grad_xy) return BD_ERR_INVALID_ARG;
    Sim &s = sim->s;
    return bd::guarded(s, [&] { return bd::adjoint_backward(s, grad_xy, grad_xy0, grad_K, true); });
}

int bd_get_state_dev(bd_sim *sim, double *xy_out, double *theta_out) {
    if (!sim) return BD_ERR_INVALID_ARG;
    Sim &s = sim->s;
    return bd::guarded(s, [&] {
        if (xy_out || theta_out)
            hipLaunchKernelGGL(bd::k_to_caller, dim3((s.n + 255) / 256), dim3(256), 0, s.stream, s.n,
                               (const int *)s.perm, (const double2 *)s.xy, s.th, xy_out, theta_out);
        bd::check(hipStreamSynchronize(s.stream), "sync");
        return (int)BD_OK;
    });
}

int bd_batch_layout(bd_sim *sim, int32_t *R_out, int32_t *disk_off, int32_t *frame_off) {
    if (!sim) return BD_ERR_INVALID_ARG;
    const Sim &s = sim->s;
    if (R_out) *R_out = s.R;
    for (int r = 0; r <= s.R; ++r) {
        if (disk_off) disk_off[r] = s.off_h[r];
        if (frame_off) frame_off[r] = s.foff_h[r];
    }
    return BD_OK;
}

int bd_get_force_config(bd_sim *sim, bd_force_config *out) {
    if (!sim || !out) return BD_ERR_INVALID_ARG;
    const Sim &s = sim->s;
    out->chunk = s.chunk_len;
    out->per_lane = s.per_lane;
    out->persistent = s.persistent;
    out->tiles = s.ntiles;
    out->grid = s.force_grid;
    out->tuned = s.tuned;
    out->tuned_ms = s.tuned_ms;
    return BD_OK;
}

int bd_step(bd_sim *sim, int64_t nsteps) {
    if (!sim || nsteps < 0) return BD_ERR_INVALID_ARG;
    Sim &s = sim->s;
    return bd::guarded(s, [&] {
        if (s.use_graph) return bd::run_graph_steps(s, nsteps);
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
        std::vector<double> hf(2 * (size_t)s.n);
        if (s.use_nl) {
            bd::check(hipMemcpyAsync(hf.data(), s.fsr, sizeof(double) * 2 * s.n, hipMemcpyDeviceToHost, s.stream),
                      "forces copy");
        } else {
            bd::launch_reduce_forces(s);
            bd::check(hipMemcpyAsync(hf.data(), s.fout, sizeof(double) * 2 * s.n, hipMemcpyDeviceToHost, s.stream),
                      "forces copy");
        }
        bd::check(hipStreamSynchronize(s.stream), "sync");
        for (int k = 0; k < s.n; ++k) {
            f_out[2 * (size_t)s.perm_h[k]] = hf[2 * (size_t)k];
            f_out[2 * (size_t)s.perm_h[k] + 1] = hf[2 * (size_t)k + 1];
        }
        return (int)BD_OK;
    });
}

int bd_get_state(const bd_sim *sim, double *xy_out, double *theta_out, int64_t *step_out, bd_stats *stats_out) {
    if (!sim) return BD_ERR_INVALID_ARG;
    // reading the state changes nothing the caller sees; only the detail of a failure is recorded
    Sim &s = const_cast<bd_sim *>(sim)->s;
    return bd::guarded(s, [&] {
        // positions from the packed copy, so every state a caller sees has been through it
        std::vector<double2> hp(s.n);
        std::vector<double> ht(s.n);
        if (xy_out)
            bd::check(hipMemcpyAsync(hp.data(), s.xy, sizeof(double2) * s.n, hipMemcpyDeviceToHost, s.stream), "xy");
        if (theta_out)
            bd::check(hipMemcpyAsync(ht.data(), s.th, sizeof(double) * s.n, hipMemcpyDeviceToHost, s.stream), "th");
        bd::check(hipMemcpyAsync(s.hacc, s.acc, sizeof(unsigned long long) * bd::N_ACC, hipMemcpyDeviceToHost,
                                 s.stream),
                  "acc");
        bd::check(hipStreamSynchronize(s.stream), "sync");
        for (int k = 0; k < s.n; ++k) {
            const size_t i = (size_t)s.perm_h[k];
            if (xy_out) {
                xy_out[2 * i] = hp[k].x;
                xy_out[2 * i + 1] = hp[k].y;
            }
            if (theta_out) theta_out[i] = ht[k];
        }
        if (step_out) *step_out = s.step;
        if (stats_out) {
            bd_stats st = s.st;
            st.flips_total = (int64_t)s.hacc[bd::A_FLIPS];
            st.inversion_flips = (int64_t)s.hacc[bd::A_INV_FLIPS];
            st.reversals = (int64_t)s.hacc[bd::A_REVERSALS];
            st.noise_clamps = (int64_t)s.hacc[bd::A_NOISE_CLAMPS];
            for (int j = 0; j < bd::A_CLAMP_SLOTS; ++j)
                st.noise_clamps += (int64_t)s.hacc[bd::A_CLAMP_BASE + j * bd::A_CLAMP_STRIDE];
            st.cap_hits = (int64_t)s.hacc[bd::A_CAP_HITS];
            *stats_out = st;
        }
        return (int)BD_OK;
    });
}

int bd_get_triangulation(const bd_sim *sim, int32_t *tri_out, int32_t cap, int32_t *ntri_out) {
    if (!sim || !tri_out || !ntri_out) return BD_ERR_INVALID_ARG;
    Sim &s = const_cast<bd_sim *>(sim)->s;
    if (s.ovl_method != 0) {
        s.last_error = "the list overlap method keeps no triangulation";
        return BD_ERR_INVALID_ARG;
    }
    return bd::guarded(s, [&] {
        std::vector<int> hv(s.H);
        bd::check(hipMemcpyAsync(hv.data(), s.he_v, sizeof(int) * s.H, hipMemcpyDeviceToHost, s.stream), "he_v");
        bd::check(hipStreamSynchronize(s.stream), "sync");
        int cnt = 0;
        for (int t = 0; t < s.T; ++t) {
            int a = hv[3 * t], b = hv[3 * t + 1], c = hv[3 * t + 2];
            if (a >= s.inf || b >= s.inf || c >= s.inf) continue;
            if (cnt >= cap) {
                s.last_error = "triangle buffer too small";
                return (int)BD_ERR_INVALID_ARG;
            }
            // disks in the caller's numbering; frame points keep theirs
            tri_out[3 * cnt] = a < s.n ? s.perm_h[a] : a;
            tri_out[3 * cnt + 1] = b < s.n ? s.perm_h[b] : b;
            tri_out[3 * cnt + 2] = c < s.n ? s.perm_h[c] : c;
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
        for (int r = 0; r < s.R; ++r) {
            const double L = s.L_h[r];
            for (int i = s.off_h[r]; i < s.off_h[r + 1]; ++i) {
                hx[i] = xy[2 * (size_t)s.perm_h[i]];
                hy[i] = xy[2 * (size_t)s.perm_h[i] + 1];
                const bool out = s.period > 0.0
                                     ? (hx[i] < 0.0 || hx[i] >= L || hy[i] < 0.0 || hy[i] >= L)
                                     : (hx[i] < hr[i] || hx[i] > L - hr[i] || hy[i] < hr[i] || hy[i] > L - hr[i]);
                if (!std::isfinite(hx[i]) || !std::isfinite(hy[i]) || out) {
                    s.last_error = s.period > 0.0 ? "position outside [0, L)^2 or not finite"
                                                  : "position outside the walls or not finite";
                    return (int)BD_ERR_BAD_INPUT;
                }
            }
        }
        bd::check(hipMemcpyAsync(s.xo, s.x, sizeof(double) * s.n, hipMemcpyDeviceToDevice, s.stream), "xo");
        bd::check(hipMemcpyAsync(s.yo, s.y, sizeof(double) * s.n, hipMemcpyDeviceToDevice, s.stream), "yo");
        bd::check(hipMemcpyAsync(s.x, hx.data(), sizeof(double) * s.n, hipMemcpyHostToDevice, s.stream), "x");
        bd::check(hipMemcpyAsync(s.y, hy.data(), sizeof(double) * s.n, hipMemcpyHostToDevice, s.stream), "y");
        bd::launch_pack_xy(s, s.n);
        bd::fill_int(s, s.ctl, bd::N_CTL, 0);
        s.need_rebuild = true;
        if (s.ovl_method != 0) {   // no triangulation to repair
            bd::check(hipStreamSynchronize(s.stream), "sync");
            return (int)BD_OK;
        }
        bd::Cursor c;
        return bd::host_repair(s, c, true, false, bd::MoveFrom::Previous, 0);
    });
}

int bd_set_tail_mode(bd_sim *sim, int mode) {
    if (!sim || mode < -1 || mode > 2) return BD_ERR_INVALID_ARG;
    Sim &s = sim->s;
    return bd::guarded(s, [&] {
        bd::check(hipStreamSynchronize(s.stream), "sync");
        s.tail_mode = mode;
        return (int)BD_OK;
    });
}

int bd_set_graph_mode(bd_sim *sim, int enable) {
    if (!sim) return BD_ERR_INVALID_ARG;
    Sim &s = sim->s;
    return bd::guarded(s, [&] {
        bd::check(hipStreamSynchronize(s.stream), "sync");
        s.use_graph = enable != 0;
        return (int)BD_OK;
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
    {
        bd::UseSim use(sim->s);
        bd::free_all(sim->s);
    }
    delete sim;
}

int bd_batch_step(bd_batch *b, int64_t nsteps) { return bd_step(b, nsteps); }

int bd_batch_get_state(const bd_batch *b, double *xy_out, double *theta_out, int64_t *step_out,
                       bd_stats *stats_out) {
    return bd_get_state(b, xy_out, theta_out, step_out, stats_out);
}

void bd_batch_destroy(bd_batch *b) { bd_destroy(b); }

int bd_rollout(bd_sim *sim, int64_t nsteps, int64_t checkpoint_every) {
    if (checkpoint_every < 1 || checkpoint_every > INT32_MAX) return BD_ERR_INVALID_ARG;
    return bd_adjoint_begin(sim, nsteps, (int32_t)checkpoint_every);
}

int bd_backward(bd_sim *sim, const double *grad_xy, double *grad_K, double *grad_xy0) {
    return bd_adjoint_backward(sim, grad_xy, grad_xy0, grad_K);
}

int bd_backward_dev(bd_sim *sim, const double *grad_xy, double *grad_K, double *grad_xy0) {
    return bd_adjoint_backward_dev(sim, grad_xy, grad_xy0, grad_K);
}

int bd_set_allocator(void *(*alloc_fn)(size_t bytes, void *stream, void *ctx),
                     void (*free_fn)(void *ptr, void *stream, void *ctx), void *ctx) {
    if ((alloc_fn == nullptr) != (free_fn == nullptr)) return BD_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(bd::g_alloc_mu);
    bd::g_alloc.alloc = alloc_fn;
    bd::g_alloc.free = free_fn;
    bd::g_alloc.ctx = alloc_fn ? ctx : nullptr;
    return BD_OK;
}

}  // extern "C"
