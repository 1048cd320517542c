// Short-range forces through Verlet neighbour lists on a cell grid (Sec. 2.1
// neighbour lists with cells; Sec. 2.2 cutoff rule; Sec. 5: lists built by
// grouping the particles of each cell).
//
// Lists hold every disk j within r_list = r_cut + skin of disk i at build
// time, in a fixed order (cells of the 3 x 3 block in turn, ids ascending
// inside a cell), stored slot-major (nl[k * n + i]) for coalesced reads.
// They stay valid while no disk has moved more than skin / 2 since the build:
// then every pair with d <= r_cut at force time is in the list.  The build is a
// counting sort of the disks by cell (count, exclusive scan, scatter, sort of
// each cell's few ids) followed by one thread per disk scanning the 3 x 3
// cells around it.  In graph mode the build kernels are part of every
// queued step and do nothing unless the previous step's skin test asked for
// new lists (`req` points at the step's flag; null: always build).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "bd_internal.h"
#include "geom.h"

namespace bd {
namespace {

// Separation component: from the nearest image in a periodic box of side P > 0, as is with walls (P = 0).
__device__ __forceinline__ double sep(double v, double P) { return P > 0.0 ? bd_min_image(v, P) : v; }
// The same with the box kind fixed at compile time: the list passes are instantiated for each kind, so
// the minimum image (an FP64 division) is absent from the wall-box kernels instead of selected per pair.
template <bool PER>
__device__ __forceinline__ double sep_k(double v, double P) { return PER ? bd_min_image(v, P) : v; }

__device__ __forceinline__ int cell_coord(double v, double inv_cell, int nc) {
    int c = (int)(v * inv_cell);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

// List passes (force, overlap gather): neighbours whose loads are issued together.
constexpr int kNlBatch = 2;

// The build kernels loop over their items with a grid of at most kBuildGrid
// workgroups: in a queued step they usually find no request and return at
// once, and a launch of few workgroups costs less.
constexpr int kBuildGrid = 512;

__global__ void k_cell_count(int n, const double *__restrict__ x, const double *__restrict__ y, double inv_cell,
                             int nc, int *__restrict__ cell_of, int *__restrict__ cell_count, const int *req) {
    if (req && !*req) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int c = cell_coord(y[i], inv_cell, nc) * nc + cell_coord(x[i], inv_cell, nc);
        cell_of[i] = c;
        atomicAdd(&cell_count[c], 1);
    }
}

// Exclusive scan of the cell counts (m = cells + 1 entries; the last count is
// 0, so start[m - 1] = n): each 1024-entry block scans in LDS and records its
// total, then every block adds the totals of the blocks before it.
constexpr int kScanBlk = 1024;

// Segments of kScanBlk entries, each scanned by one workgroup at a time (a
// workgroup takes segments blockIdx.x, blockIdx.x + gridDim.x, ...).
__global__ __launch_bounds__(kScanBlk) void k_scan_local(int m, const int *__restrict__ cnt, int *__restrict__ start,
                                                         int *__restrict__ bsum, const int *req) {
    __shared__ int buf[kScanBlk];
    if (req && !*req) return;
    const int nseg = (m + kScanBlk - 1) / kScanBlk;
    for (int seg = blockIdx.x; seg < nseg; seg += gridDim.x) {
        const int i = seg * kScanBlk + threadIdx.x;
        const int v = i < m ? cnt[i] : 0;
        __syncthreads();   // the previous segment's reads of buf are done
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < kScanBlk; off <<= 1) {
            const int add = threadIdx.x >= (unsigned)off ? buf[threadIdx.x - off] : 0;
            __syncthreads();
            buf[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < m) start[i] = buf[threadIdx.x] - v;
        if (threadIdx.x == kScanBlk - 1) bsum[seg] = buf[threadIdx.x];
    }
}

__global__ __launch_bounds__(kScanBlk) void k_scan_offsets(int m, int *__restrict__ start,
                                                           const int *__restrict__ bsum, const int *req) {
    __shared__ int total;
    if (req && !*req) return;
    const int nseg = (m + kScanBlk - 1) / kScanBlk;
    for (int seg = blockIdx.x; seg < nseg; seg += gridDim.x) {
        if (seg == 0) continue;   // uniform in the workgroup
        __syncthreads();          // the previous segment's read of total is done
        if (threadIdx.x == 0) total = 0;
        __syncthreads();
        int acc = 0;
        for (int b = threadIdx.x; b < seg; b += kScanBlk) acc += bsum[b];
        if (acc) atomicAdd(&total, acc);
        __syncthreads();
        const int i = seg * kScanBlk + threadIdx.x;
        if (i < m) start[i] += total;
    }
}

__global__ void k_cell_scatter(int n, const int *__restrict__ cell_of, const int *__restrict__ cell_start,
                               int *__restrict__ cell_fill, int *__restrict__ cell_items, const int *req) {
    if (req && !*req) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int c = cell_of[i];
        cell_items[cell_start[c] + atomicAdd(&cell_fill[c], 1)] = i;
    }
}

// One thread per cell: the scatter filled each cell in arbitrary order; sort
// it by id (cells hold a few disks) so that the lists below are deterministic.
// The cell's count and fill counter are zeroed for the next build.
__global__ void k_cell_sort(int ncell, const int *__restrict__ cell_start, int *__restrict__ cell_items,
                            int *__restrict__ cell_count, int *__restrict__ cell_fill, const int *req) {
    if (req && !*req) return;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncell; c += gridDim.x * blockDim.x) {
        cell_count[c] = 0;
        cell_fill[c] = 0;
        const int b = cell_start[c], e = cell_start[c + 1];
        for (int p = b + 1; p < e; ++p) {
            const int v = cell_items[p];
            int q = p;
            while (q > b && cell_items[q - 1] > v) {
                cell_items[q] = cell_items[q - 1];
                --q;
            }
            cell_items[q] = v;
        }
    }
}

// One thread per disk: neighbours within r_list from the 3 x 3 cells, in cell
// order and by id inside a cell, written straight to the slot-major list (at
// most CAP; the largest count above CAP is reported so the caller can grow the
// lists).  The position at build time is kept for the skin test.
// The list of disk i (see k_nl_build).
template <int CAP>
__device__ __forceinline__ void nl_build_one(int i, int n, const double *__restrict__ x, const double *__restrict__ y,
                                             double inv_cell, int nc, double rl2, const int *__restrict__ cell_start,
                                             const int *__restrict__ cell_items, int *__restrict__ nl,
                                             int *__restrict__ nl_cnt, double *__restrict__ xb,
                                             double *__restrict__ yb, int *__restrict__ overflow, double P) {
#pragma clang fp contract(off)
    const double xi = x[i], yi = y[i];
    const int cx = cell_coord(xi, inv_cell, nc), cy = cell_coord(yi, inv_cell, nc);
    int cnt = 0;
    // periodic box (P > 0): the 3 x 3 block wraps around (at least 3 cells a row, so no cell twice)
    for (int oy = -1; oy <= 1; ++oy) {
        int gy = cy + oy;
        if (P > 0.0)
            gy = gy < 0 ? gy + nc : (gy >= nc ? gy - nc : gy);
        else if (gy < 0 || gy >= nc)
            continue;
        for (int ox = -1; ox <= 1; ++ox) {
            int gx = cx + ox;
            if (P > 0.0)
                gx = gx < 0 ? gx + nc : (gx >= nc ? gx - nc : gx);
            else if (gx < 0 || gx >= nc)
                continue;
            const int c = gy * nc + gx;
            for (int p = cell_start[c]; p < cell_start[c + 1]; ++p) {
                const int j = cell_items[p];
                if (j == i) continue;
                const double dx = sep(xi - x[j], P), dy = sep(yi - y[j], P);
                if (dx * dx + dy * dy > rl2) continue;
                if (cnt < CAP) nl[(size_t)cnt * n + i] = j;
                ++cnt;
            }
        }
    }
    if (cnt > CAP) atomicMax(overflow, cnt);
    nl_cnt[i] = cnt < CAP ? cnt : CAP;
    xb[i] = xi;
    yb[i] = yi;
}

template <int CAP>
__global__ __launch_bounds__(256) void k_nl_build(int n, const double *__restrict__ x, const double *__restrict__ y,
                                                  double inv_cell, int nc, double rl2,
                                                  const int *__restrict__ cell_start,
                                                  const int *__restrict__ cell_items, int *__restrict__ nl,
                                                  int *__restrict__ nl_cnt, double *__restrict__ xb,
                                                  double *__restrict__ yb, int *__restrict__ overflow, const int *req,
                                                  double P) {
#pragma clang fp contract(off)
    if (req && !*req) return;
    for (int i = xcd_block() * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        nl_build_one<CAP>(i, n, x, y, inv_cell, nc, rl2, cell_start, cell_items, nl, nl_cnt, xb, yb, overflow, P);
}

// Pair force over the list: F_i = sum_j K[s_i][s_j] g(d) (r_i - r_j)/d for
// d <= r_cut, g(d) = A exp(-d/lam)/d (screened) or d^-q (power).  The
// separation, its length and the cutoff test are FP64 (positions stay FP64);
// T is the precision of the law's arithmetic and of the sum (FP32 or FP64).  ONE_SPECIES: a single
// species, so no neighbour's species is read.
template <typename T, bool ONE_SPECIES, bool PER>
__global__ __launch_bounds__(256) void k_force_nl(int n, const double2 *__restrict__ xy, const int *__restrict__ sp, const double *__restrict__ K, int S,
                                                  int kind, double q, double A, double lam, double rc,
                                                  const int *__restrict__ nl, const int *__restrict__ nl_cnt,
                                                  double2 *__restrict__ f, const StepBase *__restrict__ base,
                                                  int *__restrict__ ctl, double P) {
#pragma clang fp contract(off)
    int i = xcd_block() * blockDim.x + threadIdx.x;
    if (base->stop) return;
    // after a rebuild inside a queued step: count it, and stop the step here if a disk had more
    // neighbours than the lists hold (the host grows them and runs the step again)
    const bool built = base->nl_now != 0;
    const bool over = built && ctl[K_NL_OVERFLOW] > 0;
    if (built && blockIdx.x == 0 && threadIdx.x == 0) {
        ctl[K_NL_BUILT] = 1;
        if (over) {
            ctl[K_REASON] = HALT_NL_CAPACITY;
            ctl[K_STAGE] = 0;
            ctl[K_HALT] = 1;
        }
    }
    if (over || i >= n) return;
    const double2 pi = xy[i];
    const double xi = pi.x, yi = pi.y;
    const int si = ONE_SPECIES ? 0 : sp[i];
    const T k0 = (T)K[0];
    const T lamT = (T)lam, AT = (T)A, qT = (T)q;
    constexpr bool F32 = sizeof(T) == 4;
    const T inv_lam = (T)(1.0 / lam);   // FP32: one reciprocal of the separation per pair instead of three divisions
    const int m = nl_cnt[i];
    T fx = (T)0, fy = (T)0;
    // kNlBatch neighbours at a time: their ids, then their positions, are all loaded before the sums,
    // which keep the list order (slots past the count read disk i itself and are not summed)
    for (int k = 0; k < m; k += kNlBatch) {
        int jb[kNlBatch];
#pragma unroll
        for (int u = 0; u < kNlBatch; ++u) jb[u] = k + u < m ? nl[(size_t)(k + u) * n + i] : i;
        double xj[kNlBatch], yj[kNlBatch];
        int sj[kNlBatch];
#pragma unroll
        for (int u = 0; u < kNlBatch; ++u) {
            const double2 pj = xy[jb[u]];
            xj[u] = pj.x;
            yj[u] = pj.y;
            sj[u] = ONE_SPECIES ? 0 : sp[jb[u]];
        }
#pragma unroll
        for (int u = 0; u < kNlBatch; ++u) {
            if (k + u >= m) break;
            const double ddx = sep_k<PER>(xi - xj[u], P), ddy = sep_k<PER>(yi - yj[u], P);
            const double dd = sqrt(ddx * ddx + ddy * ddy);
            if (dd > rc) continue;   // the cutoff decision in FP64 in both precisions
            const T dx = (T)ddx, dy = (T)ddy, d = (T)dd;
            T s;
            if (kind == BD_FORCE_SCREENED) {
                if (F32) {
                    const T r = (T)1 / d;
                    s = AT * exp(-d * inv_lam) * (r * r);
                } else {
                    s = AT * exp(-d / lamT) / d / d;
                }
            } else
                s = pow(d, -qT) / d;
            s *= ONE_SPECIES ? k0 : (T)K[si * S + sj[u]];
            fx += s * dx;
            fy += s * dy;
        }
    }
    f[i] = make_double2((double)fx, (double)fy);
}

// Skin test at the end of a step: has any disk moved more than skin / 2 since
// the lists were built?  (strict, displacement including corrections and walls)
// The request also goes to the step base, where the next queued step finds it.
// (Steps queued after one that halted run it too, harmlessly: the host clears
// both flags before it tests the halted step's final positions itself.)
__global__ void k_skin_check(int n, const double *__restrict__ x, const double *__restrict__ y,
                             const double *__restrict__ xb, const double *__restrict__ yb, double half_skin2,
                             int *__restrict__ flag, StepBase *__restrict__ base, double P) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool out = false;
    if (i < n) {
        const double dx = sep(x[i] - xb[i], P), dy = sep(y[i] - yb[i], P);
        out = dx * dx + dy * dy > half_skin2;
    }
    if (__ballot(out) != 0 && __lane_id() == 0) {
        atomicOr(flag, 1);
        atomicOr(&base->nl_req, 1);
    }
}

// ---------------------------------------------------------------- overlap rounds over the lists
// The paper's short-range variant (Sec. 5) finds overlapping pairs through the
// neighbour lists instead of a triangulation.  Round k, gather: every disk sums
// its Jacobi displacement over the listed partners that overlap it (Sec. 2.3
// displacement along the unit vector, factor f), truncates the sum to
// cap_frac * r (Sec. 4.4) and applies the walls; a disk that moved is queued
// with its new position.  Overlapping pairs are counted once (from the lower
// id).  The lists contain every pair closer than contact only while no disk
// has moved more than `margin` since the build; a disk beyond it raises
// K_NL_STALE and the round is not applied (the host rebuilds the lists and
// repeats the detection).  Apply: if the round found nothing the overlap loop
// is done; otherwise the queued disks take their new positions (all at once,
// after every gather has read the old ones).
// Workgroups of 1024 threads, at most kNlGatherGrid of them, each disk once
// (grid-stride): the disks a workgroup queues are staged in LDS with their
// new positions and reserved on the shared counter once per workgroup, and the
// pair, cap and stale counts are added once per workgroup (updates of one
// address from every CU serialise).
constexpr int kNlGatherBlock = 1024;
constexpr int kNlGatherGrid = 512;
constexpr int kNlStage = 2048;

// UNI: every disk has the same radius (the contact distance is then 2 r_i, the same value rad[i] + rad[j]
// gives), so the neighbours' radii are not loaded.
// The arguments of the overlap rounds over the lists.
struct NlArgs {
    int n;
    const double2 *xy;
    const double *rad;
    double L;
    const int *nl, *nl_cnt;
    const double *xb, *yb;
    double margin2, f, cap_frac, keep, P;
};

// Round k's gather for disk i: the sum over its listed neighbours closer than
// contact (in list order), truncated to cap_frac * r_i, walls or wrap; moved
// when it has an overlapping neighbour.  Counts the overlapping pairs it owns
// (the lower id), cap hits, and whether the disk is beyond the list margin.
template <bool PER, bool UNI>
__device__ __forceinline__ void nl_gather_disk(const NlArgs &a, int i, bool &moved, double &nx, double &ny,
                                               int &pairs, int &caps, bool &stale_any) {
#pragma clang fp contract(off)
    const int n = a.n;
    const double2 *__restrict__ xy = a.xy;
    const double *__restrict__ rad = a.rad;
    const int *__restrict__ nl = a.nl;
    const double P = a.P, keep = a.keep, f = a.f;
    const double2 pi = xy[i];
    const double xi = pi.x, yi = pi.y, ri = rad[i];
    const double ex = sep_k<PER>(xi - a.xb[i], P), ey = sep_k<PER>(yi - a.yb[i], P);
    stale_any |= ex * ex + ey * ey > a.margin2;
    const int m = a.nl_cnt[i];
    double sx = 0.0, sy = 0.0;
    for (int q = 0; q < m; q += kNlBatch) {   // batched loads as in k_force_nl, sums in list order
        int jb[kNlBatch];
#pragma unroll
        for (int u = 0; u < kNlBatch; ++u) jb[u] = q + u < m ? nl[(size_t)(q + u) * n + i] : i;
        double xj[kNlBatch], yj[kNlBatch], rj[kNlBatch];
#pragma unroll
        for (int u = 0; u < kNlBatch; ++u) {
            const double2 pj = xy[jb[u]];
            xj[u] = pj.x;
            yj[u] = pj.y;
            rj[u] = UNI ? ri : rad[jb[u]];
        }
#pragma unroll
        for (int u = 0; u < kNlBatch; ++u) {
            if (q + u >= m) break;
            const double dx = sep_k<PER>(xi - xj[u], P), dy = sep_k<PER>(yi - yj[u], P);
            const double d = sqrt(dx * dx + dy * dy);
            const double contact = ri + rj[u];
            if (d < contact * keep) {
                const double sc = f * (contact - d) / d;
                sx += sc * dx;
                sy += sc * dy;
                moved = true;
                if (i < jb[u]) ++pairs;
            }
        }
    }
    if (moved) {
        const double len = sqrt(sx * sx + sy * sy);
        const double cap = a.cap_frac * ri;
        if (len > cap) {
            const double sc = cap / len;
            sx = sx * sc;
            sy = sy * sc;
            ++caps;
        }
        nx = PER ? bd_wrap(xi + sx, P) : bd_wall(xi + sx, ri, a.L);
        ny = PER ? bd_wrap(yi + sy, P) : bd_wall(yi + sy, ri, a.L);
    }
}

template <bool PER, bool UNI>
__global__ __launch_bounds__(kNlGatherBlock) void k_ovl_nl_gather(NlArgs a, int *__restrict__ touched,
                                                                  double2 *__restrict__ newpos, int *__restrict__ ctl,
                                                                  unsigned long long *__restrict__ acc, int k) {
#pragma clang fp contract(off)
    const int n = a.n;
    __shared__ int s_id[kNlStage];
    __shared__ double2 s_pos[kNlStage];
    __shared__ int s_cnt, s_base, s_pairs, s_caps, s_stale;
    if ((ctl[K_HALT] | ctl[K_DONE]) != 0) return;   // nothing in this launch writes them: uniform
    if (threadIdx.x == 0) {
        s_cnt = 0;
        s_pairs = 0;
        s_caps = 0;
        s_stale = 0;
    }
    __syncthreads();
    int pairs = 0, caps = 0;
    bool stale_any = false;
    const int stride = gridDim.x * blockDim.x;
    for (int i0 = xcd_block() * blockDim.x; i0 < n; i0 += stride) {   // same trip count in the workgroup
        const int i = i0 + (int)threadIdx.x;
        bool moved = false;
        double nx = 0.0, ny = 0.0;
        if (i < n) nl_gather_disk<PER, UNI>(a, i, moved, nx, ny, pairs, caps, stale_any);
        // stage the queued disk (one LDS atomic per wavefront; every lane is here)
        const unsigned long long mm = __ballot(moved);
        if (mm != 0) {
            const int lane = __lane_id(), leader = __ffsll((unsigned long long)mm) - 1;
            int base = 0;
            if (lane == leader) base = atomicAdd(&s_cnt, __popcll(mm));
            base = __shfl(base, leader);
            if (moved) {
                const int pos = base + __popcll(mm & ((1ull << lane) - 1ull));
                if (pos < kNlStage) {
                    s_id[pos] = i;
                    s_pos[pos] = make_double2(nx, ny);
                } else {
                    const int g = atomicAdd(&ctl[K_TOUCH + k], 1);
                    touched[g] = i;
                    newpos[g] = make_double2(nx, ny);
                }
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        pairs += __shfl_xor(pairs, off);
        caps += __shfl_xor(caps, off);
    }
    const bool stale_w = __ballot(stale_any) != 0;
    if (__lane_id() == 0) {
        if (pairs) atomicAdd(&s_pairs, pairs);
        if (caps) atomicAdd(&s_caps, caps);
        if (stale_w) s_stale = 1;
    }
    __syncthreads();
    const int cnt = s_cnt < kNlStage ? s_cnt : kNlStage;
    if (threadIdx.x == 0) {
        if (cnt > 0) s_base = atomicAdd(&ctl[K_TOUCH + k], cnt);
        if (s_pairs) atomicAdd(&ctl[K_OVL + k], s_pairs);
        if (s_caps) atomicAdd(&acc[A_CAP_HITS], (unsigned long long)s_caps);
        if (s_stale) atomicOr(&ctl[K_NL_STALE], 1);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < cnt; q += blockDim.x) {
        touched[s_base + q] = s_id[q];
        newpos[s_base + q] = s_pos[q];
    }
}

// final_check: the last budgeted round's detection; overlaps left halt the
// step (the host continues the loop) instead of being applied.
__global__ __launch_bounds__(256) void k_ovl_nl_apply(double *__restrict__ x, double *__restrict__ y,
                                                      double2 *__restrict__ xy,
                                                      const int *__restrict__ touched,
                                                      const double2 *__restrict__ newpos, int *__restrict__ ctl, int k,
                                                      int final_check) {
    if ((ctl[K_HALT] | ctl[K_DONE]) != 0) return;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    // the counters below were written by the gather launch before this one: every thread reads the same
    if (ctl[K_NL_STALE] != 0) {
        if (lead) {
            ctl[K_REASON] = HALT_NL_STALE;
            ctl[K_STAGE] = k;
            ctl[K_HALT] = 1;
        }
        return;
    }
    if (ctl[K_OVL + k] == 0) {
        if (lead) ctl[K_DONE] = 1;
        return;
    }
    if (final_check) {
        if (lead) {
            ctl[K_REASON] = HALT_OVERLAP_BUDGET;
            ctl[K_STAGE] = k;
            ctl[K_HALT] = 1;
        }
        return;
    }
    if (lead) ctl[K_OVL_ROUNDS] = k + 1;
    const int cnt = ctl[K_TOUCH + k];
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < cnt; idx += gridDim.x * blockDim.x) {
        const int v = touched[idx];
        const double2 p = newpos[idx];
        x[v] = p.x;
        y[v] = p.y;
        xy[v] = p;
    }
}

// The later overlap rounds over the lists in one workgroup.  After a round,
// only a disk that moved in it, or a listed neighbour of one, can overlap
// another (a pair whose disks both stayed keeps its distance, and every disk
// that had an overlapping neighbour moved): round r gathers over exactly those
// disks (each once, marked with the round's stamp), with the arithmetic of the
// full pass, so it moves the same disks to the same places and counts the same
// pairs; the margin test of a disk that did not move since its last test would
// give the same answer.  Each round ends as k_ovl_nl_apply does (lists stale:
// halt; no overlap: done; the budget's last round with overlaps left: halt;
// else the queued disks take their positions), phases separated by barriers.
constexpr int kNlTailBlock = 1024;

__device__ __forceinline__ bool nl_stopped(const int *ctl) {
    return (__hip_atomic_load(ctl + K_HALT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) |
            __hip_atomic_load(ctl + K_DONE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0;
}

// (xyw is the array a.xy reads: the gathers and the position writes of a round are separated by barriers.)
template <bool PER, bool UNI>
__global__ __launch_bounds__(kNlTailBlock) void k_nl_tail(NlArgs a, NlTailPlan p, double *x, double *y, double2 *xyw,
                                                          int *touched, double2 *newpos, int *mark, int *cand,
                                                          int *ctl, unsigned long long *acc,
                                                          const StepBase *__restrict__ base) {
    __shared__ int s_nc, s_cnt, s_pairs, s_caps, s_stale, s_go;
    const int tid = threadIdx.x, n = a.n;
    // the decisions every thread follows are taken by thread 0 and read from LDS after a barrier
    if (tid == 0) s_go = nl_stopped(ctl) ? 0 : 1;
    __syncthreads();
    if (!s_go) return;
    int kprev = p.kprev;
    for (int r = 0; r < p.nr; ++r) {
        const int k = p.k[r];
        const int stamp = p.stamp0 + r + base->vbase;
        if (tid == 0) {
            s_nc = 0;
            s_cnt = 0;
            s_pairs = 0;
            s_caps = 0;
            s_stale = 0;
        }
        __syncthreads();
        // the disks of this round: those the previous round moved and their listed neighbours
        const int nprev = ctl[K_TOUCH + kprev];
        const int *prev = touched + (size_t)(kprev & 1) * n;
        for (int idx = tid; idx < nprev; idx += kNlTailBlock) {
            const int v = prev[idx];
            if ((unsigned)v >= (unsigned)n) continue;
            if (atomicExch(&mark[v], stamp) != stamp) cand[atomicAdd(&s_nc, 1)] = v;
            const int m = a.nl_cnt[v];
            for (int q = 0; q < m; ++q) {
                const int w = a.nl[(size_t)q * n + v];
                if (atomicExch(&mark[w], stamp) != stamp) cand[atomicAdd(&s_nc, 1)] = w;
            }
        }
        __syncthreads();
        const int nc = s_nc;
        int *cur = touched + (size_t)(k & 1) * n;
        int pairs = 0, caps = 0;
        bool stale = false;
        for (int c = tid; c < nc; c += kNlTailBlock) {
            const int i = cand[c];
            bool moved = false;
            double nx = 0.0, ny = 0.0;
            nl_gather_disk<PER, UNI>(a, i, moved, nx, ny, pairs, caps, stale);
            if (moved) {
                const int g = atomicAdd(&s_cnt, 1);
                cur[g] = i;
                newpos[g] = make_double2(nx, ny);
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            pairs += __shfl_xor(pairs, off);
            caps += __shfl_xor(caps, off);
        }
        const bool stale_w = __ballot(stale) != 0;
        if (__lane_id() == 0) {
            if (pairs) atomicAdd(&s_pairs, pairs);
            if (caps) atomicAdd(&s_caps, caps);
            if (stale_w) s_stale = 1;
        }
        __syncthreads();
        if (tid == 0) {
            ctl[K_TOUCH + k] = s_cnt;
            ctl[K_OVL + k] += s_pairs;
            if (s_caps) atomicAdd(&acc[A_CAP_HITS], (unsigned long long)s_caps);
            if (s_stale) {
                ctl[K_NL_STALE] = 1;
                ctl[K_REASON] = HALT_NL_STALE;
                ctl[K_STAGE] = k;
                ctl[K_HALT] = 1;
            } else if (s_pairs == 0) {
                ctl[K_DONE] = 1;
            } else if (p.final_last && r + 1 == p.nr) {
                ctl[K_REASON] = HALT_OVERLAP_BUDGET;
                ctl[K_STAGE] = k;
                ctl[K_HALT] = 1;
            } else {
                ctl[K_OVL_ROUNDS] = k + 1;
            }
            s_go = ctl[K_HALT] == 0 && ctl[K_DONE] == 0;
        }
        __syncthreads();
        if (!s_go) return;
        const int cnt = s_cnt;
        for (int idx = tid; idx < cnt; idx += kNlTailBlock) {
            const int v = cur[idx];
            const double2 np = newpos[idx];
            x[v] = np.x;
            y[v] = np.y;
            xyw[v] = np;
        }
        __syncthreads();
        kprev = k;
    }
}

inline int blocks(int n) { return (n + 255) / 256; }
inline int capped(int b, int cap = kBuildGrid) { return b < 1 ? 1 : (b > cap ? cap : b); }

NlArgs nl_args(const Sim &s) {
    NlArgs a;
    a.n = s.n;
    a.xy = s.xy;
    a.rad = s.rad;
    a.L = s.L_h[0];
    a.nl = s.nl;
    a.nl_cnt = s.nl_cnt;
    a.xb = s.xbuild;
    a.yb = s.ybuild;
    a.margin2 = s.nl_margin * s.nl_margin;
    a.f = s.p.overlap_factor;
    a.cap_frac = s.p.cap_frac;
    a.keep = 1.0 - s.p.contact_tol;
    a.P = s.period;
    return a;
}

}  // namespace

// Blocks of the cell-count scan (cells + 1 entries); sizes its per-block totals.
int verlet_scan_blocks(int ncells) { return (ncells + 1 + kScanBlk - 1) / kScanBlk; }

namespace {

// The build kernels; req = null builds unconditionally (the caller zeroed
// cell_count, cell_fill and the overflow flag), else only when *req != 0.
void enqueue_build(Sim &s, const int *req) {
    const double inv_cell = (double)s.nl_nc / s.L_h[0];
    const int m = s.nl_ncell + 1;
    hipLaunchKernelGGL(k_cell_count, dim3(capped(blocks(s.n))), dim3(256), 0, s.stream, s.n, s.x, s.y, inv_cell, s.nl_nc,
                       s.cell_of, s.cell_count, req);
    hipLaunchKernelGGL(k_scan_local, dim3(capped(verlet_scan_blocks(s.nl_ncell), 256)), dim3(kScanBlk), 0, s.stream, m,
                       (const int *)s.cell_count, s.cell_start, s.scan_bsum, req);
    hipLaunchKernelGGL(k_scan_offsets, dim3(capped(verlet_scan_blocks(s.nl_ncell), 256)), dim3(kScanBlk), 0, s.stream, m,
                       s.cell_start, (const int *)s.scan_bsum, req);
    hipLaunchKernelGGL(k_cell_scatter, dim3(capped(blocks(s.n))), dim3(256), 0, s.stream, s.n, s.cell_of, s.cell_start,
                       s.cell_fill, s.cell_items, req);
    hipLaunchKernelGGL(k_cell_sort, dim3(capped(blocks(s.nl_ncell))), dim3(256), 0, s.stream, s.nl_ncell, s.cell_start,
                       s.cell_items, s.cell_count, s.cell_fill, req);
    const double rl = s.fp.cutoff + s.fp.skin;
    if (s.nl_cap <= 32)
        hipLaunchKernelGGL(k_nl_build<32>, dim3(capped(blocks(s.n), 2 * kBuildGrid)), dim3(256), 0, s.stream, s.n, s.x, s.y, inv_cell,
                           s.nl_nc, rl * rl, s.cell_start, s.cell_items, s.nl, s.nl_cnt, s.xbuild, s.ybuild,
                           s.ctl + K_NL_OVERFLOW, req, s.period);
    else
        hipLaunchKernelGGL(k_nl_build<96>, dim3(capped(blocks(s.n), 2 * kBuildGrid)), dim3(256), 0, s.stream, s.n, s.x, s.y, inv_cell,
                           s.nl_nc, rl * rl, s.cell_start, s.cell_items, s.nl, s.nl_cnt, s.xbuild, s.ybuild,
                           s.ctl + K_NL_OVERFLOW, req, s.period);
}

}  // namespace

// Rebuilds the lists from the current positions.  The caller zeroed
// cell_count, cell_fill and the overflow flag.
void launch_verlet_build(Sim &s) { enqueue_build(s, nullptr); }

void launch_verlet_build_requested(Sim &s) {
    StepBase *b = (StepBase *)s.dbase;
    enqueue_build(s, &b->nl_now);   // the force kernel that follows records the rebuild and checks its capacity
}

void launch_force_nl(Sim &s) {
    const bool per = s.period > 0.0;
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(blocks(s.n)), dim3(256), 0, s.stream, s.n, (const double2 *)s.xy,
                           (const int *)s.sp, (const double *)s.Kd, s.S, s.fp.kind, s.fp.q,
                           s.fp.A, s.fp.lambda, s.fp.cutoff, (const int *)s.nl, (const int *)s.nl_cnt, s.fsr,
                           (const StepBase *)s.dbase, s.ctl, s.period);
    };
    if (s.fp32)
        per ? (s.S == 1 ? go(k_force_nl<float, true, true>) : go(k_force_nl<float, false, true>))
            : (s.S == 1 ? go(k_force_nl<float, true, false>) : go(k_force_nl<float, false, false>));
    else
        per ? (s.S == 1 ? go(k_force_nl<double, true, true>) : go(k_force_nl<double, false, true>))
            : (s.S == 1 ? go(k_force_nl<double, true, false>) : go(k_force_nl<double, false, false>));
}

void launch_ovl_nl_gather(Sim &s, int k) {
    const int g = std::max(1, std::min(kNlGatherGrid, (s.n + kNlGatherBlock - 1) / kNlGatherBlock));
    const bool per = s.period > 0.0, uni = s.rad_uni > 0.0;
    hipLaunchKernelGGL(per ? (uni ? k_ovl_nl_gather<true, true> : k_ovl_nl_gather<true, false>)
                           : (uni ? k_ovl_nl_gather<false, true> : k_ovl_nl_gather<false, false>),
                       dim3(g), dim3(kNlGatherBlock), 0, s.stream, nl_args(s), s.touched + (size_t)(k & 1) * s.n,
                       s.newpos, s.ctl, s.acc, k);
}

void launch_nl_tail(Sim &s, const NlTailPlan &p) {
    const bool per = s.period > 0.0, uni = s.rad_uni > 0.0;
    hipLaunchKernelGGL(per ? (uni ? k_nl_tail<true, true> : k_nl_tail<true, false>)
                           : (uni ? k_nl_tail<false, true> : k_nl_tail<false, false>),
                       dim3(1), dim3(kNlTailBlock), 0, s.stream, nl_args(s), p, s.x, s.y, s.xy, s.touched, s.newpos,
                       s.vstamp, s.nl_cand, s.ctl, s.acc, (const StepBase *)s.dbase);
}

void launch_ovl_nl_apply(Sim &s, int k, bool final_check) {
    // the queued disks are usually a few percent of all: a grid for a tenth of them
    const int g = std::max(1, std::min(blocks(s.n), blocks(s.n / 10 + 1)));
    hipLaunchKernelGGL(k_ovl_nl_apply, dim3(g), dim3(256), 0, s.stream, s.x, s.y, s.xy,
                       (const int *)(s.touched + (size_t)(k & 1) * s.n), (const double2 *)s.newpos, s.ctl, k,
                       final_check ? 1 : 0);
}

void launch_skin_check(Sim &s) {
    const double h = 0.5 * s.fp.skin;
    hipLaunchKernelGGL(k_skin_check, dim3(blocks(s.n)), dim3(256), 0, s.stream, s.n, s.x, s.y, s.xbuild, s.ybuild,
                       h * h, s.ctl + K_NL_REBUILD, (StepBase *)s.dbase, s.period);
}

}  // namespace bd
