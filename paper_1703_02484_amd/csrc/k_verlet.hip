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
// cells around it.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "bd_internal.h"
#include "geom.h"

namespace bd {
namespace {

__device__ __forceinline__ int cell_coord(double v, double inv_cell, int nc) {
    int c = (int)(v * inv_cell);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__global__ void k_cell_count(int n, const double *__restrict__ x, const double *__restrict__ y, double inv_cell,
                             int nc, int *__restrict__ cell_of, int *__restrict__ cell_count) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = cell_coord(y[i], inv_cell, nc) * nc + cell_coord(x[i], inv_cell, nc);
    cell_of[i] = c;
    atomicAdd(&cell_count[c], 1);
}

__global__ void k_cell_scatter(int n, const int *__restrict__ cell_of, const int *__restrict__ cell_start,
                               int *__restrict__ cell_fill, int *__restrict__ cell_items) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = cell_of[i];
    cell_items[cell_start[c] + atomicAdd(&cell_fill[c], 1)] = i;
}

// One thread per cell: the scatter filled each cell in arbitrary order; sort
// it by id (cells hold a few disks) so that the lists below are deterministic.
__global__ void k_cell_sort(int ncell, const int *__restrict__ cell_start, int *__restrict__ cell_items) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
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

// One thread per disk: neighbours within r_list from the 3 x 3 cells, in cell
// order and by id inside a cell, written straight to the slot-major list (at
// most CAP; the largest count above CAP is reported so the caller can grow the
// lists).  The position at build time is kept for the skin test.
template <int CAP>
__global__ __launch_bounds__(256) void k_nl_build(int n, const double *__restrict__ x, const double *__restrict__ y,
                                                  double inv_cell, int nc, double rl2,
                                                  const int *__restrict__ cell_start,
                                                  const int *__restrict__ cell_items, int *__restrict__ nl,
                                                  int *__restrict__ nl_cnt, double *__restrict__ xb,
                                                  double *__restrict__ yb, int *__restrict__ overflow) {
#pragma clang fp contract(off)
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double xi = x[i], yi = y[i];
    const int cx = cell_coord(xi, inv_cell, nc), cy = cell_coord(yi, inv_cell, nc);
    int cnt = 0;
    for (int gy = cy - 1; gy <= cy + 1; ++gy) {
        if (gy < 0 || gy >= nc) continue;
        for (int gx = cx - 1; gx <= cx + 1; ++gx) {
            if (gx < 0 || gx >= nc) continue;
            const int c = gy * nc + gx;
            for (int p = cell_start[c]; p < cell_start[c + 1]; ++p) {
                const int j = cell_items[p];
                if (j == i) continue;
                const double dx = xi - x[j], dy = yi - y[j];
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

// Pair force over the list (FP64): F_i = sum_j K[s_i][s_j] g(d) (r_i - r_j)/d
// for d <= r_cut, g(d) = A exp(-d/lam)/d (screened) or d^-q (power).
__global__ __launch_bounds__(256) void k_force_nl(int n, const double *__restrict__ x, const double *__restrict__ y,
                                                  const int *__restrict__ sp, const double *__restrict__ K, int S,
                                                  int kind, double q, double A, double lam, double rc,
                                                  const int *__restrict__ nl, const int *__restrict__ nl_cnt,
                                                  double2 *__restrict__ f, const StepBase *__restrict__ base) {
#pragma clang fp contract(off)
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || base->stop) return;
    const double xi = x[i], yi = y[i];
    const int si = sp[i];
    const int m = nl_cnt[i];
    double fx = 0.0, fy = 0.0;
    for (int k = 0; k < m; ++k) {
        const int j = nl[(size_t)k * n + i];
        const double dx = xi - x[j], dy = yi - y[j];
        const double d = sqrt(dx * dx + dy * dy);
        if (d > rc) continue;
        double s;
        if (kind == BD_FORCE_SCREENED)
            s = A * exp(-d / lam) / d / d;
        else
            s = pow(d, -q) / d;
        s *= K[si * S + sp[j]];
        fx += s * dx;
        fy += s * dy;
    }
    f[i] = make_double2(fx, fy);
}

// Skin test at the end of a step: has any disk moved more than skin / 2 since
// the lists were built?  (strict, displacement including corrections and walls)
__global__ void k_skin_check(int n, const double *__restrict__ x, const double *__restrict__ y,
                             const double *__restrict__ xb, const double *__restrict__ yb, double half_skin2,
                             int *__restrict__ flag) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool out = false;
    if (i < n) {
        const double dx = x[i] - xb[i], dy = y[i] - yb[i];
        out = dx * dx + dy * dy > half_skin2;
    }
    if (__ballot(out) != 0 && __lane_id() == 0) atomicOr(flag, 1);
}

inline int blocks(int n) { return (n + 255) / 256; }

}  // namespace

// Sizes the scan's temporary storage; called once at init.
size_t verlet_scan_bytes(int ncells) {
    size_t bytes = 0;
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, (int *)nullptr, (int *)nullptr, ncells + 1);
    return bytes;
}

// Rebuilds the lists from the current positions.  The caller zeroed
// cell_count, cell_fill and the overflow flag.
void launch_verlet_build(Sim &s) {
    const double inv_cell = (double)s.nl_nc / s.L_h[0];
    hipLaunchKernelGGL(k_cell_count, dim3(blocks(s.n)), dim3(256), 0, s.stream, s.n, s.x, s.y, inv_cell, s.nl_nc,
                       s.cell_of, s.cell_count);
    size_t bytes = s.scan_bytes;
    (void)hipcub::DeviceScan::ExclusiveSum(s.scan_tmp, bytes, s.cell_count, s.cell_start, s.nl_ncell + 1, s.stream);
    hipLaunchKernelGGL(k_cell_scatter, dim3(blocks(s.n)), dim3(256), 0, s.stream, s.n, s.cell_of, s.cell_start,
                       s.cell_fill, s.cell_items);
    hipLaunchKernelGGL(k_cell_sort, dim3(blocks(s.nl_ncell)), dim3(256), 0, s.stream, s.nl_ncell, s.cell_start,
                       s.cell_items);
    const double rl = s.fp.cutoff + s.fp.skin;
    if (s.nl_cap <= 32)
        hipLaunchKernelGGL(k_nl_build<32>, dim3(blocks(s.n)), dim3(256), 0, s.stream, s.n, s.x, s.y, inv_cell,
                           s.nl_nc, rl * rl, s.cell_start, s.cell_items, s.nl, s.nl_cnt, s.xbuild, s.ybuild,
                           s.ctl + K_NL_OVERFLOW);
    else
        hipLaunchKernelGGL(k_nl_build<96>, dim3(blocks(s.n)), dim3(256), 0, s.stream, s.n, s.x, s.y, inv_cell,
                           s.nl_nc, rl * rl, s.cell_start, s.cell_items, s.nl, s.nl_cnt, s.xbuild, s.ybuild,
                           s.ctl + K_NL_OVERFLOW);
}

void launch_force_nl(Sim &s) {
    hipLaunchKernelGGL(k_force_nl, dim3(blocks(s.n)), dim3(256), 0, s.stream, s.n, s.x, s.y, s.sp, s.Kd, s.S,
                       s.fp.kind, s.fp.q, s.fp.A, s.fp.lambda, s.fp.cutoff, s.nl, s.nl_cnt, s.fsr,
                       (const StepBase *)s.dbase);
}

void launch_skin_check(Sim &s) {
    const double h = 0.5 * s.fp.skin;
    hipLaunchKernelGGL(k_skin_check, dim3(blocks(s.n)), dim3(256), 0, s.stream, s.n, s.x, s.y, s.xbuild, s.ybuild,
                       h * h, s.ctl + K_NL_REBUILD);
}

}  // namespace bd
