// Adjoint (reverse-mode) sweep of the time step: gradients of a loss on the
// final positions with respect to the initial positions and the strength
// matrix K.  Not part of the paper's method.  The step is differentiated as
// written with every discrete choice of the forward pass held fixed: the
// overlapping partners of each correction round (the correction acts as a
// projection onto that round's contact set), the cap branch and the wall
// branches.  Noise and the director angles do not depend on the positions.
//
// Per step, in reverse (lambda = dL/dx after the step):
//   overlap rounds, last first: mu = S_w lambda (wall slopes), nu = C^T mu
//     (cap: (c/|D|)(I - e e^T) when the cap acted), then for a moved disk m
//     lambda_m = mu_m + sum_{j overlapping m} A_mj (nu_m - nu_j),
//     A = f((sigma/d - 1) I - (sigma/d) n n^T) at the positions before the round;
//   the move x* = x + dt F(x) + noise, then walls:
//     lambda* = S_w lambda,
//     dL/dK[a][b] += dt sum_{i in a} lambda*_i . Phi_{i,b},  Phi_{i,b} = sum_{j in b} u_ij / d^3,
//     lambda = lambda* + dt g,  g_m = sum_j J(u_mj) (K[s_m][s_j] lambda*_m - K[s_j][s_m] lambda*_j),
//     J(u) = (I - 3 n n^T) / d^3 for the inverse-square law.
// g is an all-pairs sum like the force; it runs over the force's tiles and
// is reduced per particle in a fixed chunk order, so the sweep is
// deterministic.
#include <hip/hip_runtime.h>

#include "bd_internal.h"
#include "geom.h"

namespace bd {
namespace {

constexpr int kAdjBlock = 256;

// ---------------------------------------------------------------- overlap rounds
__global__ void k_adj_round_prep(int e0, int cnt, const int *__restrict__ ev, const double2 *__restrict__ eold,
                                 const double2 *__restrict__ edisp, const signed char *__restrict__ ewf,
                                 const double *__restrict__ rad, double cap_frac, const double2 *__restrict__ lam,
                                 double2 *__restrict__ nu, double *__restrict__ bx, double *__restrict__ by) {
#pragma clang fp contract(off)
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= cnt) return;
    const int e = e0 + idx;
    const int v = ev[e];
    const double2 l = lam[v];
    double mx = ewf[2 * (size_t)e] * l.x, my = ewf[2 * (size_t)e + 1] * l.y;
    const double2 D = edisp[e];
    const double len = sqrt(D.x * D.x + D.y * D.y);
    const double cap = cap_frac * rad[v];
    if (len > cap) {
        const double ex = D.x / len, ey = D.y / len, sc = cap / len;
        const double em = ex * mx + ey * my;
        mx = sc * (mx - ex * em);
        my = sc * (my - ey * em);
    }
    nu[v] = make_double2(mx, my);
    bx[v] = eold[e].x;
    by[v] = eold[e].y;
}

__global__ void k_adj_round_apply(int e0, int cnt, const int *__restrict__ ev, const signed char *__restrict__ ewf,
                                  const int *__restrict__ ecnt, const int *__restrict__ enb,
                                  const double *__restrict__ rad, double f, const double2 *__restrict__ nu,
                                  const double *__restrict__ bx, const double *__restrict__ by,
                                  double2 *__restrict__ lam) {
#pragma clang fp contract(off)
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= cnt) return;
    const int e = e0 + idx;
    const int v = ev[e];
    const double2 l = lam[v];
    double ax = ewf[2 * (size_t)e] * l.x, ay = ewf[2 * (size_t)e + 1] * l.y;
    const double2 nv = nu[v];
    const double xv = bx[v], yv = by[v], rv = rad[v];
    const int na = ecnt[e];
    for (int k = 0; k < na; ++k) {
        const int j = enb[(size_t)e * MAXACT + k];
        const double ux = xv - bx[j], uy = yv - by[j];
        const double d = sqrt(ux * ux + uy * uy);
        const double nx = ux / d, ny = uy / d;
        const double a = (rv + rad[j]) / d;
        const double2 nj = nu[j];
        const double dx = nv.x - nj.x, dy = nv.y - nj.y;
        const double nd = nx * dx + ny * dy;
        ax += f * ((a - 1.0) * dx - a * nx * nd);
        ay += f * ((a - 1.0) * dy - a * ny * nd);
    }
    lam[v] = make_double2(ax, ay);
}

// ---------------------------------------------------------------- the move
__global__ void k_adj_em_slopes(int n, const signed char *__restrict__ wf, double2 *__restrict__ lam) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 l = lam[i];
    lam[i] = make_double2(wf[2 * (size_t)i] * l.x, wf[2 * (size_t)i + 1] * l.y);
}

// Sorted copies of the positions before the step: (x, y, lambda*) in FP64 for
// the adjoint pair sum, and the force kernel's own copy to recompute Phi.
template <typename T2>
__global__ void k_adj_cast(int n, const double *__restrict__ px, const double *__restrict__ py,
                           const double2 *__restrict__ lam, const int *__restrict__ sorted_id,
                           double4 *__restrict__ pj4, T2 *__restrict__ pj) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int i = sorted_id[k];
    const double x = px[i], y = py[i];
    const double2 l = lam[i];
    pj4[k] = make_double4(x, y, l.x, l.y);
    T2 v;
    v.x = x;
    v.y = y;
    pj[k] = v;
}

// dL/dK[a][b] += dt sum_{i in a} lambda*_i . Phi_{i,b}.  First each particle
// writes its row dt lambda*_i . Phi_{i,b} (b = 0..S-1), then every block of
// kAdjBlock particles adds its sum per (a, b) to its own accumulator in
// particle order, so the result does not depend on scheduling.
template <typename T2>
__global__ void k_adj_dk_rows(int n, int S, const T2 *__restrict__ part, const RepInfo *__restrict__ reps,
                              const int *__restrict__ rep_of, const int *__restrict__ chunk_spec,
                              const int *__restrict__ pos_of, const double2 *__restrict__ lam, double dt,
                              double *__restrict__ rows) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const RepInfo ri = reps[rep_of[i]];
    const long long row = ri.poff + (pos_of[i] - ri.off);
    const double2 l = lam[i];
    double *out = rows + (size_t)i * S;
    for (int b = 0; b < S; ++b) out[b] = 0.0;
    for (int c = 0; c < ri.nch; ++c) {
        const int b = chunk_spec[ri.cfirst + c];
        const T2 p = part[row + (long long)c * ri.n];
        out[b] += dt * (l.x * (double)p.x + l.y * (double)p.y);
    }
}

__global__ void k_adj_dk_blocks(int n, int S, int nblk, const int *__restrict__ sp, const double *__restrict__ rows,
                                double *__restrict__ dk_blk) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nblk * S * S) return;
    const int blk = t / (S * S), ab = t % (S * S), a = ab / S, b = ab % S;
    const int i0 = blk * kAdjBlock, i1 = i0 + kAdjBlock < n ? i0 + kAdjBlock : n;
    double sum = 0.0;
    for (int i = i0; i < i1; ++i)
        if (sp[i] == a) sum += rows[(size_t)i * S + b];
    dk_blk[t] += sum;
}

__global__ void k_adj_dk_final(int nblk, int S, const double *__restrict__ dk_blk, double *__restrict__ dk) {
    const int ab = threadIdx.x;
    if (ab >= S * S) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += dk_blk[(size_t)b * S * S + ab];
    dk[ab] = s;
}

// Adjoint pair sum over one tile: for each i of the tile and the chunk's
// species b, M = sum_j J(u_ij) and v = sum_j J(u_ij) lambda*_j, then
// gpart = K[s_i][b] M lambda*_i - K[b][s_i] v.
template <int P, bool SELF>
__device__ __forceinline__ void adj_range(const double4 *__restrict__ pj4, int j0, int j1, int ib,
                                          const double (&xi)[P], const double (&yi)[P], double (&mxx)[P],
                                          double (&mxy)[P], double (&myy)[P], double (&vx)[P],
                                          double (&vy)[P]) {
    for (int j = j0; j < j1; ++j) {
        const double4 q = pj4[j];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            if (SELF && j == ib + k * kAdjBlock + (int)threadIdx.x) continue;
            const double ux = xi[k] - q.x, uy = yi[k] - q.y;
            const double d2 = ux * ux + uy * uy;
            // d^-1 from the hardware estimate y0, corrected with e = 1 - d2 y0^2:
            // y0 (1 - e)^-1/2 ~ y0 (1 + e/2 + 3/8 e^2), relative error O(e^3)
            const double y0 = __builtin_amdgcn_rsq(d2);
            const double e = fma(-d2, y0 * y0, 1.0);
            const double inv = y0 * fma(fma(0.375, e, 0.5), e, 1.0);
            const double inv2 = inv * inv;
            const double inv3 = inv2 * inv;
            const double c5 = 3.0 * inv3 * inv2;
            const double tx = c5 * ux, ty = c5 * uy;
            const double jxx = inv3 - tx * ux;
            const double jxy = -tx * uy;
            const double jyy = inv3 - ty * uy;
            mxx[k] += jxx;
            mxy[k] += jxy;
            myy[k] += jyy;
            vx[k] += jxx * q.z + jxy * q.w;
            vy[k] += jxy * q.z + jyy * q.w;
        }
    }
}

template <int P>
__global__ __launch_bounds__(kAdjBlock) void k_adj_pairs(const double4 *__restrict__ pj4,
                                                         const int *__restrict__ sps, const Tile *__restrict__ tiles,
                                                         const double *__restrict__ K, int S,
                                                         double2 *__restrict__ gpart) {
    const Tile tl = tiles[blockIdx.x];
    const int ib = tl.i0;
    double xi[P], yi[P], mxx[P], mxy[P], myy[P], vx[P], vy[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const int i = ib + k * kAdjBlock + threadIdx.x;
        const double4 v = pj4[i < tl.i1 ? i : tl.i1 - 1];
        xi[k] = v.x;
        yi[k] = v.y;
        mxx[k] = mxy[k] = myy[k] = vx[k] = vy[k] = 0.0;
    }
    const int lo = tl.js > ib ? tl.js : ib;
    const int hi = tl.je < tl.i1 ? tl.je : tl.i1;
    if (lo < hi) {
        adj_range<P, false>(pj4, tl.js, lo, ib, xi, yi, mxx, mxy, myy, vx, vy);
        adj_range<P, true>(pj4, lo, hi, ib, xi, yi, mxx, mxy, myy, vx, vy);
        adj_range<P, false>(pj4, hi, tl.je, ib, xi, yi, mxx, mxy, myy, vx, vy);
    } else {
        adj_range<P, false>(pj4, tl.js, tl.je, ib, xi, yi, mxx, mxy, myy, vx, vy);
    }
    const int b = sps[tl.js];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const int i = ib + k * kAdjBlock + threadIdx.x;
        if (i < tl.i1) {
            const double4 v = pj4[i];
            const int si = sps[i];
            const double kab = K[si * S + b], kba = K[b * S + si];
            const double gx = kab * (mxx[k] * v.z + mxy[k] * v.w) - kba * vx[k];
            const double gy = kab * (mxy[k] * v.z + myy[k] * v.w) - kba * vy[k];
            gpart[tl.pbase + i] = make_double2(gx, gy);
        }
    }
}

// lambda = lambda* + dt g, g reduced over the particle's chunks in a fixed order.
__global__ void k_adj_update(int n, const double2 *__restrict__ gpart, const RepInfo *__restrict__ reps,
                             const int *__restrict__ rep_of, const int *__restrict__ pos_of, double dt,
                             double2 *__restrict__ lam) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const RepInfo ri = reps[rep_of[i]];
    const long long row = ri.poff + (pos_of[i] - ri.off);
    double gx = 0.0, gy = 0.0;
    for (int c = 0; c < ri.nch; ++c) {
        const double2 g = gpart[row + (long long)c * ri.n];
        gx += g.x;
        gy += g.y;
    }
    const double2 l = lam[i];
    lam[i] = make_double2(l.x + dt * gx, l.y + dt * gy);
}

inline int nblocks(long long n) { return (int)((n + kAdjBlock - 1) / kAdjBlock); }

}  // namespace

void launch_adj_round(Sim &s, int first_entry, int count) {
    if (count <= 0) return;
    const Tape &tp = s.adj.tape;
    AdjState &a = s.adj;
    hipLaunchKernelGGL(k_adj_round_prep, dim3(nblocks(count)), dim3(kAdjBlock), 0, s.stream, first_entry, count,
                       tp.ev, tp.eold, tp.edisp, tp.ewf, s.rad, s.p.cap_frac, a.lam, a.nu, a.bx, a.by);
    hipLaunchKernelGGL(k_adj_round_apply, dim3(nblocks(count)), dim3(kAdjBlock), 0, s.stream, first_entry, count,
                       tp.ev, tp.ewf, tp.ecnt, tp.enb, s.rad, s.p.overlap_factor, a.nu, a.bx, a.by, a.lam);
}

void launch_adj_step(Sim &s, int t) {
    const Tape &tp = s.adj.tape;
    AdjState &a = s.adj;
    const int nb = nblocks(s.n);
    hipLaunchKernelGGL(k_adj_em_slopes, dim3(nb), dim3(kAdjBlock), 0, s.stream, s.n,
                       tp.emwf + (size_t)t * 2 * s.n, a.lam);
    const double *px = tp.px + (size_t)t * s.n, *py = tp.py + (size_t)t * s.n;
    if (s.fp32)
        hipLaunchKernelGGL(k_adj_cast<float2>, dim3(nb), dim3(kAdjBlock), 0, s.stream, s.n, px, py, a.lam,
                           s.sorted_id, a.pj4, (float2 *)s.pj);
    else
        hipLaunchKernelGGL(k_adj_cast<double2>, dim3(nb), dim3(kAdjBlock), 0, s.stream, s.n, px, py, a.lam,
                           s.sorted_id, a.pj4, (double2 *)s.pj);
    // Phi at the positions before the step: kept by the replay, else recomputed
    const size_t vec = s.fp32 ? sizeof(float2) : sizeof(double2);
    const void *phi = tp.phi ? (const char *)tp.phi + (size_t)t * s.part_cap * vec : s.part;
    if (!tp.phi) launch_force(s);
    if (s.fp32)
        hipLaunchKernelGGL(k_adj_dk_rows<float2>, dim3(nb), dim3(kAdjBlock), 0, s.stream, s.n, s.S,
                           (const float2 *)phi, s.reps, s.rep_of, s.chunk_spec, s.pos_of, a.lam, s.p.dt,
                           a.dk_rows);
    else
        hipLaunchKernelGGL(k_adj_dk_rows<double2>, dim3(nb), dim3(kAdjBlock), 0, s.stream, s.n, s.S,
                           (const double2 *)phi, s.reps, s.rep_of, s.chunk_spec, s.pos_of, a.lam, s.p.dt,
                           a.dk_rows);
    hipLaunchKernelGGL(k_adj_dk_blocks, dim3(nblocks((long long)a.dk_blocks * s.S * s.S)), dim3(kAdjBlock), 0,
                       s.stream, s.n, s.S, a.dk_blocks, s.sp, a.dk_rows, a.dk_blk);
    if (s.per_lane == 2)
        hipLaunchKernelGGL(k_adj_pairs<2>, dim3(s.ntiles), dim3(kAdjBlock), 0, s.stream, a.pj4, s.sp_sorted, s.tiles,
                           s.Kd, s.S, a.gpart);
    else
        hipLaunchKernelGGL(k_adj_pairs<4>, dim3(s.ntiles), dim3(kAdjBlock), 0, s.stream, a.pj4, s.sp_sorted, s.tiles,
                           s.Kd, s.S, a.gpart);
    hipLaunchKernelGGL(k_adj_update, dim3(nb), dim3(kAdjBlock), 0, s.stream, s.n, a.gpart, s.reps, s.rep_of,
                       s.pos_of, s.p.dt, a.lam);
}

void launch_adj_dk_final(Sim &s) {
    hipLaunchKernelGGL(k_adj_dk_final, dim3(1), dim3(64), 0, s.stream, s.adj.dk_blocks, s.S, s.adj.dk_blk,
                       s.adj.dk);
}

}  // namespace bd
