// Per-particle kernels of the time step: the all-pairs force (Sec. 2.2,
// Sec. 4.1 "one thread per particle, no symmetry used"), the Euler-Maruyama
// move with Brownian noise and self-propulsion (Sec. 2.2, 2.4, 7) and hard
// walls.
//
// Force layout.  Inside each system the particles are permuted once so that
// species are contiguous ("sorted order").  A system's j range is cut into
// chunks that never straddle a species boundary; one workgroup handles one
// tile (a block of 256*P particles i of one system against one chunk of the
// same system) and writes the unweighted sum
// Phi_{i,c} = sum_{j in chunk c} (r_i - r_j)/d^3.  Tiles of all systems form one
// launch, longest first.  The update kernel then forms
// F_i = sum_c K[s_i][spec(c)] Phi_{i,c} in FP64 in a fixed chunk order
// (deterministic, no atomics).  Inside the j loop every lane of the wavefront
// needs the same j, so j positions are wave-uniform loads (scalar data cache)
// and the VALU only sees the pair arithmetic.
#include <hip/hip_runtime.h>

#include "bd_internal.h"
#include "geom.h"

namespace bd {
namespace {

constexpr int kForceBlock = 256;
constexpr int kPerLane = 4;   // particles i per lane (register blocking)

// ---------------------------------------------------------------- cast
template <typename T2>
__global__ void k_cast(int n, const double *__restrict__ x, const double *__restrict__ y,
                       const int *__restrict__ sorted_id, T2 *__restrict__ pj, const StepBase *__restrict__ base) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n || base->stop) return;
    int i = sorted_id[k];
    T2 v;
    v.x = x[i];
    v.y = y[i];
    pj[k] = v;
}

__global__ void k_pack_xy(int m, const double *__restrict__ x, const double *__restrict__ y,
                          double2 *__restrict__ xy) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) xy[i] = make_double2(x[i], y[i]);
}

// ---------------------------------------------------------------- forces
// d^-3 from d^2.  FP32: the hardware reciprocal square root (v_rsq_f32, ~1 ulp)
// cubed.  FP64: the hardware estimate y0 of d2^-1/2 corrected with
// e = 1 - d2 y0^2 as y0^3 (1 - e)^-3/2 ~ y0^3 (1 + 3/2 e + 15/8 e^2), which
// leaves a relative error of order e^3 (far below FP64 rounding for any
// estimate better than 2^-20) without the special-case handling of the
// library rsqrt; d2 is always positive and finite here.
template <typename T>
__device__ __forceinline__ T inv_cube(T d2);
template <>
__device__ __forceinline__ float inv_cube<float>(float d2) {
    const float r = __builtin_amdgcn_rsqf(d2);
    return r * r * r;
}
template <>
__device__ __forceinline__ double inv_cube<double>(double d2) {
    const double y = __builtin_amdgcn_rsq(d2);
    const double y2 = y * y;
    const double e = fma(-d2, y2, 1.0);
    const double c = fma(fma(1.875, e, 1.5), e, 1.0);
    return (y2 * y) * c;
}

template <typename T>
__device__ __forceinline__ T self_floor();
template <>
__device__ __forceinline__ float self_floor<float>() { return 1e-20f; }
template <>
__device__ __forceinline__ double self_floor<double>() { return 1e-200; }

// Inverse-square law (q = 2, all pairs): Phi += (r_i - r_j) / d^3.
// SELF: the range may contain i itself; d^2 is floored so the self term is 0.
// PER: periodic box of side per (inv_per = 1 / per): separations from the nearest image.
template <typename T, bool PER>
__device__ __forceinline__ T near_image(T v, T per, T inv_per) {
    return PER ? v - per * rint(v * inv_per) : v;
}

template <typename T, typename T2, int P, bool SELF, bool PER = false>
__device__ __forceinline__ void pair_range_q2(const T2 *__restrict__ pj, int j0, int j1, const T (&xi)[P],
                                              const T (&yi)[P], T (&ax)[P], T (&ay)[P], T per = (T)0,
                                              T inv_per = (T)0) {
#pragma unroll 8
    for (int j = j0; j < j1; ++j) {
        const T2 q = pj[j];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            T dx = near_image<T, PER>(xi[k] - q.x, per, inv_per);
            T dy = near_image<T, PER>(yi[k] - q.y, per, inv_per);
            T d2 = dx * dx + dy * dy;
            if (SELF) d2 = d2 > self_floor<T>() ? d2 : self_floor<T>();
            T inv3 = inv_cube<T>(d2);
            ax[k] += dx * inv3;
            ay[k] += dy * inv3;
        }
    }
}

// General law: power d^-q or screened A exp(-d/lam)/d, optional inclusive cutoff.
struct LawArgs {
    int kind;
    double q, A, lam, cutoff;
    double period;   // > 0: periodic box (minimum-image separations)
};

template <typename T, typename T2, int P, bool PER = false>
__device__ __forceinline__ void pair_range_general(const T2 *__restrict__ pj, int j0, int j1, const T (&xi)[P],
                                                   const T (&yi)[P], T (&ax)[P], T (&ay)[P], const LawArgs law) {
    const T per = (T)law.period, inv_per = PER ? (T)(1.0 / law.period) : (T)0;
    const T cut2 = law.cutoff > 0.0 ? (T)(law.cutoff * law.cutoff) : (T)0;
    const T expo = (T)(-0.5 * (law.q + 1.0));
    const T invlam = (T)(1.0 / law.lam);
    const T A = (T)law.A;
    for (int j = j0; j < j1; ++j) {
        const T2 q = pj[j];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            T dx = near_image<T, PER>(xi[k] - q.x, per, inv_per);
            T dy = near_image<T, PER>(yi[k] - q.y, per, inv_per);
            T d2 = dx * dx + dy * dy;
            bool ok = d2 > (T)0 && (cut2 == (T)0 || d2 <= cut2);
            T dd = ok ? d2 : (T)1;
            T s;
            if (law.kind == BD_FORCE_POWER) {
                s = pow(dd, expo);
            } else {
                T d = sqrt(dd);
                s = A * exp(-d * invlam) / dd;
            }
            s = ok ? s : (T)0;
            ax[k] += dx * s;
            ay[k] += dy * s;
        }
    }
}

template <typename T, typename T2, int P, bool FAST, bool PER = false>
__device__ __forceinline__ void force_tile(const T2 *__restrict__ pj, const Tile &tl, T2 *__restrict__ part,
                                           const LawArgs &law) {
    const T per = (T)law.period, inv_per = PER ? (T)(1.0 / law.period) : (T)0;
    const int ib = tl.i0;
    T xi[P], yi[P], ax[P], ay[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        int i = ib + k * kForceBlock + threadIdx.x;
        T2 v = pj[i < tl.i1 ? i : tl.i1 - 1];
        xi[k] = v.x;
        yi[k] = v.y;
        ax[k] = (T)0;
        ay[k] = (T)0;
    }
    if (FAST) {
        // self range: the workgroup's own particles inside this chunk
        int lo = tl.js > ib ? tl.js : ib;
        int hi = tl.je < tl.i1 ? tl.je : tl.i1;
        if (lo < hi) {
            pair_range_q2<T, T2, P, false, PER>(pj, tl.js, lo, xi, yi, ax, ay, per, inv_per);
            pair_range_q2<T, T2, P, true, PER>(pj, lo, hi, xi, yi, ax, ay, per, inv_per);
            pair_range_q2<T, T2, P, false, PER>(pj, hi, tl.je, xi, yi, ax, ay, per, inv_per);
        } else {
            pair_range_q2<T, T2, P, false, PER>(pj, tl.js, tl.je, xi, yi, ax, ay, per, inv_per);
        }
    } else {
        pair_range_general<T, T2, P, PER>(pj, tl.js, tl.je, xi, yi, ax, ay, law);
    }
#pragma unroll
    for (int k = 0; k < P; ++k) {
        int i = ib + k * kForceBlock + threadIdx.x;
        if (i < tl.i1) {
            T2 v;
            v.x = ax[k];
            v.y = ay[k];
            part[tl.pbase + i] = v;
        }
    }
}

// One workgroup per tile.  PER: periodic box (law.period > 0).
template <typename T, typename T2, int P, bool FAST, bool PER = false>
__global__ __launch_bounds__(kForceBlock) void k_force(const T2 *__restrict__ pj, const Tile *__restrict__ tiles,
                                                       T2 *__restrict__ part, LawArgs law,
                                                       const StepBase *__restrict__ base) {
    if (base->stop) return;
    force_tile<T, T2, P, FAST, PER>(pj, tiles[blockIdx.x], part, law);
}

// LDS form (the shared-memory broadcast of the paper's n-body kernel, Sec. 6):
// the workgroup stages the chunk's j positions in LDS, kLdsJ at a time, and
// every lane reads the same j from there, instead of wave-uniform scalar
// loads.  Same tiles, same j order and the same pair arithmetic as k_force,
// so the partial sums are bitwise those of k_force (the self floor only
// changes a pair with d^2 below 1e-20, i.e. i itself).
constexpr int kLdsJ = 1024;

template <typename T, typename T2, int P, bool SELF>
__device__ __forceinline__ void pair_block_lds(const T2 *__restrict__ sj, int m, const T (&xi)[P], const T (&yi)[P],
                                               T (&ax)[P], T (&ay)[P]) {
#pragma unroll 8
    for (int k = 0; k < m; ++k) {
        const T2 q = sj[k];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            T dx = xi[p] - q.x;
            T dy = yi[p] - q.y;
            T d2 = dx * dx + dy * dy;
            if (SELF) d2 = d2 > self_floor<T>() ? d2 : self_floor<T>();
            T inv3 = inv_cube<T>(d2);
            ax[p] += dx * inv3;
            ay[p] += dy * inv3;
        }
    }
}

template <typename T, typename T2, int P>
__global__ __launch_bounds__(kForceBlock) void k_force_lds(const T2 *__restrict__ pj, const Tile *__restrict__ tiles,
                                                           T2 *__restrict__ part, const StepBase *__restrict__ base) {
    __shared__ T2 sj[kLdsJ];
    if (base->stop) return;
    const Tile tl = tiles[blockIdx.x];
    const int ib = tl.i0;
    T xi[P], yi[P], ax[P], ay[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        int i = ib + k * kForceBlock + threadIdx.x;
        T2 v = pj[i < tl.i1 ? i : tl.i1 - 1];
        xi[k] = v.x;
        yi[k] = v.y;
        ax[k] = (T)0;
        ay[k] = (T)0;
    }
    for (int jb = tl.js; jb < tl.je; jb += kLdsJ) {
        const int m = min(kLdsJ, tl.je - jb);
        __syncthreads();   // every lane is done with the previous block
        for (int k = threadIdx.x; k < m; k += kForceBlock) sj[k] = pj[jb + k];
        __syncthreads();
        // a block that meets the workgroup's own particles floors d^2 (the self term adds 0)
        if (jb < tl.i1 && jb + m > ib)
            pair_block_lds<T, T2, P, true>(sj, m, xi, yi, ax, ay);
        else
            pair_block_lds<T, T2, P, false>(sj, m, xi, yi, ax, ay);
    }
#pragma unroll
    for (int k = 0; k < P; ++k) {
        int i = ib + k * kForceBlock + threadIdx.x;
        if (i < tl.i1) {
            T2 v;
            v.x = ax[k];
            v.y = ay[k];
            part[tl.pbase + i] = v;
        }
    }
}

// Persistent form: a grid sized to the resident workgroups takes tiles from
// a queue (tile list longest first) until it is empty.  The queue counter is
// zeroed before the launch; every workgroup leaves once the counter passes
// the number of tiles.
template <typename T, typename T2, int P, bool FAST>
__global__ __launch_bounds__(kForceBlock) void k_force_queue(const T2 *__restrict__ pj,
                                                             const Tile *__restrict__ tiles, int ntiles,
                                                             T2 *__restrict__ part, LawArgs law,
                                                             int *__restrict__ queue,
                                                             const StepBase *__restrict__ base) {
    __shared__ int next;
    if (base->stop) return;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(queue, 1);
        __syncthreads();
        const int t = next;
        __syncthreads();
        if (t >= ntiles) return;
        force_tile<T, T2, P, FAST>(pj, tiles[t], part, law);
    }
}

// Symmetric form (inverse-square law).  A tile is a pair of chunks A, B of
// one system (at most 256 P disks each): each of the 4 wavefronts owns up to
// 64 P particles i of A, P per lane, in registers.  The particles j of B pass through the wavefront in
// groups of 128 (2 per lane); a group turns around the wavefront one lane per
// step (DPP wave_rol: lane l takes lane l+1's values) for 64 steps, so every
// lane meets every j of the group once.  g = (r_i - r_j)/d^3 is added to i's
// sum and subtracted from j's sum, which travels with j; after the 64 steps
// each j is back in its lane and the wavefront leaves its sums in LDS.  At the
// end the 4 wavefronts' sums are added in wavefront order (deterministic) and
// written for B's particles (slot of chunk A).  A chunk paired with itself
// (j0 == i0) takes i's side only, with d^2 floored so that i == j adds 0.
// Padding i (j) sit at +BIG (-BIG): their g underflow to exactly 0.
template <typename T>
__device__ __forceinline__ T rot1(T v);
template <>
__device__ __forceinline__ float rot1<float>(float v) {   // every lane has a source: no old value needed
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x134, 0xF, 0xF, true));
}
template <>
__device__ __forceinline__ double rot1<double>(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0x134, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x134, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <typename T>
__device__ __forceinline__ T sym_big();
template <>
__device__ __forceinline__ float sym_big<float>() { return 1e18f; }   // (2e18)^2 finite, (1e18)^-3 underflows
template <>
__device__ __forceinline__ double sym_big<double>() { return 1e150; }

constexpr int kSymQ = 2;

// The 64 steps of one group of j (every lane active: the rotation reads all lanes).
template <typename T, int P, bool SELF>
__device__ __forceinline__ void sym_group(const T (&xi)[P], const T (&yi)[P], T (&fx)[P], T (&fy)[P],
                                          T (&xj)[kSymQ], T (&yj)[kSymQ], T (&gx)[kSymQ], T (&gy)[kSymQ]) {
    for (int t = 0; t < 64; ++t) {
#pragma unroll
        for (int q = 0; q < kSymQ; ++q) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const T dx = xi[p] - xj[q];
                const T dy = yi[p] - yj[q];
                T d2 = dx * dx + dy * dy;
                if (SELF) d2 = d2 > self_floor<T>() ? d2 : self_floor<T>();
                const T inv3 = inv_cube<T>(d2);
                const T ex = dx * inv3, ey = dy * inv3;
                fx[p] += ex;
                fy[p] += ey;
                gx[q] -= ex;
                gy[q] -= ey;
            }
            xj[q] = rot1(xj[q]);
            yj[q] = rot1(yj[q]);
            gx[q] = rot1(gx[q]);
            gy[q] = rot1(gy[q]);
        }
    }
}

// W wavefronts per workgroup; a chunk holds at most 64 W P disks.
template <typename T, typename T2, int P, int W>
__global__ __launch_bounds__(64 * W) void k_force_sym(const T2 *__restrict__ pj, const SymTile *__restrict__ tiles,
                                                      T2 *__restrict__ part, const StepBase *__restrict__ base) {
    constexpr int kSymP = P;
    __shared__ T2 jsum[W][64 * W * P];
    if (base->stop) return;
    const SymTile tl = tiles[blockIdx.x];
    const bool self = tl.j0 == tl.i0;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ni = tl.i1 - tl.i0, nj = tl.j1 - tl.j0;
    const T big = sym_big<T>();
    T xi[kSymP], yi[kSymP], fx[kSymP], fy[kSymP];
#pragma unroll
    for (int p = 0; p < kSymP; ++p) {
        const int k = wave * 64 * kSymP + p * 64 + lane;
        const T2 v = pj[tl.i0 + (k < ni ? k : 0)];
        xi[p] = k < ni ? v.x : big;
        yi[p] = k < ni ? v.y : big;
        fx[p] = (T)0;
        fy[p] = (T)0;
    }
    for (int jg = 0; jg < nj; jg += 64 * kSymQ) {   // same trip count in every lane
        T xj[kSymQ], yj[kSymQ], gx[kSymQ], gy[kSymQ];
#pragma unroll
        for (int q = 0; q < kSymQ; ++q) {
            const int k = jg + q * 64 + lane;
            const T2 v = pj[tl.j0 + (k < nj ? k : 0)];
            xj[q] = k < nj ? v.x : -big;
            yj[q] = k < nj ? v.y : -big;
            gx[q] = (T)0;
            gy[q] = (T)0;
        }
        if (self)
            sym_group<T, P, true>(xi, yi, fx, fy, xj, yj, gx, gy);
        else
            sym_group<T, P, false>(xi, yi, fx, fy, xj, yj, gx, gy);
        if (!self) {
#pragma unroll
            for (int q = 0; q < kSymQ; ++q) {
                const int k = jg + q * 64 + lane;
                if (k < nj) {
                    T2 g;
                    g.x = gx[q];
                    g.y = gy[q];
                    jsum[wave][k] = g;
                }
            }
        }
    }
#pragma unroll
    for (int p = 0; p < kSymP; ++p) {
        const int k = wave * 64 * kSymP + p * 64 + lane;
        if (k < ni) {
            T2 v;
            v.x = fx[p];
            v.y = fy[p];
            part[tl.pbase_i + tl.i0 + k] = v;
        }
    }
    if (self) return;   // uniform in the workgroup
    __syncthreads();
    for (int k = threadIdx.x; k < nj; k += 64 * W) {
        T2 a = jsum[0][k];
#pragma unroll
        for (int w = 1; w < W; ++w) {
            a.x += jsum[w][k].x;
            a.y += jsum[w][k].y;
        }
        part[tl.pbase_j + tl.j0 + k] = a;
    }
}

// F_i = sum_c K[s_i][spec(c)] Phi_{i,c} over the chunks of i's system, FP64,
// fixed chunk order; k is i's sorted index.
template <typename T2>
__device__ __forceinline__ void gather_force(const T2 *__restrict__ part, const RepInfo &ri,
                                             const int *__restrict__ chunk_spec, const double *__restrict__ K,
                                             int S, int si, int k, double &fx, double &fy) {
    fx = 0.0;
    fy = 0.0;
    const long long row = ri.poff + (k - ri.off);
    const double *Ki = K + si * S;
    int c = 0;
    // 16 chunks at a time: the loads are all issued before the sums, which keep the chunk order (one
    // particle per thread, so the loads in flight per thread set how much of the latency is hidden)
    constexpr int kB = 16;
    for (; c + kB <= ri.nch; c += kB) {
        T2 v[kB];
        double w[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            v[u] = part[row + (long long)(c + u) * ri.n];
            w[u] = Ki[chunk_spec[ri.cfirst + c + u]];
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            fx += w[u] * (double)v[u].x;
            fy += w[u] * (double)v[u].y;
        }
    }
    for (; c < ri.nch; ++c) {
        const double w = Ki[chunk_spec[ri.cfirst + c]];
        const T2 v = part[row + (long long)c * ri.n];
        fx += w * (double)v.x;
        fy += w * (double)v.y;
    }
}

// ---------------------------------------------------------------- noise
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// multiplies whose high halves are mixed with the other counter words and the
// round key; the two key words advance by fixed Weyl constants between rounds.
__device__ __forceinline__ uint4 philox10(uint4 c, uint2 k) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const unsigned m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
        unsigned lo0 = m0 * c.x, hi0 = __umulhi(m0, c.x);
        unsigned lo1 = m1 * c.z, hi1 = __umulhi(m1, c.z);
        c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
        k.x += 0x9E3779B9u;
        k.y += 0xBB67AE85u;
    }
    return c;
}

// Box-Muller (1958) on two 53-bit uniforms: u1 in (0, 1], u2 in [0, 1).
__device__ __forceinline__ void box_muller(uint4 w, double &z0, double &z1) {
#pragma clang fp contract(off)
    unsigned long long m1 = ((((unsigned long long)w.x) << 32) | w.y) >> 11;
    unsigned long long m2 = ((((unsigned long long)w.z) << 32) | w.w) >> 11;
    double u1 = ((double)m1 + 1.0) * 0x1.0p-53;
    double u2 = (double)m2 * 0x1.0p-53;
    double rho = sqrt(-2.0 * log(u1));
    double ang = 2.0 * M_PI * u2;
    z0 = rho * cos(ang);
    z1 = rho * sin(ang);
}

// The first of the two normals of box_muller alone (same operations, same value).
__device__ __forceinline__ double box_muller_first(uint4 w) {
#pragma clang fp contract(off)
    unsigned long long m1 = ((((unsigned long long)w.x) << 32) | w.y) >> 11;
    unsigned long long m2 = ((((unsigned long long)w.z) << 32) | w.w) >> 11;
    double u1 = ((double)m1 + 1.0) * 0x1.0p-53;
    double u2 = (double)m2 * 0x1.0p-53;
    double rho = sqrt(-2.0 * log(u1));
    double ang = 2.0 * M_PI * u2;
    return rho * cos(ang);
}

struct EmArgs {
    int n, S;
    double dt, amp, amp_r, v0, clip;
    double D, Dr;          // for the bridge amplitudes of a sub-interval
    int level;             // 0: the whole step; > 0: sub-interval `index` of 2^level after reversals (Sec. 4.3)
    unsigned index;
    int periodic;          // fold into the periodic box [0, L)^2 instead of reflecting at the walls
};

// Fused Euler-Maruyama update: gather forces, draw noise (stream 0:
// translation, stream 1: rotation), move, reflect at the walls, keep the
// previous state for the reversal check and for error rollback.
// DIRECT: the forces come in fdirect (the list force), else as partial sums to reduce with K.
// BRIDGE: a sub-interval of a halved step (level > 0); the bridge draws hold about twice the registers
// of the rest, so the whole steps (level 0) run an instance without them at twice the waves per SIMD.
template <typename T2, bool DIRECT, bool BRIDGE>
__global__ __launch_bounds__(256) void k_em(EmArgs a, const StepBase *__restrict__ base, const T2 *__restrict__ part,
                                            const RepInfo *__restrict__ reps,
                                            const int *__restrict__ rep_of, const int *__restrict__ chunk_spec,
                                            const double *__restrict__ K, const int *__restrict__ pos_of,
                                            const int *__restrict__ key_id,
                                            const int *__restrict__ sp, const double *__restrict__ rad,
                                            double *__restrict__ x, double *__restrict__ y,
                                            double2 *__restrict__ xy,
                                            double *__restrict__ xo, double *__restrict__ yo,
                                            double *__restrict__ th, double *__restrict__ tho,
                                            unsigned long long *__restrict__ acc, const double2 *__restrict__ fdirect,
                                            signed char *__restrict__ wf, const int *__restrict__ ctl) {
#pragma clang fp contract(off)
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int clamps = 0;
    if (base->stop || ctl[K_HALT]) return;   // K_HALT this early: the step's neighbour lists overflowed
    if (i < a.n) {
        const RepInfo ri = reps[rep_of[i]];
        double fx, fy;
        if (DIRECT) {
            fx = fdirect[i].x;
            fy = fdirect[i].y;
        } else {
            gather_force<T2>(part, ri, chunk_spec, K, a.S, sp[i], pos_of[i], fx, fy);
        }
        // noise keyed by the system's seed and the caller's index of the disk inside its system
        const unsigned id = (unsigned)key_id[i];
        const unsigned long long step = (unsigned long long)base->step;
        const unsigned slo = (unsigned)step;
        const unsigned shi = (unsigned)(step >> 32);
        const uint2 key = make_uint2((unsigned)ri.seed, (unsigned)(ri.seed >> 32));
        // without rotational diffusion (Dr = 0) the angle never changes and its draw is not needed;
        // without self-propulsion (v0 = 0) the angle does not enter the move
        const bool rot = a.Dr != 0.0;
        double zx, zy;
        box_muller(philox10(make_uint4(id, slo, shi, 0u), key), zx, zy);
        const double nr = rot ? box_muller_first(philox10(make_uint4(id, slo, shi, 1u), key)) : 0.0;
        if (zx > a.clip) { zx = a.clip; ++clamps; }
        if (zx < -a.clip) { zx = -a.clip; ++clamps; }
        if (zy > a.clip) { zy = a.clip; ++clamps; }
        if (zy < -a.clip) { zy = -a.clip; ++clamps; }
        // noise increments of the step, then down the Brownian bridge to the sub-interval: the
        // increment over the first half of an interval of length h with increment w is
        // w/2 + sqrt(D h / 2) eta (eta keyed by the level of the halves and the parent's index,
        // clamped like xi), the second half takes the rest
        double wx = a.amp * zx, wy = a.amp * zy, wt = a.amp_r * nr;
        double hsub = a.dt;
        for (int lv = 1; BRIDGE && lv <= a.level; ++lv) {
            const unsigned par = a.index >> (a.level - lv + 1), side = (a.index >> (a.level - lv)) & 1u;
            const unsigned skey = 0x80000000u | ((unsigned)lv << 24) | (par << 1);
            double ex, ey;
            box_muller(philox10(make_uint4(id, slo, shi, skey), key), ex, ey);
            const double er = rot ? box_muller_first(philox10(make_uint4(id, slo, shi, skey | 1u), key)) : 0.0;
            ex = ex > a.clip ? a.clip : (ex < -a.clip ? -a.clip : ex);
            ey = ey > a.clip ? a.clip : (ey < -a.clip ? -a.clip : ey);
            const double at = sqrt(0.5 * a.D * hsub), ar = sqrt(0.5 * a.Dr * hsub);
            const double lx = 0.5 * wx + at * ex, ly = 0.5 * wy + at * ey, lt = 0.5 * wt + ar * er;
            wx = side ? wx - lx : lx;
            wy = side ? wy - ly : ly;
            wt = side ? wt - lt : lt;
            hsub = 0.5 * hsub;
        }
        if (a.level > 0) clamps = 0;   // the step's own draws were counted when it was first tried
        const bool angle = rot || a.v0 != 0.0;
        const double2 p0 = xy[i];   // the packed copy: a writer that missed it would show in every later state
        const double x0 = p0.x, y0 = p0.y, t0 = angle ? th[i] : 0.0, r = rad[i];
        const double vx = a.v0 != 0.0 ? fx + a.v0 * cos(t0) : fx;
        const double vy = a.v0 != 0.0 ? fy + a.v0 * sin(t0) : fy;
        const double xn = x0 + vx * hsub + wx;
        const double yn = y0 + vy * hsub + wy;
        xo[i] = x0;
        yo[i] = y0;
        if (rot) tho[i] = t0;
        const double xw = a.periodic ? bd_wrap(xn, ri.L) : bd_wall(xn, r, ri.L);
        const double yw = a.periodic ? bd_wrap(yn, ri.L) : bd_wall(yn, r, ri.L);
        x[i] = xw;
        y[i] = yw;
        xy[i] = make_double2(xw, yw);
        if (wf) {   // adjoint tape: wall slopes of this move
            wf[2 * (size_t)i] = bd_wall_slope(xn, r, ri.L);
            wf[2 * (size_t)i + 1] = bd_wall_slope(yn, r, ri.L);
        }
        if (rot) th[i] = t0 + wt;
    }
    // one atomic per workgroup (every thread is here), on the workgroup's clamp slot
    __shared__ int wg_clamps;
    if (threadIdx.x == 0) wg_clamps = 0;
    for (int off = 32; off > 0; off >>= 1) clamps += __shfl_xor(clamps, off);
    __syncthreads();
    if (__lane_id() == 0 && clamps) atomicAdd(&wg_clamps, clamps);
    __syncthreads();
    if (threadIdx.x == 0 && wg_clamps)
        atomicAdd(&acc[A_CLAMP_BASE + (blockIdx.x % A_CLAMP_SLOTS) * A_CLAMP_STRIDE], (unsigned long long)wg_clamps);
}

template <typename T2>
__global__ void k_reduce_forces(int n, int S, const T2 *__restrict__ part, const RepInfo *__restrict__ reps,
                                const int *__restrict__ rep_of, const int *__restrict__ chunk_spec,
                                const double *__restrict__ K, const int *__restrict__ pos_of,
                                const int *__restrict__ sp, double *__restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double fx, fy;
    gather_force<T2>(part, reps[rep_of[i]], chunk_spec, K, S, sp[i], pos_of[i], fx, fy);
    out[2 * i] = fx;
    out[2 * i + 1] = fy;
}

inline int blocks_for(int n, int b) { return (n + b - 1) / b; }

__global__ void k_zero_one(int *p) {
    if (threadIdx.x == 0) *p = 0;
}

__device__ __forceinline__ void step_begin_body(int *__restrict__ ctl, StepBase *__restrict__ base) {
    if (base->stop) {   // keep the halted step's control block for the host; no list rebuild
        if (threadIdx.x == 0) base->nl_now = 0;
        return;
    }
    for (int i = threadIdx.x; i < N_CTL; i += blockDim.x) ctl[i] = 0;
    if (threadIdx.x == 0) {   // a rebuild the last step's skin test asked for happens in this step
        base->nl_now = base->nl_req;
        base->nl_req = 0;
    }
}

__global__ void k_step_begin(int *__restrict__ ctl, StepBase *__restrict__ base) { step_begin_body(ctl, base); }

// The step's start and the cast in one launch (all-pairs path): workgroup 0 also clears the control
// block.  Nothing in the cast reads what the clear writes (the control block, the list flags), and
// the stop flag both read is not written here.
template <typename T2>
__global__ void k_step_begin_cast(int *__restrict__ ctl, StepBase *__restrict__ base, int n,
                                  const double *__restrict__ x, const double *__restrict__ y,
                                  const int *__restrict__ sorted_id, T2 *__restrict__ pj) {
    if (blockIdx.x == 0) step_begin_body(ctl, base);
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n || base->stop) return;
    const int i = sorted_id[k];
    T2 v;
    v.x = x[i];
    v.y = y[i];
    pj[k] = v;
}

// End of a queued step, one workgroup: record its control block in the ring,
// then (after a barrier: every thread has read the step base) either advance
// the step counter and the stamp bases, or stop the batch when the step halted
// (the host finishes it) or the ring is full.
__global__ void k_step_end(const int *__restrict__ ctl, StepBase *__restrict__ base, int *__restrict__ ring,
                           int r_used, int v_used) {
    if (base->stop) return;   // uniform: written by this kernel only after the barrier below
    const int idx = base->batch_idx;
    for (int i = threadIdx.x; i < N_CTL; i += blockDim.x) ring[(size_t)idx * N_CTL + i] = ctl[i];
    __syncthreads();
    if (threadIdx.x != 0) return;
    if (ctl[K_HALT]) {
        base->stop = 1;
        return;
    }
    base->step += 1;
    base->rbase += r_used;
    base->vbase += v_used;
    base->batch_idx = idx + 1;
    if (idx + 1 >= kRing) base->stop = 2;
}

}  // namespace

void launch_step_begin(Sim &s) {
    hipLaunchKernelGGL(k_step_begin, dim3(1), dim3(256), 0, s.stream, s.ctl, s.dbase);
}

void launch_step_end(Sim &s, int r_used, int v_used) {
    hipLaunchKernelGGL(k_step_end, dim3(1), dim3(256), 0, s.stream, (const int *)s.ctl, s.dbase, s.ring, r_used,
                       v_used);
}

void launch_pack_xy(Sim &s, int m) {
    if (m > 0)
        hipLaunchKernelGGL(k_pack_xy, dim3(blocks_for(m, 256)), dim3(256), 0, s.stream, m, (const double *)s.x,
                           (const double *)s.y, s.xy);
}

void launch_step_begin_cast(Sim &s) {
    const int nb = blocks_for(s.n, 256);
    if (s.fp32)
        hipLaunchKernelGGL(k_step_begin_cast<float2>, dim3(nb), dim3(256), 0, s.stream, s.ctl, s.dbase, s.n,
                           (const double *)s.x, (const double *)s.y, (const int *)s.sorted_id, (float2 *)s.pj);
    else
        hipLaunchKernelGGL(k_step_begin_cast<double2>, dim3(nb), dim3(256), 0, s.stream, s.ctl, s.dbase, s.n,
                           (const double *)s.x, (const double *)s.y, (const int *)s.sorted_id, (double2 *)s.pj);
}

void launch_cast(Sim &s) {
    const int nb = blocks_for(s.n, 256);
    if (s.fp32)
        hipLaunchKernelGGL(k_cast<float2>, dim3(nb), dim3(256), 0, s.stream, s.n, s.x, s.y, s.sorted_id,
                           (float2 *)s.pj, (const StepBase *)s.dbase);
    else
        hipLaunchKernelGGL(k_cast<double2>, dim3(nb), dim3(256), 0, s.stream, s.n, s.x, s.y, s.sorted_id,
                           (double2 *)s.pj, (const StepBase *)s.dbase);
}

namespace {

template <typename T, typename T2, int P, bool FAST>
void launch_force_t(Sim &s, const LawArgs &law) {
    if (s.period > 0.0) {   // periodic box: one workgroup per tile, minimum-image separations
        hipLaunchKernelGGL((k_force<T, T2, P, FAST, true>), dim3(s.ntiles), dim3(kForceBlock), 0, s.stream,
                           (const T2 *)s.pj, s.tiles, (T2 *)s.part, law, s.dbase);
    } else if (FAST && s.persistent == 3) {   // j staged through LDS (inverse-square law)
        hipLaunchKernelGGL((k_force_lds<T, T2, P>), dim3(s.ntiles), dim3(kForceBlock), 0, s.stream,
                           (const T2 *)s.pj, s.tiles, (T2 *)s.part, s.dbase);
    } else if (s.persistent) {
        hipLaunchKernelGGL((k_force_queue<T, T2, P, FAST>), dim3(s.force_grid), dim3(kForceBlock), 0, s.stream,
                           (const T2 *)s.pj, s.tiles, s.ntiles, (T2 *)s.part, law, s.ctl + K_FQUEUE, s.dbase);
    } else {
        hipLaunchKernelGGL((k_force<T, T2, P, FAST>), dim3(s.ntiles), dim3(kForceBlock), 0, s.stream,
                           (const T2 *)s.pj, s.tiles, (T2 *)s.part, law, s.dbase);
    }
}

template <typename T, typename T2, int P>
void launch_force_p(Sim &s, const LawArgs &law) {
    if (s.kind_fast)
        launch_force_t<T, T2, P, true>(s, law);
    else
        launch_force_t<T, T2, P, false>(s, law);
}

template <typename T, typename T2, int P, bool FAST>
int max_grid_t() {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_force_queue<T, T2, P, FAST>, kForceBlock, 0) !=
            hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    return per_cu;
}

template <typename T, typename T2, int P>
int max_grid_p(bool fast) {
    return fast ? max_grid_t<T, T2, P, true>() : max_grid_t<T, T2, P, false>();
}

}  // namespace

// Tiles of 256 * per_lane particles; per_lane is 2 or 4.
void launch_force(Sim &s) {
    LawArgs law{s.fp.kind, s.fp.q, s.fp.A, s.fp.lambda, s.fp.cutoff, s.period};
    if (s.persistent == 2) {   // symmetric chunk pairs (the host builds them only for the inverse-square law)
        // per_lane 2 / 4: 4 wavefronts (chunks of 512 / 1024); 8: 2 wavefronts (chunks of 1024)
        const dim3 g(s.nstiles), b4(256), b2(128);
        const SymTile *st = s.stiles;
        const StepBase *base = s.dbase;
        if (s.fp32) {
            const float2 *pj = (const float2 *)s.pj;
            float2 *part = (float2 *)s.part;
            if (s.per_lane == 2)
                hipLaunchKernelGGL((k_force_sym<float, float2, 2, 4>), g, b4, 0, s.stream, pj, st, part, base);
            else if (s.per_lane == 4)
                hipLaunchKernelGGL((k_force_sym<float, float2, 4, 4>), g, b4, 0, s.stream, pj, st, part, base);
            else
                hipLaunchKernelGGL((k_force_sym<float, float2, 8, 2>), g, b2, 0, s.stream, pj, st, part, base);
        } else {
            const double2 *pj = (const double2 *)s.pj;
            double2 *part = (double2 *)s.part;
            if (s.per_lane == 2)
                hipLaunchKernelGGL((k_force_sym<double, double2, 2, 4>), g, b4, 0, s.stream, pj, st, part, base);
            else if (s.per_lane == 4)
                hipLaunchKernelGGL((k_force_sym<double, double2, 4, 4>), g, b4, 0, s.stream, pj, st, part, base);
            else
                hipLaunchKernelGGL((k_force_sym<double, double2, 8, 2>), g, b2, 0, s.stream, pj, st, part, base);
        }
        return;
    }
    if (s.persistent == 1) hipLaunchKernelGGL(k_zero_one, dim3(1), dim3(64), 0, s.stream, s.ctl + K_FQUEUE);
    if (s.fp32) {
        if (s.per_lane == 2)
            launch_force_p<float, float2, 2>(s, law);
        else
            launch_force_p<float, float2, 4>(s, law);
    } else {
        if (s.per_lane == 2)
            launch_force_p<double, double2, 2>(s, law);
        else
            launch_force_p<double, double2, 4>(s, law);
    }
}

int force_max_grid(Sim &s, int per_lane) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s.device) != hipSuccess || cus < 1)
        cus = 256;
    const bool fast = s.kind_fast != 0;
    int per_cu;
    if (s.fp32)
        per_cu = per_lane == 2 ? max_grid_p<float, float2, 2>(fast) : max_grid_p<float, float2, 4>(fast);
    else
        per_cu = per_lane == 2 ? max_grid_p<double, double2, 2>(fast) : max_grid_p<double, double2, 4>(fast);
    return cus * per_cu;
}

void launch_em(Sim &s, int level, unsigned index) {
    EmArgs a;
    a.n = s.n;
    a.S = s.S;
    a.dt = s.p.dt;
    a.amp = std::sqrt(2.0 * s.p.D * s.p.dt);
    a.amp_r = std::sqrt(2.0 * s.p.Dr * s.p.dt);
    a.v0 = s.p.v0;
    a.clip = s.p.noise_clip;
    a.D = s.p.D;
    a.Dr = s.p.Dr;
    a.level = level;
    a.index = index;
    a.periodic = s.period > 0.0 ? 1 : 0;
    const int nb = blocks_for(s.n, 256);
    const Tape &tp = s.adj.tape;
    signed char *wf = tp.on ? tp.emwf + (size_t)tp.step_idx * 2 * s.n : nullptr;
    const bool bridge = level > 0;
    auto go = [&](auto kern, auto part, const double2 *fdirect) {
        hipLaunchKernelGGL(kern, dim3(nb), dim3(256), 0, s.stream, a, (const StepBase *)s.dbase, part, s.reps,
                           s.rep_of, s.chunk_spec, s.Kd, s.pos_of, s.key_id, s.sp, s.rad, s.x, s.y, s.xy, s.xo, s.yo, s.th,
                           s.tho, s.acc, fdirect, wf, (const int *)s.ctl);
    };
    const float2 *p32 = (const float2 *)s.part;
    const double2 *p64 = (const double2 *)s.part, *none = nullptr, *fsr = (const double2 *)s.fsr;
    if (s.use_nl)
        bridge ? go(k_em<float2, true, true>, p32, fsr) : go(k_em<float2, true, false>, p32, fsr);
    else if (s.fp32)
        bridge ? go(k_em<float2, false, true>, p32, none) : go(k_em<float2, false, false>, p32, none);
    else
        bridge ? go(k_em<double2, false, true>, p64, none) : go(k_em<double2, false, false>, p64, none);
}

void launch_reduce_forces(Sim &s) {
    const int nb = blocks_for(s.n, 256);
    if (s.fp32)
        hipLaunchKernelGGL(k_reduce_forces<float2>, dim3(nb), dim3(256), 0, s.stream, s.n, s.S,
                           (const float2 *)s.part, s.reps, s.rep_of, s.chunk_spec, s.Kd, s.pos_of, s.sp, s.fout);
    else
        hipLaunchKernelGGL(k_reduce_forces<double2>, dim3(nb), dim3(256), 0, s.stream, s.n, s.S,
                           (const double2 *)s.part, s.reps, s.rep_of, s.chunk_spec, s.Kd, s.pos_of, s.sp, s.fout);
}

}  // namespace bd
