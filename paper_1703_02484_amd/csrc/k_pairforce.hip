// Stateless pair forces of the Sec. 2.2 law on caller device arrays:
//   F_i = sum_{j != i} K[s_i][s_j] g(d_ij) (r_i - r_j) / d_ij
// for positions and species that live in device memory owned by the caller,
// with no simulation handle.
//
// Layout.  The j range is cut into J equal splits; one workgroup takes 512
// particles i (2 per lane) against one split, stages the split's positions and
// species through LDS in blocks of 512 (the shared-memory broadcast of the
// paper's n-body kernel, Sec. 6: every lane reads the same j from LDS), and
// writes its K-weighted sums to part[split][i].  A second kernel adds the J
// splits in FP64 in split order and writes F in caller order, so results do
// not depend on the launch timing.  The only device memory beyond the
// caller's inputs and outputs is `part` (J * n * 2 values of the working
// precision).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "../../include/bd.h"

namespace {

constexpr int kPfBlock = 256;
constexpr int kPfPer = 2;                      // particles i per lane
constexpr int kPfI = kPfBlock * kPfPer;        // particles i per workgroup
constexpr int kPfJ = 512;                      // j staged in LDS per pass
constexpr int kPfTargetGroups = 2048;          // workgroups aimed for (8 per CU)
constexpr int kPfMaxSplits = 64;

struct PfLaw {
    int kind, S;
    double q, A, lam, cutoff;
    double K[BD_MAX_SPECIES * BD_MAX_SPECIES];
};

template <typename T>
struct Vec2;
template <>
struct Vec2<float> {
    using type = float2;
};
template <>
struct Vec2<double> {
    using type = double2;
};

// g(d)/d for the law (the factor multiplying r_i - r_j); 0 beyond the cutoff.
template <typename T>
__device__ __forceinline__ T law_factor(T d2, const PfLaw &law, T cut2, T expo, T invlam) {
    if (cut2 > (T)0 && d2 > cut2) return (T)0;
    if (law.kind == BD_FORCE_POWER) {
        if (law.q == 2.0) {
            const T r = (T)1 / sqrt(d2);
            return r * r * r;
        }
        return pow(d2, expo);
    }
    const T d = sqrt(d2);
    return (T)law.A * exp(-d * invlam) / d2;
}

// grid (ceil(n / 512), J); part[split * n + i] = sum over the split's j of K[s_i][s_j] g (r_i - r_j) / d.
template <typename T>
__global__ __launch_bounds__(kPfBlock) void k_pf_tiles(int n, int J, const double *__restrict__ xy,
                                                       const int32_t *__restrict__ species, PfLaw law,
                                                       typename Vec2<T>::type *__restrict__ part) {
    using T2 = typename Vec2<T>::type;
    __shared__ T2 pos[kPfJ];
    __shared__ int spc[kPfJ];
    __shared__ T kw[BD_MAX_SPECIES * BD_MAX_SPECIES];
    const int S = law.S;
    for (int k = threadIdx.x; k < S * S; k += kPfBlock) kw[k] = (T)law.K[k];
    const T cut2 = law.cutoff > 0.0 ? (T)(law.cutoff * law.cutoff) : (T)0;
    const T expo = (T)(-0.5 * (law.q + 1.0));
    const T invlam = (T)(1.0 / law.lam);

    const int ib = blockIdx.x * kPfI;
    T xi[kPfPer], yi[kPfPer], ax[kPfPer], ay[kPfPer];
    int ii[kPfPer], si[kPfPer];
#pragma unroll
    for (int p = 0; p < kPfPer; ++p) {
        const int i = ib + p * kPfBlock + threadIdx.x;
        const int c = i < n ? i : n - 1;
        ii[p] = i;
        xi[p] = (T)xy[2 * (size_t)c];
        yi[p] = (T)xy[2 * (size_t)c + 1];
        si[p] = species[c];
        ax[p] = (T)0;
        ay[p] = (T)0;
    }
    const long long per = ((long long)n + J - 1) / J;
    const int j0 = (int)min((long long)n, per * blockIdx.y);
    const int j1 = (int)min((long long)n, per * (blockIdx.y + 1));
    for (int jb = j0; jb < j1; jb += kPfJ) {
        const int m = min(kPfJ, j1 - jb);
        __syncthreads();   // the previous block of j has been read (and kw written before the first)
        for (int k = threadIdx.x; k < m; k += kPfBlock) {
            T2 v;
            v.x = (T)xy[2 * (size_t)(jb + k)];
            v.y = (T)xy[2 * (size_t)(jb + k) + 1];
            pos[k] = v;
            spc[k] = species[jb + k];
        }
        __syncthreads();
        for (int k = 0; k < m; ++k) {
            const T2 q = pos[k];
            const int sj = spc[k];
            const int j = jb + k;
#pragma unroll
            for (int p = 0; p < kPfPer; ++p) {
                const T dx = xi[p] - q.x;
                const T dy = yi[p] - q.y;
                const T d2 = dx * dx + dy * dy;
                const T g = ii[p] == j ? (T)0 : kw[si[p] * S + sj] * law_factor<T>(d2, law, cut2, expo, invlam);
                ax[p] += dx * g;
                ay[p] += dy * g;
            }
        }
    }
#pragma unroll
    for (int p = 0; p < kPfPer; ++p) {
        if (ii[p] < n) {
            T2 v;
            v.x = ax[p];
            v.y = ay[p];
            part[(size_t)blockIdx.y * n + ii[p]] = v;
        }
    }
}

// f[2i], f[2i+1] = sum over the splits in split order, in FP64.
template <typename T>
__global__ void k_pf_reduce(int n, int J, const typename Vec2<T>::type *__restrict__ part, double *__restrict__ f) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double fx = 0.0, fy = 0.0;
    for (int s = 0; s < J; ++s) {
        const auto v = part[(size_t)s * n + i];
        fx += (double)v.x;
        fy += (double)v.y;
    }
    f[2 * (size_t)i] = fx;
    f[2 * (size_t)i + 1] = fy;
}

// Number of j splits for n particles: enough workgroups to fill the device,
// at least one block of i per split.  Depends on n only.
int pf_splits(int n) {
    const long long nb = ((long long)n + kPfI - 1) / kPfI;
    long long J = (kPfTargetGroups + nb - 1) / nb;
    J = J < 1 ? 1 : J;
    J = J > kPfMaxSplits ? kPfMaxSplits : J;
    const long long jmax = ((long long)n + kPfI - 1) / kPfI;
    return (int)(J > jmax ? jmax : J);
}

size_t pf_value_bytes(int precision) { return precision == BD_PREC_FP32 ? sizeof(float2) : sizeof(double2); }

int pf_check(int32_t n, const double *xy, const int32_t *species, const bd_force_params *fp, int32_t precision,
             const double *f_out, PfLaw &law) {
    if (n < 1 || !xy || !species || !fp || !f_out || !fp->K) return BD_ERR_INVALID_ARG;
    if (precision != BD_PREC_FP32 && precision != BD_PREC_FP64) return BD_ERR_INVALID_ARG;
    if (fp->S < 1 || fp->S > BD_MAX_SPECIES) return BD_ERR_INVALID_ARG;
    if (fp->kind != BD_FORCE_POWER && fp->kind != BD_FORCE_SCREENED) return BD_ERR_INVALID_ARG;
    if (fp->kind == BD_FORCE_POWER && !(std::isfinite(fp->q) && fp->q > 0.0)) return BD_ERR_INVALID_ARG;
    if (fp->kind == BD_FORCE_SCREENED && !(std::isfinite(fp->A) && std::isfinite(fp->lambda) && fp->lambda > 0.0))
        return BD_ERR_INVALID_ARG;
    if (!std::isfinite(fp->cutoff)) return BD_ERR_INVALID_ARG;
    std::memset(&law, 0, sizeof(law));
    law.kind = fp->kind;
    law.S = fp->S;
    law.q = fp->q;
    law.A = fp->A;
    law.lam = fp->kind == BD_FORCE_SCREENED ? fp->lambda : 1.0;
    law.cutoff = fp->cutoff;
    for (int k = 0; k < fp->S * fp->S; ++k) {
        if (!std::isfinite(fp->K[k])) return BD_ERR_INVALID_ARG;
        law.K[k] = fp->K[k];
    }
    return BD_OK;
}

// Enqueues the two kernels on `stream` with `part` as the split sums.
int pf_enqueue(int32_t n, const double *xy, const int32_t *species, const PfLaw &law, int32_t precision,
               double *f_out, hipStream_t stream, void *part, int J) {
    const dim3 grid((n + kPfI - 1) / kPfI, J);
    const dim3 rgrid((n + 255) / 256);
    if (precision == BD_PREC_FP32) {
        hipLaunchKernelGGL(k_pf_tiles<float>, grid, dim3(kPfBlock), 0, stream, n, J, xy, species, law,
                           (float2 *)part);
        hipLaunchKernelGGL(k_pf_reduce<float>, rgrid, dim3(256), 0, stream, n, J, (const float2 *)part, f_out);
    } else {
        hipLaunchKernelGGL(k_pf_tiles<double>, grid, dim3(kPfBlock), 0, stream, n, J, xy, species, law,
                           (double2 *)part);
        hipLaunchKernelGGL(k_pf_reduce<double>, rgrid, dim3(256), 0, stream, n, J, (const double2 *)part, f_out);
    }
    return hipGetLastError() == hipSuccess ? BD_OK : BD_ERR_DEVICE;
}

}  // namespace

extern "C" int bd_pair_forces_dev(int32_t n, const double *xy, const int32_t *species, const bd_force_params *fp,
                                  int32_t precision, double *f_out, void *stream) {
    PfLaw law;
    const int rc = pf_check(n, xy, species, fp, precision, f_out, law);
    if (rc != BD_OK) return rc;
    const hipStream_t st = (hipStream_t)stream;
    const int J = pf_splits(n);
    void *part = nullptr;
    if (hipMalloc(&part, (size_t)J * n * pf_value_bytes(precision)) != hipSuccess) {
        (void)hipGetLastError();
        return BD_ERR_OOM;
    }
    int out = pf_enqueue(n, xy, species, law, precision, f_out, st, part, J);
    if (hipStreamSynchronize(st) != hipSuccess) out = BD_ERR_DEVICE;
    if (hipFree(part) != hipSuccess) out = BD_ERR_DEVICE;
    return out;
}

// ------------------------------------------------------------------ no-allocation variant
// For callers that cannot allocate device memory (code under HIP graph capture,
// serving loops, harnesses that forbid hipMalloc): the split sums live in a
// fixed device array of kScratchBytes, one copy per GPU, held until the
// process ends.  Its device address is looked up once per device (with that
// device current) on the first call there; kernels receive that address,
// never the array's host-side name.
namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Device address of this device's scratch array, or nullptr on failure.
void *scratch_for_current_device() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" int bd_pair_forces_dev_noalloc(int32_t n, const double *xy, const int32_t *species,
                                          const bd_force_params *fp, int32_t precision, double *f_out, void *stream) {
    PfLaw law;
    const int rc = pf_check(n, xy, species, fp, precision, f_out, law);
    if (rc != BD_OK) return rc;
    const int J = pf_splits(n);
    const size_t need = (size_t)J * (size_t)n * pf_value_bytes(precision);
    if (need > kScratchBytes) {
        std::fprintf(stderr, "bd_pair_forces_dev_noalloc: n = %d needs %zu bytes of scratch, more than its %zu\n",
                     (int)n, need, kScratchBytes);
        return BD_ERR_INVALID_ARG;
    }
    void *part = scratch_for_current_device();
    if (!part) return BD_ERR_DEVICE;
    // every split sum that the reduction reads is written first: nothing to clear
    return pf_enqueue(n, xy, species, law, precision, f_out, (hipStream_t)stream, part, J);
}
