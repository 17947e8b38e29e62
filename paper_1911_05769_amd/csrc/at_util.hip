// Utility kernels of libat.so for gfx950: the delay generator, fills, the
// ring-poisoning debug pass, device copies and the reductions (diagnostics,
// misfit, dJ/dnu).  None of them is part of a time step.
#include <mutex>

#include "../../include/at.h"
#include "at_internal.h"

at_status at_fail(at_status st, const char *msg);   // at_api.hip: keeps the message

namespace atk {

namespace {

// Delay array: SplitMix64 (Steele, Lea & Flood 2014) output for the state
// seed + gamma*(1 + n*F + f), mapped to the distribution by a multiply-shift
// of the high 32 bits, then clamped to min(k, L, max(0, n - m + 1)).
__global__ void k_delays(int8_t *out, int64_t total, int64_t F, int L, int m, int dist,
                         uint64_t seed)
{
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        uint64_t z = seed + 0x9E3779B97F4A7C15ULL * (uint64_t)(idx + 1);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        z = z ^ (z >> 31);
        const uint64_t hi = z >> 32, lo = z & 0xFFFFFFFFULL;
        int k;
        if (dist == 0) k = (int)((hi * (uint64_t)(L + 1)) >> 32);
        else k = (L == 0 || lo < 0x80000000ULL) ? 0 : 1 + (int)((hi * (uint64_t)L) >> 32);
        const int64_t n = idx / F;
        int64_t lim = n - m + 1;
        if (lim < 0) lim = 0;
        if (lim > L) lim = L;
        out[idx] = (int8_t)(k < lim ? k : lim);
    }
}

__global__ void k_fill(double *p, int64_t n, double v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// NaN into every ring slot outside the live window of nlive slots starting at
// slot s0 (wrapping at R); lev doubles per slot
__global__ void k_poison(double *ring, int64_t R, int64_t lev, int s0, int nlive)
{
    const int64_t n = R * lev;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t rel = i / lev - s0;
        if (rel < 0) rel += R;
        if (rel >= nlive) ring[i] = __builtin_nan("");
    }
}

__global__ void k_copy(double *__restrict__ dst, const double *__restrict__ src, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// One 16-byte element per thread and no loop, so every workgroup moves one
// contiguous 4 KiB block: the form that streams fastest here (about 6.2 TB/s
// for 1 GiB, against about 5.1 for the runtime's device-to-device copy).  The
// odd last double, if any, is copied by thread 0.
__global__ __launch_bounds__(kThreads) void k_copy16(double2 *__restrict__ dst,
                                                     const double2 *__restrict__ src, int64_t n2,
                                                     double *dtail, const double *stail)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n2) dst[i] = src[i];
    if (dtail && i == 0) *dtail = *stail;
}

// ---------------------------------------------------------------------------
// Reductions: per-thread compensated accumulation, wave64 shuffles, one
// partial per workgroup, then a single-workgroup pass in fixed order.
// ---------------------------------------------------------------------------

// Maximum that keeps a NaN once one is seen (fmax would drop it, so a field
// that has blown up would report a finite maximum)
__device__ __forceinline__ double nan_max(double a, double b)
{
    return (a > b || a != a) ? a : b;
}

__device__ __forceinline__ double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = nan_max(v, __shfl_down(v, off, 64));
    return v;
}

// part[b*6 + {0..5}] = max|u|, sum u (s, c), sum|u| (s, c), count of
// non-finite values
__global__ __launch_bounds__(kThreads) void k_stats_part(const double *u, int64_t n, double *part)
{
    double mx = 0.0;
    Acc s{0.0, 0.0}, sa{0.0, 0.0};
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        const double v = u[i];
        const double a = fabs(v);
        mx = nan_max(mx, a);
        bad += (a == a && a <= 1.79769313486231570815e308) ? 0 : 1;
        acc_add(s, v);
        acc_add(sa, a);
    }
    mx = wave_max(mx);
    s = wave_acc(s);
    sa = wave_acc(sa);
    for (int off = 32; off > 0; off >>= 1) bad += __shfl_down(bad, off, 64);
    __shared__ double red[kThreads / 64][6];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        red[wv][0] = mx; red[wv][1] = s.s; red[wv][2] = s.c; red[wv][3] = sa.s; red[wv][4] = sa.c;
        red[wv][5] = (double)bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0][0], nb = red[0][5];
        Acc S{red[0][1], red[0][2]}, SA{red[0][3], red[0][4]};
        for (int q = 1; q < kThreads / 64; ++q) {
            m = nan_max(m, red[q][0]);
            acc_merge(S, Acc{red[q][1], red[q][2]});
            acc_merge(SA, Acc{red[q][3], red[q][4]});
            nb += red[q][5];
        }
        double *o = part + (int64_t)blockIdx.x * 6;
        o[0] = m; o[1] = S.s; o[2] = S.c; o[3] = SA.s; o[4] = SA.c; o[5] = nb;
    }
}

__global__ void k_stats_final(const double *part, int nb, int64_t n, double *out4)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double m = 0.0, bad = 0.0;
    Acc S{0.0, 0.0}, SA{0.0, 0.0};
    for (int b = 0; b < nb; ++b) {
        const double *o = part + (int64_t)b * 6;
        m = nan_max(m, o[0]);
        acc_merge(S, Acc{o[1], o[2]});
        acc_merge(SA, Acc{o[3], o[4]});
        bad += o[5];
    }
    out4[0] = m;
    out4[1] = (S.s + S.c) / (double)n;
    out4[2] = SA.s + SA.c;
    out4[3] = bad;
}

// part[b*2 + {0,1}] = sum 0.5 d^2 (s, c); lam = d = u - t
__global__ __launch_bounds__(kThreads) void k_loss_part(const double *u, const double *t,
                                                       double *lam, int64_t n, double *part)
{
    Acc s{0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        const double d = u[i] - t[i];
        if (lam) lam[i] = d;
        acc_add(s, 0.5 * (d * d));
    }
    s = wave_acc(s);
    __shared__ double red[kThreads / 64][2];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) { red[wv][0] = s.s; red[wv][1] = s.c; }
    __syncthreads();
    if (threadIdx.x == 0) {
        Acc S{red[0][0], red[0][1]};
        for (int q = 1; q < kThreads / 64; ++q) acc_merge(S, Acc{red[q][0], red[q][1]});
        part[(int64_t)blockIdx.x * 2] = S.s;
        part[(int64_t)blockIdx.x * 2 + 1] = S.c;
    }
}

// out = sum of the compensated pairs part[i*2], part[i*2+1] in a fixed
// order: thread t merges pairs t, t+256, ... in turn, each wave combines its
// lanes by the fixed shuffle tree, wave 0 the four wave sums in order
__global__ __launch_bounds__(kThreads) void k_pairs_final(const double *part, int64_t np,
                                                          double *out)
{
    __shared__ double red[kThreads / 64][2];
    const int t = threadIdx.x;
    Acc S{0.0, 0.0};
#pragma unroll 4
    for (int64_t b = t; b < np; b += kThreads) acc_merge(S, Acc{part[b * 2], part[b * 2 + 1]});
    S = wave_acc(S);
    if ((t & 63) == 0) { red[t >> 6][0] = S.s; red[t >> 6][1] = S.c; }
    __syncthreads();
    if (t == 0) {
        Acc T{0.0, 0.0};
        for (int w = 0; w < kThreads / 64; ++w) acc_merge(T, Acc{red[w][0], red[w][1]});
        out[0] = T.s + T.c;
    }
}

int grid_for(int64_t n)
{
    int64_t g = (n + kThreads - 1) / kThreads;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

hipError_t launch_delays(int8_t *out, int64_t nsteps, int64_t F, int L, int m, int dist,
                         uint64_t seed, hipStream_t st)
{
    const int64_t total = nsteps * F;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_delays, dim3(grid_for(total)), dim3(kThreads), 0, st, out, total, F, L,
                       m, dist, seed);
    return hipGetLastError();
}

hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kThreads), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_poison(double *ring, int64_t R, int64_t lev, int s0, int nlive, hipStream_t st)
{
    const int64_t n = R * lev;
    if (n <= 0 || nlive >= R) return hipSuccess;
    int64_t g = grid_for(n);
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_poison, dim3((unsigned)g), dim3(kThreads), 0, st, ring, R, lev, s0, nlive);
    return hipGetLastError();
}

hipError_t launch_copy(double *dst, const double *src, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t n2 = n / 2;
    const int64_t blocks = (n2 + kThreads - 1) / kThreads;
    const bool aligned = (((uintptr_t)dst | (uintptr_t)src) & 15) == 0;
    if (aligned && n2 > 0 && blocks <= 0x7fffffff) {
        double *dt = (n & 1) ? dst + (n - 1) : nullptr;
        const double *stl = (n & 1) ? src + (n - 1) : nullptr;
        hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(kThreads), 0, st,
                           reinterpret_cast<double2 *>(dst), reinterpret_cast<const double2 *>(src),
                           n2, dt, stl);
    } else {
        hipLaunchKernelGGL(k_copy, dim3(grid_for(n)), dim3(kThreads), 0, st, dst, src, n);
    }
    return hipGetLastError();
}

hipError_t launch_stats(const double *u, int64_t n, double *part, double *out4, hipStream_t st)
{
    int nb = grid_for(n);
    if (nb > kRedBlocks) nb = kRedBlocks;
    hipLaunchKernelGGL(k_stats_part, dim3(nb), dim3(kThreads), 0, st, u, n, part);
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(64), 0, st, part, nb, n, out4);
    return hipGetLastError();
}

hipError_t launch_loss(const double *u, const double *t, double *lam, int64_t n, double *part,
                       double *J, hipStream_t st)
{
    int nb = grid_for(n);
    if (nb > kRedBlocks) nb = kRedBlocks;
    hipLaunchKernelGGL(k_loss_part, dim3(nb), dim3(kThreads), 0, st, u, t, lam, n, part);
    hipLaunchKernelGGL(k_pairs_final, dim3(1), dim3(kThreads), 0, st, part, (int64_t)nb, J);
    return hipGetLastError();
}

hipError_t launch_gnu_final(const double *part, int64_t nparts, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_pairs_final, dim3(1), dim3(kThreads), 0, st, part, nparts, out);
    return hipGetLastError();
}

}  // namespace atk

// ---------------------------------------------------------------------------
// at_stats_noalloc: the diagnostics reduction with its per-workgroup partials
// in a static device array instead of a context's workspace
// ---------------------------------------------------------------------------

namespace atk {

namespace {

// partials of the first reduction pass: kRedBlocks workgroups x 6 doubles
// (48 KiB); each GPU the library runs on holds its own copy until the
// process ends.  In host code this name is only a stand-in for the symbol:
// kernels get the device address that hipGetSymbolAddress returns.
__device__ __align__(256) double scratch[kRedBlocks * 6];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device, looked up once per
// device (with that device current)
hipError_t scratch_on_current_device(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

}  // namespace atk

extern "C" {

at_status at_stats_noalloc(const double *u, int64_t n, double *out4, void *stream)
{
    using namespace atk;
    char msg[160];
    if (!u || !out4) return at_fail(AT_ERR_ARG, "at_stats_noalloc: null argument");
    if (n < 1 || n > AT_NOALLOC_MAX_POINTS) {
        snprintf(msg, sizeof msg, "at_stats_noalloc: n = %lld outside 1..%lld", (long long)n,
                 (long long)AT_NOALLOC_MAX_POINTS);
        return at_fail(AT_ERR_ARG, msg);
    }
    double *part = nullptr;
    hipError_t e = scratch_on_current_device(&part);
    if (e == hipSuccess) e = launch_stats(u, n, part, out4, (hipStream_t)stream);
    if (e != hipSuccess) {
        snprintf(msg, sizeof msg, "at_stats_noalloc: %s", hipGetErrorString(e));
        return at_fail(AT_ERR_HIP, msg);
    }
    return AT_OK;
}

}  // extern "C"

