// Weakly-synchronous 1D stepper of libat.so for gfx950: the delays EMERGE from
// the progress of the tiles instead of being prescribed.
//
// Method (paper section 5.2, Algorithm 2): every tile advances on its own.
// After computing level n+1 it writes its two edges into the circular buffer
// ("ring") slot (n+1) mod R and then announces the level through a per-edge
// counter (the analogue of a notified put: data first, notification after;
// the data moves with device-coherent stores and loads, and the counter is
// written only once those stores have completed).  Before step n a tile reads
// the newest announced level t of each neighbour edge; the delay is
// k = n - min(t, n).  A tile waits only while k would exceed the bound the
// method allows, min(L, max(0, n - m + 1)) (the blocking receive of
// Algorithm 2, including its start-up synchrony); otherwise it proceeds at
// once with the AT halo of section 2, Eqs. (1)-(2), built from levels n-k,
// n-k-1(, n-k-2) of the neighbour's edge.  The delay actually used is stored
// as k[n][f], so a run can be replayed exactly with prescribed delays.
//
// Work decomposition: one workgroup of NT threads (256, or one wave of 64
// for narrow tiles) per tile of width W = NT * PPT, PPT consecutive points
// per thread held in registers for the whole run; h values per side are
// traded with the neighbouring threads through LDS each step.  Thread 0
// receives the left halo and publishes the tile's left edge, thread NT-1 the
// right ones.  All tiles must be resident at
// once (cooperative launch), and every wait is bounded: past the spin limit a
// workgroup sets the error flag and leaves, and a waiting workgroup that sees
// the flag leaves too, so every wave reaches the end of the kernel.
#include "at_internal.h"
#include "at_stencil1d.h"
#include "at_ws.h"

namespace atk {

namespace {

template <int ORDER, bool LINEAR, int PPT, int NT>
__global__ __launch_bounds__(NT) void k_ws1d(Ws1D A)
{
    constexpr int H = ORDER / 2;
    constexpr int M = ORDER == 2 ? 2 : 3;
    static_assert(PPT >= H, "a thread holds at least h points");
    __shared__ double lo[2][NT][H], hi[2][NT][H];
    __shared__ int s_stop;
    const int t = threadIdx.x;
    const int64_t P = A.P, b = blockIdx.x;
    const int64_t bl = b == 0 ? P - 1 : b - 1, br = b + 1 == P ? 0 : b + 1;
    const int64_t base = b * A.W + (int64_t)t * PPT;
    const bool stale = A.stale != 0;
    const int64_t tile2h = 2 * H;
    double v[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) v[j] = A.u[base + j];
    if (t == 0) s_stop = 0;

    // edge of tile q, side s (0 left, 1 right), level n: ring slot n mod R
    auto edge = [&](int64_t n, int64_t q, int s) -> double * {
        return A.ring + ((n % A.R) * P + q) * tile2h + s * H;
    };
    auto publish = [&](int64_t n) {
        if (t == 0) {
            double *e = edge(n, b, 0);
#pragma unroll
            for (int i = 0; i < H; ++i) st_coherent(e + i, v[i]);
            announce(A.cnt + 2 * b + 0, (int32_t)n);
        }
        if (t == NT - 1) {
            double *e = edge(n, b, 1);
#pragma unroll
            for (int i = 0; i < H; ++i) st_coherent(e + i, v[PPT - H + i]);
            announce(A.cnt + 2 * b + 1, (int32_t)n);
        }
    };
    // AT halo value i (0 .. h-1, left to right along x) of neighbour tile q's
    // edge s at delay k for step n
    auto halo = [&](int64_t n, int k, int64_t q, int s, double (&out)[H]) {
        const double *e0 = edge(n - k, q, s);
        if (k == 0 || stale) {
#pragma unroll
            for (int i = 0; i < H; ++i) out[i] = ld_coherent(e0 + i);
            return;
        }
        const double *e1 = edge(n - k - 1, q, s);
        const double *e2 = M == 3 ? edge(n - k - 2, q, s) : e1;
#pragma unroll
        for (int i = 0; i < H; ++i)
            out[i] = extrap<false>(k, false, ld_coherent(e0 + i), ld_coherent(e1 + i), ld_coherent(e2 + i), M);
    };

    __syncthreads();                                  // s_stop initialised before any wait
    publish(A.n0);
    for (int64_t n = A.n0; n < A.n0 + A.nsteps; ++n) {
        const int buf = (int)(n & 1);
        ws_idle(A.jitter, A.seed, b, n);
        // thread edges for the neighbouring threads
#pragma unroll
        for (int i = 0; i < H; ++i) {
            lo[buf][t][i] = v[i];
            hi[buf][t][i] = v[PPT - H + i];
        }
        // receive: the newest announced level of the neighbour edge, waiting
        // only while the delay would pass its bound
        const int32_t kmax = (int32_t)min((int64_t)A.L, max((int64_t)0, n - M + 1));
        double hl[H], hr[H];
        if (t == 0 || t == NT - 1) {
            const int s = t == 0 ? 1 : 0;                 // the neighbour's facing edge
            const int64_t q = t == 0 ? bl : br;
            const int32_t got = ws_wait(A.cnt + 2 * q + s, (int32_t)(n - kmax), A.err,
                                        A.spin_limit);
            if (got == -2) {
                s_stop = 1;
            } else {
                const int k = (int)(n - min((int64_t)got, n));
                A.delays[n * 2 * P + 2 * b + (t == 0 ? 0 : 1)] = (int8_t)k;
                if (t == 0) halo(n, k, q, s, hl);
                else halo(n, k, q, s, hr);
            }
        }
        __syncthreads();
        if (s_stop) break;
        // stencil: ext = [left h][own PPT][right h]
        double ext[PPT + 2 * H];
#pragma unroll
        for (int i = 0; i < H; ++i) {
            ext[i] = t == 0 ? hl[i] : hi[buf][t - 1][i];
            ext[H + PPT + i] = t == NT - 1 ? hr[i] : lo[buf][t + 1][i];
        }
#pragma unroll
        for (int j = 0; j < PPT; ++j) ext[H + j] = v[j];
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            double nb[4];
            if constexpr (ORDER == 2) {
                nb[0] = ext[j];
                nb[1] = ext[j + 2];
            } else {
                nb[0] = ext[j];
                nb[1] = ext[j + 1];
                nb[2] = ext[j + 3];
                nb[3] = ext[j + 4];
            }
            v[j] = update<ORDER, LINEAR, false>(nb, ext[H + j], A.coef);
        }
        publish(n + 1);
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) A.u[base + j] = v[j];
}

__global__ __launch_bounds__(256) void k_ws_init(int32_t *cnt, int64_t n, int32_t v, int32_t *err)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) cnt[i] = v;
    if (i == 0) *err = 0;
}

}  // namespace

// Threads per workgroup and points per thread for tile width W: 256 threads
// when W = 256 q, else one wave when W = 64 q, with q in {1, 2, 4, 8, 16} and
// q >= h; false when W fits neither.
bool ws1d_shape(int64_t W, int h, int *nt, int *ppt)
{
    for (const int t : {256, 64}) {
        if (W % t != 0) continue;
        const int64_t q = W / t;
        if ((q == 1 || q == 2 || q == 4 || q == 8 || q == 16) && q >= h) {
            *nt = t;
            *ppt = (int)q;
            return true;
        }
    }
    return false;
}

// the kernel for (order, advection mode, points per thread, threads), or null
static const void *ws1d_kernel(int order, bool linear, int ppt, int nt)
{
#define WS_PICK(O, PP, T)                                                                      \
    if (order == O && ppt == PP && nt == T)                                                    \
        return linear ? (const void *)k_ws1d<O, true, PP, T> : (const void *)k_ws1d<O, false, PP, T>;
#define WS_PICK_T(T) WS_PICK(2, 1, T) WS_PICK(2, 2, T) WS_PICK(2, 4, T) WS_PICK(2, 8, T)          \
    WS_PICK(2, 16, T) WS_PICK(4, 2, T) WS_PICK(4, 4, T) WS_PICK(4, 8, T) WS_PICK(4, 16, T)
    WS_PICK_T(256)
    WS_PICK_T(64)
#undef WS_PICK_T
#undef WS_PICK
    return nullptr;
}

// Largest number of k_ws1d workgroups that can be resident at once for this
// order, advection mode and tile width (0 if the shape is not supported)
int64_t ws1d_max_tiles(int order, bool linear, int64_t W)
{
    int nt = 0, ppt = 0;
    if (!ws1d_shape(W, order / 2, &nt, &ppt)) return 0;
    const void *f = ws1d_kernel(order, linear, ppt, nt);
    if (!f) return 0;
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, nt, 0) != hipSuccess) return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return (int64_t)per_cu * cus;
}

hipError_t launch_ws_init(int32_t *cnt, int64_t n, int32_t v, int32_t *err, hipStream_t st)
{
    const int64_t g = (n + 255) / 256;
    hipLaunchKernelGGL(k_ws_init, dim3((unsigned)(g > 0 ? g : 1)), dim3(256), 0, st, cnt, n, v,
                       err);
    return hipGetLastError();
}

hipError_t launch_ws1d(const Ws1D &a, int order, bool linear, hipStream_t st)
{
    int nt = 0, ppt = 0;
    if (!ws1d_shape(a.W, order / 2, &nt, &ppt)) return hipErrorInvalidValue;
    const void *f = ws1d_kernel(order, linear, ppt, nt);
    if (!f) return hipErrorInvalidValue;
    void *args[] = {(void *)&a};
    return hipLaunchCooperativeKernel(f, dim3((unsigned)a.P), dim3(nt), args, 0, st);
}

}  // namespace atk
