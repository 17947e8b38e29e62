// The 1D AT stepper with the whole periodic grid in one workgroup, for grids
// small enough that their state is a few KB (N <= 256 * PPT): one launch
// advances any number of steps.
//
// Same method and evaluation order as the fused kernels of at_step1d.hip
// (paper section 3.2 stencils with forward Euler; AT halos extrapolated in
// time from the neighbour edge's levels n-k, n-k-1, ..., section 2 Eqs.
// (1)-(2)), so the results are bit-identical to one launch per step.  What
// differs is the decomposition: thread i holds points [i*PPT, (i+1)*PPT) of
// the grid, the neighbour exchange wraps around the workgroup (the grid is
// periodic), so no rim is recomputed and a launch needs no overlap with its
// neighbours; the tile edges of every level live in an LDS ring of D + 2
// levels (D = L + m - 1, the deepest level a step reads below its own).
// Every thread's points lie in one tile (the tile width is a multiple of
// PPT), so the AT values are written into the halo slots of a thread's
// register window before the standard stencil, as in the aligned kernels.
#include "at_internal.h"
#include "at_stencil1d.h"

namespace atk {

namespace {

constexpr int kWT = 256;      // threads of the workgroup

// ring slot of level n0 + d (|d| < R)
__device__ __forceinline__ int64_t wslot(const Step1D &a, int64_t d)
{
    int64_t x = a.slot0 + d;
    if (x < 0) x += a.R;
    if (x >= a.R) x -= a.R;
    return x;
}

template <int ORDER, bool LINEAR, bool FMA, int PPT>
__global__ __launch_bounds__(kWT) void k_step1d_whole(Step1D a)
{
    constexpr int H = ORDER / 2;
    constexpr int M = (ORDER == 2) ? 2 : 3;
    extern __shared__ double lds[];
    const int NA = (int)(a.N / PPT);                      // threads holding points
    const int P = (int)a.P, W = (int)a.W, D = a.D, HR = D + 2, S = a.s;
    double *xch = lds;                                    // [2][kWT][2H]
    double *eh = lds + 2 * kWT * 2 * H;                   // [HR][P][2][H]: edge ring
    // ring row of level n0 + t (t >= -D): (t + D) mod HR, for t + D < 2 HR
    auto hrow = [&](int r) { return r >= HR ? r - HR : r; };

    const int tid = threadIdx.x;
    const bool act = tid < NA;
    const int g0 = tid * PPT;
    const int tile = act ? g0 / W : 0;
    const int o0 = g0 - tile * W;
    const bool lo_edge = act && o0 == 0;
    const bool hi_edge = act && o0 + PPT == W;
    const int tl = tile == 0 ? P - 1 : tile - 1;          // the tiles across the two faces
    const int tr = tile == P - 1 ? 0 : tile + 1;
    const int left = tid == 0 ? NA - 1 : tid - 1;         // periodic neighbours in the exchange
    const int right = tid == NA - 1 ? 0 : tid + 1;
    const int64_t F = 2 * a.P;

    // ---- prologue: tile edges of levels n0-D .. n0-1 into ring rows 0 .. D-1
    for (int e = tid; e < D * P * 2 * H; e += kWT) {
        const int q = e % H, side = (e / H) & 1, tp = (e / (2 * H)) % P, d = e / (2 * H * P);
        const int64_t lev = a.n0 - D + d;
        eh[e] = lev >= 0 ? a.ring[((wslot(a, lev - a.n0) * a.P + tp) * 2 + side) * H + q] : 0.0;
    }
    double w[PPT + 2 * H];
#pragma unroll
    for (int j = 0; j < PPT; ++j) w[H + j] = act ? a.uin[g0 + j] : 0.0;
#pragma unroll
    for (int q = 0; q < H; ++q) { w[q] = 0.0; w[PPT + H + q] = 0.0; }
    // delays of this thread's faces (face f = 2 tile + side), one step ahead
    int kl = 0, kr = 0;
    if (lo_edge && S > 0) kl = a.delays[a.n0 * F + 2 * tile];
    if (hi_edge && S > 0) kr = a.delays[a.n0 * F + 2 * tile + 1];
    __syncthreads();

    for (int t = 0, tb = 0; t < S; ++t, tb = (tb + 1 == HR) ? 0 : tb + 1) {
        const int64_t n = a.n0 + t;
        int kl2 = 0, kr2 = 0;
        if (t + 1 < S) {
            if (lo_edge) kl2 = a.delays[(n + 1) * F + 2 * tile];
            if (hi_edge) kr2 = a.delays[(n + 1) * F + 2 * tile + 1];
        }
        // ---- this level's tile edges: the LDS ring, and the global ring for
        // the levels a later launch reads (every level with the edge tape)
        if (lo_edge || hi_edge) {
            const int row = hrow(tb + D);
            const bool pub = a.publish == 1 || (a.publish == 2 && t + D >= S);
            const int64_t slot = wslot(a, t);
#pragma unroll
            for (int q = 0; q < H; ++q) {
                if (lo_edge) {
                    eh[((row * P + tile) * 2 + 0) * H + q] = w[H + q];
                    if (pub) a.ring[((slot * a.P + tile) * 2 + 0) * H + q] = w[H + q];
                }
                if (hi_edge) {
                    eh[((row * P + tile) * 2 + 1) * H + q] = w[PPT + q];
                    if (pub) a.ring[((slot * a.P + tile) * 2 + 1) * H + q] = w[PPT + q];
                }
            }
        }
        // ---- neighbour exchange (double-buffered by step parity)
        double *buf = xch + (t & 1) * kWT * 2 * H;
        if (act) {
#pragma unroll
            for (int q = 0; q < H; ++q) {
                buf[tid * 2 * H + q] = w[H + q];
                buf[tid * 2 * H + H + q] = w[PPT + q];
            }
        }
        __syncthreads();
        if (act) {
#pragma unroll
            for (int q = 0; q < H; ++q) {
                w[q] = buf[left * 2 * H + H + q];
                w[PPT + H + q] = buf[right * 2 * H + q];
            }
            // ---- AT halo values across the tile faces (k = 0: the raw neighbour
            // stays); the source edge's levels n-k-j from the ring rows
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const int kk = side == 0 ? (lo_edge ? kl : 0) : (hi_edge ? kr : 0);
                if (kk > 0) {
                    const int stile = side == 0 ? tl : tr;
                    const int sside = 1 - side;
#pragma unroll
                    for (int q = 0; q < H; ++q) {
                        double vv[3] = {0.0, 0.0, 0.0};
#pragma unroll
                        for (int jj = 0; jj < M; ++jj)
                            if (jj == 0 || !a.stale)
                                vv[jj] = eh[((hrow(tb + D - kk - jj) * P + stile) * 2 + sside) * H + q];
                        const double hv = extrap<FMA>(kk, a.stale != 0, vv[0], vv[1], vv[2], M);
                        if (side == 0) w[q] = hv;
                        else w[PPT + H + q] = hv;
                    }
                }
            }
            // ---- the standard stencil on every point, each new value formed after
            // the last stencil that reads its old value (same operations as update())
            step_window<ORDER, LINEAR, FMA, PPT>(w, a);
        }
        kl = kl2;
        kr = kr2;
    }
    if (act) {
#pragma unroll
        for (int j = 0; j < PPT; ++j) a.uout[g0 + j] = w[H + j];
    }
}

}  // namespace

size_t step1d_whole_lds_bytes(int order, int64_t P, int D)
{
    const int H = order / 2;
    return 8 * ((size_t)2 * kWT * 2 * H + (size_t)(D + 2) * (size_t)P * 2 * H);
}

// Points per thread for the whole grid in one workgroup: the fewest of 4, 8,
// 16 that divide N and the tile width and leave at most 256 threads; 0 when
// none does or the edge ring would exceed 64 KiB of LDS
int step1d_whole_ppt(int64_t N, int64_t W, int64_t P, int order, int D)
{
    if (step1d_whole_lds_bytes(order, P, D) > 64 * 1024) return 0;
    for (int p : {4, 8, 16})
        if (N % p == 0 && W % p == 0 && N / p <= kWT) return p;
    return 0;
}

hipError_t launch_step1d_whole(const Step1D &a, int order, bool linear, bool fma, int ppt,
                               hipStream_t st)
{
    const size_t lds = step1d_whole_lds_bytes(order, a.P, a.D);
    dim3 grid(1), block(kWT);
#define AT_W(O, LI, F, P) hipLaunchKernelGGL((k_step1d_whole<O, LI, F, P>), grid, block, lds, st, a)
#define AT_WP(O, LI, F)                                                                  \
    do {                                                                                 \
        if (ppt == 4) AT_W(O, LI, F, 4);                                                 \
        else if (ppt == 8) AT_W(O, LI, F, 8);                                            \
        else if (ppt == 16) AT_W(O, LI, F, 16);                                          \
        else return hipErrorInvalidValue;                                                \
    } while (0)
    if (order == 2) {
        if (linear) { if (fma) AT_WP(2, true, true); else AT_WP(2, true, false); }
        else { if (fma) AT_WP(2, false, true); else AT_WP(2, false, false); }
    } else {
        if (linear) { if (fma) AT_WP(4, true, true); else AT_WP(4, true, false); }
        else { if (fma) AT_WP(4, false, true); else AT_WP(4, false, false); }
    }
#undef AT_WP
#undef AT_W
    return hipGetLastError();
}

}  // namespace atk
