// 1D stepper kernels of libat.so for gfx950: the AT stepper with one or
// several fused steps per launch, and its batched form.
//
// Method: viscous Burgers u_t + u u_x = nu u_xx (or linear advection c u_x),
// central differences and forward Euler (paper section 3.2) on P tiles of a
// periodic grid.  A point whose stencil crosses its tile's edge reads a halo
// value extrapolated in time from the neighbour edge's levels n-k, n-k-1, ...
// (section 2, Eqs. (1)-(2); three levels for the 4th-order scheme), with the
// delay k prescribed per directed face and step.  As in section 5.2, the halo
// approximation is separate from the stencil, which is the same everywhere.
//
// Arithmetic is binary64 with contraction disabled (-ffp-contract=off); the
// evaluation order of every formula is fixed:
//   order 2: D1 = (r1 - l1)*c1,                 D2 = ((r1 - 2u) + l1)*c2
//   order 4: D1 = (8(r1 - l1) - (r2 - l2))*c1,  D2 = ((16(r1 + l1) - 30u) - (r2 + l2))*c2
//   F = nu*D2 - a*D1 (a = u, or c for linear advection),  u' = u + dt*F
//   halo, two levels:   H = v0 + k*(v0 - v1)
//   halo, three levels: H = (v0 + k*d1) + w2*(d1 - (v1 - v2)), d1 = v0 - v1, w2 = 0.5*k*(k+1)
//
// Work decomposition of k_step1d (s steps per launch):
//   * a workgroup of 256 threads owns CH consecutive points and loads the
//     region [c0 - s*h, c0 + CH + s*h) of level n0 (coalesced, through LDS);
//   * each thread keeps PPT consecutive region points in registers and trades
//     h values per side with its neighbours through LDS once per step;
//   * the valid part of the region shrinks by h per step (overlapped
//     trapezoids); neighbouring tiles' edges inside the region are recomputed
//     redundantly with the same operations, so the result is bit-identical to
//     one launch per step;
//   * edge values of in-launch levels are kept in an LDS edge history for
//     delayed halo reads; levels before n0 come from the ring in HBM;
//   * owned tile-edge points are published to ring slot n mod R: those of every
//     level when the run keeps the edge tape for the adjoint, else those of the
//     last L + m - 1 levels of a launch, the only ones a later launch reads.
#include "at_internal.h"
#include "at_stencil1d.h"

namespace atk {

namespace {

constexpr int kPPT = 16;      // region points per thread (fused and general kernels)
constexpr int kPPTPlain = 8;  // region points per thread of the single-step kernel

__device__ __forceinline__ int64_t floordiv(int64_t a, int64_t b)
{
    int64_t q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

// ring slot of level n0 + d for d in [-(R-1), R-1] (the levels a launch
// touches lie within one ring length of n0)
__device__ __forceinline__ int64_t ring_slot(const Step1D &a, int64_t d)
{
    int64_t x = a.slot0 + d;
    if (x < 0) x += a.R;
    if (x >= a.R) x -= a.R;
    return x;
}

// whether step t of a launch of S steps writes its level's tile edges to the
// ring: every level (publish 1), or only the last D levels of the launch
// (publish 2), the only ones a later launch reads when no edge tape is kept
__device__ __forceinline__ bool publish_level(const Step1D &a, int t, int S)
{
    return a.publish == 1 || (a.publish == 2 && t + a.D >= S);
}

// The region's field passes through a padded LDS stage (point r of a part at
// r + r/PPT, so that neither the coalesced accesses nor the per-thread ones
// conflict on banks) in stage_parts(PPT) parts: at 16 points per thread in two
// halves of 2048 points, which keeps the stage at 17 KB instead of 34 KB so
// that LDS does not cap the workgroups per CU below what registers allow.
__host__ __device__ constexpr int stage_parts(int ppt) { return ppt >= 16 ? 2 : 1; }

// doubles of one stage part at ppt points per thread
__host__ __device__ constexpr int stage_doubles(int ppt)
{
    return (kThreads * ppt + kThreads) / stage_parts(ppt);
}

// where the edge history of the aligned kernels starts: after both the stage
// and the exchange buffers, so that the prologue can fill it while the stage
// is in use
template <int PPT>
__device__ __forceinline__ constexpr int aligned_history_offset(int H)
{
    return stage_doubles(PPT) > 2 * kThreads * 2 * H ? stage_doubles(PPT) : 2 * kThreads * 2 * H;
}

// Level n0 of a region of E points that starts at periodic index G0w (in
// [0, N)) into wp[0 .. PPT) of every thread (thread tid holds region points
// tid*PPT ..), 0 past E.  Every thread issues all of its PPT loads before its
// first LDS write, so their latencies overlap.  Indices are wrapped into
// [0, N) (one subtraction when the grid is at least one region wide), so
// every load is in bounds; the values past E are loaded and dropped.
// early() runs once the loads are issued, before the first stage write.  Ends
// with a barrier: the stage may be reused at once.
template <int PPT, typename Early>
__device__ __forceinline__ void load_window(const double *__restrict__ uin, int64_t N,
                                            int64_t G0w, int E, int tid, double *stage,
                                            double *wp, Early early)
{
    constexpr int PARTS = stage_parts(PPT);
    constexpr int IT = PPT / PARTS;                 // loads per thread in one part
    constexpr int TP = kThreads / PARTS;            // threads whose points a part holds
    double v[PPT];
    if (N >= (int64_t)kThreads * PPT) {
#pragma unroll
        for (int it = 0; it < PPT; ++it) {
            int64_t g = G0w + it * kThreads + tid;
            if (g >= N) g -= N;
            v[it] = uin[g];
        }
    } else {
#pragma unroll
        for (int it = 0; it < PPT; ++it) v[it] = uin[(G0w + it * kThreads + tid) % N];
    }
    early();    // LDS writes of values loaded before these (outside the stage)
#pragma unroll
    for (int h = 0; h < PARTS; ++h) {
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int rr = i * kThreads + tid;      // point h*IT*kThreads + rr of the region
            stage[rr + rr / PPT] = h * IT * kThreads + rr < E ? v[h * IT + i] : 0.0;
        }
        __syncthreads();
        if (tid / TP == h) {
#pragma unroll
            for (int j = 0; j < PPT; ++j) wp[j] = stage[(tid - h * TP) * (PPT + 1) + j];
        }
        __syncthreads();
    }
}

// The inverse: the points wp[0 .. PPT) of every thread through the stage to
// out[r - lo] for the region points r in [lo, hi), coalesced
template <int PPT>
__device__ __forceinline__ void store_window(const double *wp, int tid, double *stage, int lo,
                                             int hi, double *__restrict__ out)
{
    constexpr int PARTS = stage_parts(PPT);
    constexpr int IT = PPT / PARTS;
    constexpr int TP = kThreads / PARTS;
#pragma unroll
    for (int h = 0; h < PARTS; ++h) {
        __syncthreads();
        if (tid / TP == h) {
#pragma unroll
            for (int j = 0; j < PPT; ++j) stage[(tid - h * TP) * (PPT + 1) + j] = wp[j];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int rr = i * kThreads + tid;
            const int r = h * IT * kThreads + rr;
            if (r >= lo && r < hi) out[r - lo] = stage[rr + rr / PPT];
        }
    }
}

template <int ORDER, bool LINEAR, bool FMA>
__global__ __launch_bounds__(kThreads) void k_step1d(Step1D a)
{
    constexpr int H = ORDER / 2;
    constexpr int M = (ORDER == 2) ? 2 : 3;
    constexpr int PPT = kPPT;
    extern __shared__ double lds[];
    double *stage = lds;                                  // one part of the stage (load_window)
    double *xch = lds;                                    // [2][kThreads][2H]  (aliases stage)
    double *eh = lds + 2 * kThreads * 2 * H;              // [D+s-1][NT][2][H]  (aliases stage)

    const int tid = threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.x * a.CH;
    const int64_t owned = (a.N - c0 < a.CH) ? (a.N - c0) : a.CH;
    const int sh = a.s * H;
    const int E = (int)owned + 2 * sh;                    // region length (<= kThreads*PPT)
    const int64_t G0 = c0 - sh;                           // unwrapped start (may be < 0)
    int64_t G0w = G0 % a.N;
    if (G0w < 0) G0w += a.N;

    // ---- level n0 of the region: coalesced loads -> LDS -> registers
    double w[PPT + 2 * H];
    load_window<PPT>(a.uin, a.N, G0w, E, tid, stage, w + H, [] {});
#pragma unroll
    for (int q = 0; q < H; ++q) { w[q] = 0.0; w[PPT + H + q] = 0.0; }

    // ---- tile bookkeeping of this thread's first point
    const int rp0 = tid * PPT;                            // region position of point 0
    const int64_t Gt = G0 + rp0;
    const int64_t tdiv = floordiv(Gt, a.W);
    const int64_t o0 = Gt - tdiv * a.W;                   // offset in its tile, [0, W)
    const int tl0 = (int)(tdiv - floordiv(G0, a.W));      // region-local tile index
    int64_t tp0 = tdiv % a.P;
    if (tp0 < 0) tp0 += a.P;                              // physical tile index
    const bool has_edge = (rp0 < E) && ((o0 < H) || (o0 + PPT - 1 + H >= a.W));
    const int64_t F = 2 * a.P;

    for (int t = 0; t < a.s; ++t) {
        const int64_t n = a.n0 + t;
        // ---- edge points of level n: LDS history for later steps, ring for later launches
        if (has_edge) {
            const int64_t slot = ring_slot(a, t);
            const bool pub = publish_level(a, t, a.s);
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                const int rp = rp0 + j;
                int64_t oj = o0 + j;
                int e = 0;
                while (oj >= a.W) { oj -= a.W; ++e; }
                const bool lo = oj < H, hi = oj >= a.W - H;
                if (rp < E && (lo || hi)) {
                    const int side = lo ? 0 : 1;
                    const int q = lo ? (int)oj : (int)(oj - (a.W - H));
                    if (t < a.s - 1)
                        eh[((t * a.NT + (tl0 + e)) * 2 + side) * H + q] = w[H + j];
                    if (pub && rp >= sh && rp < sh + owned) {
                        int64_t tp = tp0 + e;
                        while (tp >= a.P) tp -= a.P;
                        a.ring[((slot * a.P + tp) * 2 + side) * H + q] = w[H + j];
                    }
                }
            }
        }
        // ---- neighbour exchange: first and last H values of every thread
        double *buf = xch + (t & 1) * kThreads * 2 * H;
#pragma unroll
        for (int q = 0; q < H; ++q) {
            buf[tid * 2 * H + q] = w[H + q];
            buf[tid * 2 * H + H + q] = w[PPT + q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < H; ++q) {
            w[q] = (tid > 0) ? buf[(tid - 1) * 2 * H + H + q] : 0.0;
            w[PPT + H + q] = (tid < kThreads - 1) ? buf[(tid + 1) * 2 * H + q] : 0.0;
        }
        // ---- standard stencil on every point
        double res[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            double nb[2 * H];
#pragma unroll
            for (int q = 0; q < H; ++q) { nb[q] = w[j + q]; nb[H + q] = w[j + H + 1 + q]; }
            res[j] = update<ORDER, LINEAR, FMA>(nb, w[H + j], a);
        }
        // ---- points next to a tile edge: stencil again with AT halo values
        if (has_edge) {
            const int8_t *krow = a.delays + n * F;
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                const int rp = rp0 + j;
                int64_t oj = o0 + j;
                int e = 0;
                while (oj >= a.W) { oj -= a.W; ++e; }
                const bool valid = rp >= (t + 1) * H && rp < E - (t + 1) * H;   // inside the cone
                if (valid && (oj < H || oj >= a.W - H)) {
                    int64_t tp = tp0 + e;
                    while (tp >= a.P) tp -= a.P;
                    const int tl = tl0 + e;
                    double nb[2 * H];
#pragma unroll
                    for (int sl = 0; sl < 2 * H; ++sl) {
                        const int d = (sl < H) ? -(H - sl) : (sl - H + 1);
                        double v = w[H + j + d];
                        const int64_t od = oj + d;
                        if (od < 0 || od >= a.W) {
                            const int side = (od < 0) ? 0 : 1;
                            const int kk = krow[2 * tp + side];
                            if (kk > 0) {
                                const int q = (side == 0) ? (int)(od + H) : (int)(od - a.W);
                                const int stl = tl + (side ? 1 : -1);
                                int64_t stp = tp + (side ? 1 : -1);
                                if (stp < 0) stp += a.P;
                                if (stp >= a.P) stp -= a.P;
                                const int sside = 1 - side;
                                double vv[3] = {0.0, 0.0, 0.0};
#pragma unroll
                                for (int jj = 0; jj < M; ++jj) {
                                    if (jj == 0 || !a.stale) {
                                        const int64_t lev = n - kk - jj;
                                        if (lev >= a.n0)
                                            vv[jj] = eh[(((int)(lev - a.n0) * a.NT + stl) * 2 + sside) * H + q];
                                        else
                                            vv[jj] = a.ring[((ring_slot(a, lev - a.n0) * a.P + stp) * 2 + sside) * H + q];
                                    }
                                }
                                v = extrap<FMA>(kk, a.stale != 0, vv[0], vv[1], vv[2], M);
                            }
                        }
                        nb[sl] = v;
                    }
                    res[j] = update<ORDER, LINEAR, FMA>(nb, w[H + j], a);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < PPT; ++j) w[H + j] = res[j];
    }

    // ---- level n0+s of the owned points: registers -> LDS -> coalesced stores
    store_window<PPT>(w + H, tid, stage, sh, sh + (int)owned, a.uout + c0);
}


// Aligned variant: the tile width is a multiple of PPT and the region starts
// on a multiple of PPT, so every thread's PPT points lie in one tile.  A
// thread that starts a tile writes its left AT halo values into the left
// part of its register window, a thread that ends a tile its right ones, and
// then every point runs the same stencil (the split of section 5.2); the
// window slots replaced belong to this thread alone.
// FUSED = true: before the first step the launch copies into LDS the delay
// rows of its s steps for every tile of the region and the ring levels
// n0-D .. n0-1 of those tiles' edges; with the edges of the levels it
// computes recorded beside them, no step waits on a global load.
// FUSED = false: exactly one step per launch (delays and delayed levels read
// from global memory where used; no LDS edge history)
template <int ORDER, bool LINEAR, bool FMA, bool FUSED = true, int PPT = kPPT, bool DENSE = false>
__device__ __forceinline__ void step1d_aligned_body(const Step1D &a, int64_t chunk)
{
    constexpr int H = ORDER / 2;
    constexpr int M = (ORDER == 2) ? 2 : 3;
    extern __shared__ double lds[];
    double *stage = lds;                                  // one part of the stage (load_window)
    double *xch = lds;                                    // [2][kThreads][2H]  (aliases stage)
    double *eh = lds + aligned_history_offset<PPT>(H);    // [HR][NT][2][H]  (after both)

    const int tid = threadIdx.x;
    const int64_t c0 = chunk * a.CH;
    const int owned = (int)((a.N - c0 < a.CH) ? (a.N - c0) : a.CH);
    const int S = FUSED ? a.s : 1;
    const int sh = S * H;
    const int E = a.RL + owned + sh;                      // region length (<= kThreads*PPT)
    const int64_t G0 = c0 - a.RL;                         // unwrapped start, multiple of PPT
    int64_t G0w = G0 % a.N;
    if (G0w < 0) G0w += a.N;

    // ---- sources of the LDS copies of this launch's delays and of the ring
    // levels below n0 (eh row d holds level n0 - D + d; kd[(t*NT + tl)*2 +
    // side] the delay of region tile tl's face at level n0 + t).  A thread's
    // first element of each is loaded before the field and written to LDS
    // (which the stage does not overlap) as soon as the field loads are
    // issued: their latencies overlap, and no register holds them longer.
    const int D = a.D;
    // DENSE (the batched kernel, whose regions hold many tiles) keeps the edge
    // history as a ring of D + 2 levels instead of all D + s - 1, so that its
    // LDS does not grow with s: level n0 + x - D in row x mod HR
    const int HR = DENSE ? D + 2 : D + S - 1;
    auto hrow = [&](int x) -> int {                 // x in [0, 2 HR)
        if constexpr (DENSE) return x >= HR ? x - HR : x;
        else return x;
    };
    int8_t *kd = reinterpret_cast<int8_t *>(eh + (size_t)HR * a.NT * 2 * H);
    // AT halo values of the region's tile faces, one step at a time
    // (double-buffered): [2][NT][2][H], after the delay bytes
    double *hal = eh + (size_t)HR * a.NT * 2 * H + ((size_t)S * a.NT * 2 + 7) / 8;
    int64_t tb = floordiv(G0, a.W) % a.P;
    if (tb < 0) tb += a.P;
    const int nk = FUSED ? S * a.NT * 2 : 0;
    const int nr = FUSED ? D * a.NT * 2 * H : 0;
    auto kd_src = [&](int e) -> int64_t {
        const int side = e & 1;
        const int tl = (e >> 1) % a.NT;
        const int t = (e >> 1) / a.NT;
        const int64_t tp = (tb + tl) % a.P;
        return (a.n0 + t) * (2 * a.P) + 2 * tp + side;
    };
    auto eh_src = [&](int e) -> int64_t {                 // -1: a level before the start
        const int q = e % H;
        const int side = (e / H) & 1;
        const int tl = (e / (2 * H)) % a.NT;
        const int d = (e / (2 * H)) / a.NT;
        const int64_t lev = a.n0 - D + d;
        if (lev < 0) return -1;
        const int64_t tp = (tb + tl) % a.P;
        return ((ring_slot(a, lev - a.n0) * a.P + tp) * 2 + side) * H + q;
    };
    int8_t k_first = 0;
    double e_first = 0.0;
    int64_t e_first_at = -1;
    if constexpr (FUSED) {
        if (tid < nk) k_first = a.delays[kd_src(tid)];
        if (tid < nr) {
            e_first_at = eh_src(tid);
            if (e_first_at >= 0) e_first = a.ring[e_first_at];
        }
    }

    double w[PPT + 2 * H];
    load_window<PPT>(a.uin, a.N, G0w, E, tid, stage, w + H, [&] {
        if constexpr (FUSED) {
            if (tid < nk) kd[tid] = k_first;
            if (e_first_at >= 0) eh[tid] = e_first;
        }
    });
#pragma unroll
    for (int q = 0; q < H; ++q) { w[q] = 0.0; w[PPT + H + q] = 0.0; }

    if constexpr (FUSED) {
        for (int e = tid + kThreads; e < nk; e += kThreads) kd[e] = a.delays[kd_src(e)];
        for (int e = tid + kThreads; e < nr; e += kThreads) {
            const int64_t at = eh_src(e);
            if (at >= 0) eh[e] = a.ring[at];
        }
        if (DENSE) __syncthreads();   // the dense halo table reads them before step 0's barrier
    }

    const int rp0 = tid * PPT;
    const int64_t Gt = G0 + rp0;
    const int64_t tdiv = floordiv(Gt, a.W);
    const int o0 = (int)(Gt - tdiv * a.W);                // multiple of PPT
    const int tl0 = (int)(tdiv - floordiv(G0, a.W));
    int64_t tp0 = tdiv % a.P;
    if (tp0 < 0) tp0 += a.P;
    const int64_t tpl = tp0 == 0 ? a.P - 1 : tp0 - 1;     // left / right neighbour tiles
    const int64_t tpr = tp0 == a.P - 1 ? 0 : tp0 + 1;
    // tile edges of every thread with points in the region: their values may
    // still be inside the dependency cone of the owned points even when the
    // thread sticks out of the region
    const bool lo_edge = o0 == 0 && rp0 < E;
    const bool hi_edge = o0 + PPT == a.W && rp0 < E;
    const bool owns = rp0 >= a.RL && rp0 < a.RL + owned;
    const int64_t F = 2 * a.P;

    for (int t = 0, tr = 0; t < S; ++t, tr = (DENSE && tr + 1 == HR) ? 0 : tr + 1) {
        const int64_t n = a.n0 + t;
        const int64_t slot = ring_slot(a, t);
        // ---- record this level's tile edges (LDS history; ring when owned)
        if (lo_edge || hi_edge) {
            const bool pub = publish_level(a, t, S);
#pragma unroll
            for (int q = 0; q < H; ++q) {
                if (lo_edge) {
                    if (FUSED && t < S - 1) eh[((hrow(tr + D) * a.NT + tl0) * 2 + 0) * H + q] = w[H + q];
                    if (pub && owns) a.ring[((slot * a.P + tp0) * 2 + 0) * H + q] = w[H + q];
                }
                if (hi_edge) {
                    if (FUSED && t < S - 1) eh[((hrow(tr + D) * a.NT + tl0) * 2 + 1) * H + q] = w[PPT + q];
                    if (pub && owns) a.ring[((slot * a.P + tp0) * 2 + 1) * H + q] = w[PPT + q];
                }
            }
        }
        // ---- neighbour exchange
        double *buf = xch + (t & 1) * kThreads * 2 * H;
#pragma unroll
        for (int q = 0; q < H; ++q) {
            buf[tid * 2 * H + q] = w[H + q];
            buf[tid * 2 * H + H + q] = w[PPT + q];
        }
        // ---- DENSE (regions holding many tile edges, as in the batched form):
        // the AT halo values of every tile face of the region for this step
        // (section 2, Eqs. (1)-(2)), one lane per (tile, side, point) instead of
        // a divergent branch in every edge thread; they read only levels below
        // n (k >= 1), all recorded before the previous barrier
        double *halt = hal + (t & 1) * (a.NT * 2 * H);
        if constexpr (FUSED && DENSE) {
            for (int e = tid; e < a.NT * 2 * H; e += kThreads) {
                const int q = e % H, side = (e / H) & 1, tl = e / (2 * H);
                const int stl = side == 0 ? tl - 1 : tl + 1;     // the tile the values come from
                const int kk = kd[(t * a.NT + tl) * 2 + side];
                if (kk > 0 && stl >= 0 && stl < a.NT) {
                    double vv[3] = {0.0, 0.0, 0.0};
#pragma unroll
                    for (int jj = 0; jj < M; ++jj)
                        if (jj == 0 || !a.stale)
                            vv[jj] = eh[((hrow(tr + D - kk - jj) * a.NT + stl) * 2 + (1 - side)) * H + q];
                    halt[e] = extrap<FMA>(kk, a.stale != 0, vv[0], vv[1], vv[2], M);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < H; ++q) {
            w[q] = (tid > 0) ? buf[(tid - 1) * 2 * H + H + q] : 0.0;
            w[PPT + H + q] = (tid < kThreads - 1) ? buf[(tid + 1) * 2 * H + q] : 0.0;
        }
        // ---- AT halo approximation at tile edges (k = 0: the raw neighbour stays)
        if (lo_edge || hi_edge) {
            int kl = 0, kr = 0;                                       // tid 0: no left source
            if constexpr (FUSED) {
                if (lo_edge && tid > 0) kl = kd[(t * a.NT + tl0) * 2 + 0];
                if (hi_edge) kr = kd[(t * a.NT + tl0) * 2 + 1];
            } else {
                const int8_t *krow = a.delays + n * F;
                if (lo_edge && tid > 0) kl = krow[2 * tp0 + 0];
                if (hi_edge) kr = krow[2 * tp0 + 1];
            }
            if constexpr (FUSED && DENSE) {
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    if ((side == 0 ? kl : kr) > 0) {
#pragma unroll
                        for (int q = 0; q < H; ++q) {
                            const double hv = halt[(tl0 * 2 + side) * H + q];
                            if (side == 0) w[q] = hv;
                            else w[PPT + H + q] = hv;
                        }
                    }
                }
            } else {
                // both tile sides in one pass: a lane that starts a tile takes its
                // left halo, one that ends a tile its right halo, with the same
                // arithmetic; a lane that does both (a tile PPT points wide) takes
                // its right halo in a second pass
                const bool both = lo_edge && hi_edge;
#pragma unroll
                for (int pass = 0; pass < 2; ++pass) {
                    const bool left = pass == 0 && lo_edge;
                    const int kk = pass == 0 ? (lo_edge ? kl : kr) : (both ? kr : 0);
                    if (kk > 0) {
                        const int stl = left ? tl0 - 1 : tl0 + 1;
                        const int64_t stp = left ? tpl : tpr;
                        const int sside = left ? 1 : 0;
#pragma unroll
                        for (int q = 0; q < H; ++q) {
                            double vv[3] = {0.0, 0.0, 0.0};
#pragma unroll
                            for (int jj = 0; jj < M; ++jj) {
                                if (jj == 0 || !a.stale) {
                                    const int dl = t - kk - jj;        // level n - k - jj, from n0
                                    vv[jj] = FUSED
                                        ? eh[((hrow(tr + D - kk - jj) * a.NT + stl) * 2 + sside) * H + q]
                                        : a.ring[((ring_slot(a, dl) * a.P + stp) * 2 + sside) * H + q];
                                }
                            }
                            const double hv = extrap<FMA>(kk, a.stale != 0, vv[0], vv[1], vv[2], M);
                            if (left) w[q] = hv;
                            else w[PPT + H + q] = hv;
                        }
                    }
                }
            }
        }
        // ---- the standard stencil on every point, each new value formed after
        // the last stencil that reads its old value (same operations as update())
        step_window<ORDER, LINEAR, FMA, PPT>(w, a);
        // every intermediate level of the owned points, straight from registers
        // (used to rebuild a checkpoint segment for the adjoint)
        if (FUSED && a.levels && owns && t + 1 < S) {
            double *dst = a.levels + (int64_t)(t + 1) * a.N + c0 + (rp0 - a.RL);
#pragma unroll
            for (int j = 0; j < PPT; ++j) dst[j] = w[H + j];
        }
    }

    store_window<PPT>(w + H, tid, stage, a.RL, a.RL + owned, a.uout + c0);
}

// Five waves per SIMD (at most 96 VGPRs): with the stage in two parts the
// LDS of a 16-point region allows five workgroups per CU, and the step loop
// fits the registers without spilling
template <int ORDER, bool LINEAR, bool FMA, int PPT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(5)))
void k_step1d_aligned(Step1D a)
{
    step1d_aligned_body<ORDER, LINEAR, FMA, true, PPT>(a, blockIdx.x);
}

// one step per launch (the plain form): 8 points per thread, a smaller
// workgroup footprint and more workgroups in flight
template <int ORDER, bool LINEAR, bool FMA>
__global__ __launch_bounds__(kThreads) void k_step1d_plain(Step1D a)
{
    step1d_aligned_body<ORDER, LINEAR, FMA, false, kPPTPlain>(a, blockIdx.x);
}

// Batched form: workgroup b advances chunk tbl[b].y of instance tbl[b].x;
// instance descriptors carry each instance's grid, ring, delays and
// coefficients; flip = 1 swaps the field pointers (ping-pong launches).
template <int ORDER, bool LINEAR, bool FMA, int PPT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(5)))
void k_step1d_aligned_batch(const Step1D *descs, const int2 *tbl, int64_t n0, int flip)
{
    const int2 e = tbl[blockIdx.x];
    Step1D a = descs[e.x];
    a.n0 = n0;
    a.slot0 = (int32_t)(n0 % a.R);    // once per workgroup (uniform)
    if (flip) {
        const double *t = a.uin;
        a.uin = a.uout;
        a.uout = const_cast<double *>(t);
    }
    step1d_aligned_body<ORDER, LINEAR, FMA, true, PPT, true>(a, e.y);
}

}  // namespace

int step1d_points_per_thread() { return kPPT; }
int step1d_plain_points_per_thread() { return kPPTPlain; }

size_t step1d_lds_bytes(int order, int s, int NT, int D, int ppt, bool dense)
{
    const int H = order / 2;
    const size_t stage = (size_t)stage_doubles(ppt);
    const size_t xch = (size_t)2 * kThreads * 2 * H;
    // the stage part or the exchange buffers, then the edge history of D + s - 1
    // levels (the batched kernel's dense form: a ring of D + 2), the delays
    // (bytes) and, for the dense form, the AT halo table [2][NT][2][H] (the general kernel's layout, whose history
    // follows the exchange buffers, fits in the same size)
    const size_t rows = dense ? (size_t)D + 2 : (size_t)(D + s - 1);      // the edge history
    const size_t hist = rows * NT * 2 * H + ((size_t)s * NT * 2 + 7) / 8 +
                        (dense ? (size_t)2 * NT * 2 * H : 0);
    return 8 * ((stage > xch ? stage : xch) + hist);
}

hipError_t launch_step1d(const Step1D &a, int order, bool linear, bool aligned, bool fma, int ppt,
                         int64_t nblocks, hipStream_t st)
{
    const bool plain = aligned && a.s == 1 && ppt == kPPTPlain;
    size_t lds = step1d_lds_bytes(order, a.s, a.NT, a.D, aligned ? ppt : kPPT, false);
    if (plain) {
        const size_t stage = (size_t)stage_doubles(kPPTPlain);
        const size_t xch = (size_t)2 * kThreads * order;
        lds = 8 * (stage > xch ? stage : xch);
    }
    dim3 grid((unsigned)nblocks), block(kThreads);
#define AT_L(K, O, LI, F) hipLaunchKernelGGL((K<O, LI, F>), grid, block, lds, st, a)
#define AT_LP(O, LI, F, P) hipLaunchKernelGGL((k_step1d_aligned<O, LI, F, P>), grid, block, lds, st, a)
#define AT_DISPATCH(L3)                                                                  \
    do {                                                                                 \
        if (order == 2) {                                                                \
            if (linear) { if (fma) L3(2, true, true); else L3(2, true, false); }         \
            else { if (fma) L3(2, false, true); else L3(2, false, false); }              \
        } else {                                                                         \
            if (linear) { if (fma) L3(4, true, true); else L3(4, true, false); }         \
            else { if (fma) L3(4, false, true); else L3(4, false, false); }              \
        }                                                                                \
    } while (0)
#define L_PLAIN(O, LI, F) AT_L(k_step1d_plain, O, LI, F)
#define L_GEN(O, LI, F) AT_L(k_step1d, O, LI, F)
#define L_A16(O, LI, F) AT_LP(O, LI, F, 16)
#define L_A8(O, LI, F) AT_LP(O, LI, F, 8)
#define L_A4(O, LI, F) AT_LP(O, LI, F, 4)
    if (plain) AT_DISPATCH(L_PLAIN);
    else if (!aligned) AT_DISPATCH(L_GEN);
    else if (ppt == 16) AT_DISPATCH(L_A16);
    else if (ppt == 8) AT_DISPATCH(L_A8);
    else if (ppt == 4) AT_DISPATCH(L_A4);
    else return hipErrorInvalidValue;
#undef L_PLAIN
#undef L_GEN
#undef L_A16
#undef L_A8
#undef L_A4
#undef AT_DISPATCH
#undef AT_LP
#undef AT_L
    return hipGetLastError();
}

hipError_t launch_step1d_batch(const Step1D *descs, const int2 *tbl, int64_t nblocks, int order,
                               bool linear, bool fma, int ppt, int64_t n0, int flip, size_t lds,
                               hipStream_t st)
{
    dim3 grid((unsigned)nblocks), block(kThreads);
#define AT_BATCH(O, LI, F, P) hipLaunchKernelGGL((k_step1d_aligned_batch<O, LI, F, P>), grid, block, lds, st, descs, tbl, n0, flip)
#define AT_BATCH_P(O, LI, F)                                                             \
    do {                                                                                 \
        if (ppt == 16) AT_BATCH(O, LI, F, 16);                                           \
        else if (ppt == 8) AT_BATCH(O, LI, F, 8);                                        \
        else AT_BATCH(O, LI, F, 4);                                                      \
    } while (0)
    if (order == 2) {
        if (linear) { if (fma) AT_BATCH_P(2, true, true); else AT_BATCH_P(2, true, false); }
        else { if (fma) AT_BATCH_P(2, false, true); else AT_BATCH_P(2, false, false); }
    } else {
        if (linear) { if (fma) AT_BATCH_P(4, true, true); else AT_BATCH_P(4, true, false); }
        else { if (fma) AT_BATCH_P(4, false, true); else AT_BATCH_P(4, false, false); }
    }
#undef AT_BATCH_P
#undef AT_BATCH
    return hipGetLastError();
}

}  // namespace atk
