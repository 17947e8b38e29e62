// Internal declarations shared by the kernel and host translation units of
// libat.so.  Not part of the ABI (see include/at.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace atk {

constexpr int kThreads = 256;     // workgroup size of every stencil kernel (4 wave64)
constexpr int kMaxFuse = 64;      // largest steps-per-launch the ring is sized for
constexpr int kRedBlocks = 1024;  // workgroups of the first reduction pass

// Arguments of one launch of the 1D stepper: s steps n0 .. n0+s-1.
struct Step1D {
    const double *uin;        // level n0, double[N]
    double *uout;             // level n0+s, double[N]
    double *ring;             // edge levels: [R][P][2][h]
    const int8_t *delays;     // k[n][2P]
    int64_t N, P, W;
    int64_t n0;
    int64_t CH;               // points owned by one workgroup
    int32_t s;                // steps in this launch
    int32_t R;                // ring levels
    int32_t NT;               // region-local tile slots in the LDS edge history
    int32_t stale;            // 1: halo = level n-k without extrapolation
    int32_t publish;          // ring writes of level edges: 0 none, 1 every level,
                              // 2 the last D levels of the launch (1D)
    int32_t RL;               // left rim of the loaded region (aligned kernel)
    int32_t slot0;            // n0 mod R (ring slot of level n0)
    int32_t D;                // delayed levels below n0 a step may read: L + m - 1
    double *levels;           // optional: levels n0+1 .. n0+s-1 stored at levels + t*N (aligned kernel)
    double nu, dt, c1, c2, cadv;
    double A1, A2;            // contracted mode: dt*c1, dt*(nu*c2)
};

// Reverse (adjoint) step at level n of the 1D stepper.
struct Adj1D {
    const double *lam_in;     // lambda^{n+1}
    double *lam_out;          // lambda^n
    const double *u;          // u^n
    const double *ring;       // full edge history (record mode): [R][P][2][h]
    double *mu;               // halo adjoints: [Rmu][P][2][h]
    const int8_t *delays;     // k[n][2P]
    double *gnu;              // per-workgroup compensated dJ/dnu: [nblocks][2]
    int64_t N, P, W;
    int64_t n;
    int64_t nsteps_total;     // steps of the recorded run (gather window bound)
    int32_t R, Rmu, L, stale;
    int32_t mslot0;           // n mod Rmu
    int32_t pad0;
    double nu, dt, c1, c2, cadv;
};

// S reverse steps of the 1D stepper in one launch (tile width a multiple of
// the points per thread): levels nt-1 .. nt-S over overlapped regions.
struct AdjF {
    const double *lam_in;     // lambda^{nt}
    double *lam_out;          // lambda^{nt-S}
    const double *seg;        // u levels: level n at seg + (n - seg_n0) * N
    const double *ring;       // full edge history (record mode): [levels][P][2][h]
    double *mu;               // halo adjoints: [Rmu][P][2][h], level n in slot n mod Rmu
    const int8_t *delays;     // k[n][2P]
    double *gnu;              // per-workgroup compensated dJ/dnu: [nblocks][2]
    int64_t N, P, W, CH;
    int64_t nt, seg_n0, nsteps_total;
    int32_t S, Rmu, L, stale, RL, NT;
    double nu, dt, c1, c2, cadv;
};

// Weakly-synchronous 1D run (emergent delays): one workgroup per tile.
struct Ws1D {
    double *u;                // field, advanced in place: double[N]
    double *ring;             // edge levels: [R][P][2][h], level n in slot n mod R
    int32_t *cnt;             // newest announced level per tile edge: [P][2] (-1: none)
    int32_t *err;             // 0, or 1 once a wait passed the spin limit
    int8_t *delays;           // delays used, recorded: k[n][2P]
    int64_t P, W, n0, nsteps;
    int64_t spin_limit;       // polls of a counter before a wait gives up
    int32_t R, L, stale, jitter;
    uint64_t seed;            // idle-time noise
    Step1D coef;              // nu, dt, c1, c2, cadv of the update
};

// Neumaier-compensated accumulator used by the reductions.
struct Acc {
    double s, c;
};

__device__ __forceinline__ void acc_add(Acc &a, double x)
{
    const double t = a.s + x;
    if (fabs(a.s) >= fabs(x)) a.c += (a.s - t) + x;
    else a.c += (x - t) + a.s;
    a.s = t;
}

__device__ __forceinline__ void acc_merge(Acc &a, const Acc &b)
{
    acc_add(a, b.s);
    a.c += b.c;
}

__device__ __forceinline__ Acc wave_acc(Acc a)
{
    for (int off = 32; off > 0; off >>= 1) {
        Acc b;
        b.s = __shfl_down(a.s, off, 64);
        b.c = __shfl_down(a.c, off, 64);
        acc_merge(a, b);
    }
    return a;
}

// Launchers (defined in the .hip files); return hipError_t of the launch.
hipError_t launch_delays(int8_t *out, int64_t nsteps, int64_t F, int L, int m, int dist,
                         uint64_t seed, hipStream_t st);
hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t st);
hipError_t launch_poison(double *ring, int64_t R, int64_t lev, int s0, int nlive, hipStream_t st);
hipError_t launch_copy(double *dst, const double *src, int64_t n, hipStream_t st);
size_t step1d_lds_bytes(int order, int s, int NT, int D, int ppt, bool dense);
int step1d_points_per_thread();
int step1d_plain_points_per_thread();
hipError_t launch_step1d(const Step1D &a, int order, bool linear, bool aligned, bool fma, int ppt,
                         int64_t nblocks, hipStream_t st);
size_t step1d_whole_lds_bytes(int order, int64_t P, int D);
int step1d_whole_ppt(int64_t N, int64_t W, int64_t P, int order, int D);
hipError_t launch_step1d_whole(const Step1D &a, int order, bool linear, bool fma, int ppt,
                               hipStream_t st);
hipError_t launch_step1d_batch(const Step1D *descs, const int2 *tbl, int64_t nblocks, int order,
                               bool linear, bool fma, int ppt, int64_t n0, int flip, size_t lds,
                               hipStream_t st);
hipError_t launch_adj1d(const Adj1D &a, int order, bool linear, int64_t nblocks,
                        hipStream_t st);
int adj1d_points_per_block();
hipError_t launch_adj1d_fused(const AdjF &a, int order, bool linear, int ppt, int64_t nblocks,
                              size_t lds, hipStream_t st);
size_t adj1d_fused_lds_bytes(int order, int S, int NT, int L);
bool ws1d_shape(int64_t W, int h, int *nt, int *ppt);
int64_t ws1d_max_tiles(int order, bool linear, int64_t W);
hipError_t launch_ws_init(int32_t *cnt, int64_t n, int32_t v, int32_t *err, hipStream_t st);
hipError_t launch_ws1d(const Ws1D &a, int order, bool linear, hipStream_t st);
hipError_t launch_gnu_final(const double *part, int64_t nparts, double *out, hipStream_t st);
hipError_t launch_stats(const double *u, int64_t n, double *part, double *out4, hipStream_t st);
hipError_t launch_loss(const double *u, const double *t, double *lam, int64_t n, double *part,
                       double *J, hipStream_t st);

}  // namespace atk
