// Discrete adjoint of the 1D AT stepper (reverse mode), one launch per step.
//
// The forward step at level n is u'_i = u_i + dt*(nu*D2_i - a_i*D1_i) with
// the central stencils of section 3.2 and, at a tile edge, halo values
// extrapolated in time from the neighbour edge's levels n-k-j (section 2,
// Eqs. (1)-(2)).  Its transpose, given lambda^{n+1} = dJ/du^{n+1}:
//   * centre:     lambda_i * (1 + dt*(nu*dD2/du - D1))     (Burgers; linear: no -D1)
//   * neighbour:  lambda_i * dt*(nu*dD2/dnb_s - a_i*dD1/dnb_s) flows to the
//     point at stencil slot s when it lies in the same tile, otherwise to the
//     halo's source edge point at the levels n-k-j with the extrapolation
//     weights dH/dv_j ((k+1, -k) for two levels; ((k+1)(k+2)/2, -k(k+2),
//     k(k+1)/2) for three; 1 for the stale halo or k = 0);
//   * dJ/dnu += lambda_i * dt * D2_i.
// The halo contributions ("mu") of step n are needed by earlier levels of the
// neighbour's edge, so they are kept in a small ring over the last L+m
// steps and GATHERED by the owner of each edge point (no atomics): at
// reverse step n an edge point adds, for n' = n .. n+L+m-1, the weight for
// j = n' - k[n'] - n of every mu^{n'} of the face it feeds.  mu^n itself is
// recomputed in place from lambda^{n+1} and u^n, which the workgroup holds.
// Each workgroup keeps one compensated dJ/dnu accumulator across launches.
#include "at_internal.h"

namespace atk {

namespace {

constexpr int kPPA = 4;                       // points per thread
constexpr int kCHA = kThreads * kPPA;         // points per workgroup

template <int ORDER>
struct Partials {
    double g1[ORDER], g2[ORDER], g2u;
};

template <int ORDER>
__device__ __forceinline__ Partials<ORDER> partials(double c1, double c2)
{
    Partials<ORDER> p;
    if constexpr (ORDER == 2) {
        p.g1[0] = -c1; p.g1[1] = c1;
        p.g2[0] = c2;  p.g2[1] = c2;
        p.g2u = -2.0 * c2;
    } else {
        p.g1[0] = c1;  p.g1[1] = -8.0 * c1; p.g1[2] = 8.0 * c1; p.g1[3] = -c1;
        p.g2[0] = -c2; p.g2[1] = 16.0 * c2; p.g2[2] = 16.0 * c2; p.g2[3] = -c2;
        p.g2u = -30.0 * c2;
    }
    return p;
}

__device__ __forceinline__ double extrap(int kk, bool stale, double v0, double v1, double v2,
                                         int M)
{
    if (stale) return v0;
    const double dk = (double)kk;
    const double d1 = v0 - v1;
    if (M == 2) return v0 + dk * d1;
    const double w2 = 0.5 * dk * (dk + 1.0);
    return (v0 + dk * d1) + w2 * (d1 - (v1 - v2));
}

// dH/dv_j
__device__ __forceinline__ double hweight(int kk, bool stale, int j, int M)
{
    if (kk == 0 || stale) return j == 0 ? 1.0 : 0.0;
    const double dk = (double)kk;
    if (M == 2) return j == 0 ? 1.0 + dk : -dk;
    const double w2 = 0.5 * dk * (dk + 1.0);
    if (j == 0) return (1.0 + dk) + w2;
    if (j == 1) return -dk - 2.0 * w2;
    return w2;
}

template <int ORDER, bool LINEAR>
__global__ __launch_bounds__(kThreads) void k_adj1d(Adj1D a)
{
    constexpr int H = ORDER / 2;
    constexpr int M = (ORDER == 2) ? 2 : 3;
    constexpr int NS = 2 * H;                 // stencil slots: offsets -H..-1, 1..H
    __shared__ double sl[kCHA + 2 * H], su[kCHA + 2 * H];
    __shared__ double red[kThreads / 64][2];

    const int tid = threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.x * kCHA;
    const int64_t owned = (a.N - c0 < kCHA) ? (a.N - c0) : kCHA;
    const int64_t F = 2 * a.P;
    const Partials<ORDER> pd = partials<ORDER>(a.c1, a.c2);
    const bool stale = a.stale != 0;

    // all loads issued before the first use (one round trip, not one per pass)
    double vl[kPPA + 1], vu[kPPA + 1];
#pragma unroll
    for (int it = 0; it <= kPPA; ++it) {
        const int r = it * kThreads + tid;
        vl[it] = vu[it] = 0.0;
        if (r < owned + 2 * H) {
            int64_t g = c0 - H + r;
            if (g < 0) g += a.N;
            if (g >= a.N) g -= a.N;
            vl[it] = a.lam_in[g];
            vu[it] = a.u[g];
        }
    }
#pragma unroll
    for (int it = 0; it <= kPPA; ++it) {
        const int r = it * kThreads + tid;
        if (r < owned + 2 * H) { sl[r] = vl[it]; su[r] = vu[it]; }
    }
    __syncthreads();

    // P_s(u) = dt*(nu*g2[s] - a*g1[s]): sensitivity of u'_i to its slot-s neighbour
    auto Ps = [&](int s, double u) -> double {
        const double adv = LINEAR ? a.cadv : u;
        double g1 = pd.g1[0], g2 = pd.g2[0];     // select without indexing a register array
#pragma unroll
        for (int i = 1; i < NS; ++i) {
            g1 = (s == i) ? pd.g1[i] : g1;
            g2 = (s == i) ? pd.g2[i] : g2;
        }
        return a.dt * (a.nu * g2 - adv * g1);
    };
    // mu^n of face (tile tf, side sd), halo index q, from the LDS copy whose
    // index ri is the first point of the tile behind the face (side 0) or the
    // last one (side 1).
    auto mu_now = [&](int sd, int q, int ri) -> double {
        double m = 0.0;
#pragma unroll
        for (int e = 0; e < H; ++e) {
            if (sd == 0 && e <= q) m += sl[ri + e] * Ps(q - e, su[ri + e]);
            if (sd == 1 && e <= H - 1 - q) m += sl[ri - e] * Ps(H + q + e, su[ri - e]);
        }
        return m;
    };

    Acc gacc{0.0, 0.0};
    const int W32 = (int)a.W;
    // tile index and offset of this thread's first point; later points step by kThreads
    const int64_t g0 = c0 + tid;
    int64_t t = g0 / a.W;
    int o_ = (int)(g0 - t * a.W);
#pragma unroll
    for (int it = 0; it < kPPA; ++it) {
        const int l = it * kThreads + tid;
        if (it > 0) {                       // advance by kThreads points without dividing
            o_ += kThreads;
            while (o_ >= W32) { o_ -= W32; ++t; }
        }
        if (l >= owned) break;
        const int64_t g = c0 + l;
        const int64_t o = o_;
        const int r = l + H;
        const double u = su[r];
        // neighbours at level n, AT halo where the stencil leaves the tile
        double nb[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int d = (s < H) ? -(H - s) : (s - H + 1);
            double v = su[r + d];
            const int64_t od = o + d;
            if (od < 0 || od >= a.W) {
                const int side = od < 0 ? 0 : 1;
                const int kk = a.delays[a.n * F + 2 * t + side];
                if (kk > 0) {
                    const int q = side == 0 ? (int)(od + H) : (int)(od - a.W);
                    int64_t stp = t + (side ? 1 : -1);
                    if (stp < 0) stp += a.P;
                    if (stp >= a.P) stp -= a.P;
                    double vv[3] = {0.0, 0.0, 0.0};
#pragma unroll
                    for (int j = 0; j < M; ++j) {
                        if (j == 0 || !stale) {
                            const int64_t lev = a.n - kk - j;
                            // record mode keeps every level: slot = level
                            vv[j] = a.ring[((lev * a.P + stp) * 2 + (1 - side)) * H + q];
                        }
                    }
                    v = extrap(kk, stale, vv[0], vv[1], vv[2], M);
                }
            }
            nb[s] = v;
        }
        double D1, D2;
        if constexpr (ORDER == 2) {
            D1 = (nb[1] - nb[0]) * a.c1;
            D2 = ((nb[1] - 2.0 * u) + nb[0]) * a.c2;
        } else {
            D1 = (8.0 * (nb[2] - nb[1]) - (nb[3] - nb[0])) * a.c1;
            D2 = ((16.0 * (nb[2] + nb[1]) - 30.0 * u) - (nb[3] + nb[0])) * a.c2;
        }
        const double lam = sl[r];
        const double du = 1.0 + a.dt * (a.nu * pd.g2u - (LINEAR ? 0.0 : D1));
        double acc = lam * du;
        // same-tile points i = g - d that see g at their slot for offset d
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int d = (s < H) ? -(H - s) : (s - H + 1);
            const int64_t oi = o - d;
            if (oi >= 0 && oi < a.W) acc += sl[r - d] * Ps(s, su[r - d]);
        }
        // delayed halo contributions gathered over steps n .. n+L+m-1
        for (int side = 0; side < 2; ++side) {
            // side 0: g is in the tile's last h points, feeding face (t+1, low side);
            // side 1: g is in the first h points, feeding face (t-1, high side)
            const bool feeds = side == 0 ? (o >= a.W - H) : (o < H);
            if (!feeds) continue;
            int64_t tf = t + (side == 0 ? 1 : -1);
            if (tf < 0) tf += a.P;
            if (tf >= a.P) tf -= a.P;
            const int fs = side == 0 ? 0 : 1;                 // side of that face
            const int q = side == 0 ? (int)(o - (a.W - H)) : (int)o;
            // LDS index of the first (fs 0) / last (fs 1) point of tile tf
            const int ri = side == 0 ? r + (H - q) : r - (q + 1);
            for (int dn = 0; dn < a.L + M; ++dn) {
                const int64_t n2 = a.n + dn;
                if (n2 >= a.nsteps_total) break;
                const int kk = a.delays[n2 * F + 2 * tf + fs];
                const int j = dn - kk;
                const int need = (kk == 0 || stale) ? 1 : M;
                if (j < 0 || j >= need) continue;
                int64_t ms = a.mslot0 + dn;
                if (ms >= a.Rmu) ms -= a.Rmu;
                const double m = dn == 0 ? mu_now(fs, q, ri)
                                         : a.mu[((ms * a.P + tf) * 2 + fs) * H + q];
                acc += hweight(kk, stale, j, M) * m;
            }
        }
        a.lam_out[g] = acc;
        acc_add(gacc, lam * (a.dt * D2));
        // publish mu^n of this tile's faces (owners: first and last point of the tile)
        if (o == 0)
            for (int q = 0; q < H; ++q)
                a.mu[(((int64_t)a.mslot0 * a.P + t) * 2 + 0) * H + q] = mu_now(0, q, r);
        if (o == a.W - 1)
            for (int q = 0; q < H; ++q)
                a.mu[(((int64_t)a.mslot0 * a.P + t) * 2 + 1) * H + q] = mu_now(1, q, r);
    }
    gacc = wave_acc(gacc);
    const int lane = tid & 63, wv = tid >> 6;
    if (lane == 0) { red[wv][0] = gacc.s; red[wv][1] = gacc.c; }
    __syncthreads();
    if (tid == 0) {
        Acc S{a.gnu[blockIdx.x * 2], a.gnu[blockIdx.x * 2 + 1]};
        for (int q = 0; q < kThreads / 64; ++q) acc_merge(S, Acc{red[q][0], red[q][1]});
        a.gnu[blockIdx.x * 2] = S.s;
        a.gnu[blockIdx.x * 2 + 1] = S.c;
    }
}

}  // namespace

int adj1d_points_per_block() { return kCHA; }

hipError_t launch_adj1d(const Adj1D &a, int order, bool linear, int64_t nblocks, hipStream_t st)
{
    dim3 grid((unsigned)nblocks), block(kThreads);
    if (order == 2) {
        if (linear) hipLaunchKernelGGL((k_adj1d<2, true>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((k_adj1d<2, false>), grid, block, 0, st, a);
    } else {
        if (linear) hipLaunchKernelGGL((k_adj1d<4, true>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((k_adj1d<4, false>), grid, block, 0, st, a);
    }
    return hipGetLastError();
}

}  // namespace atk
