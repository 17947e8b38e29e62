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
            // summed newest level first (the order in which the fused reverse
            // launches accumulate them), then added to acc as one term
            double gsum = 0.0;
            for (int dn = a.L + M - 1; dn >= 0; --dn) {
                const int64_t n2 = a.n + dn;
                if (n2 >= a.nsteps_total) continue;
                const int kk = a.delays[n2 * F + 2 * tf + fs];
                const int j = dn - kk;
                const int need = (kk == 0 || stale) ? 1 : M;
                if (j < 0 || j >= need) continue;
                int64_t ms = a.mslot0 + dn;
                if (ms >= a.Rmu) ms -= a.Rmu;
                const double m = dn == 0 ? mu_now(fs, q, ri)
                                         : a.mu[((ms * a.P + tf) * 2 + fs) * H + q];
                gsum += hweight(kk, stale, j, M) * m;
            }
            acc += gsum;
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


__device__ __forceinline__ int64_t fdiv(int64_t a, int64_t b)
{
    int64_t q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}


// S reverse steps in one launch.  The workgroup's region is its owned chunk
// plus S*h points on each side; every reverse step reads lambda and u within
// h points (across a tile face: the mu of that face, computed from points
// within h of it), so after S steps the owned points are exact while the
// rims have gone stale, as in the forward fused launches.  lambda stays in
// registers; each step reads its level of u (the recomputed segment), the
// next level's loads in flight meanwhile.  In LDS: the delay rows of the
// launch's gather window, the record-mode ring levels that the forward
// halos of these steps read, and the mu of every face of the region for
// levels nt-S .. nt-1 (computed here) and nt .. nt+L+m-2 (from the mu ring).
// Each point's lambda^n is summed in the same order as the one-step kernel.
template <int ORDER, bool LINEAR, int PPT>
__global__ __launch_bounds__(kThreads) void k_adj1d_fused(AdjF a)
{
    constexpr int H = ORDER / 2;
    constexpr int M = (ORDER == 2) ? 2 : 3;
    constexpr int NS = 2 * H;
    extern __shared__ double lds[];
    const int S = a.S, NT = a.NT;
    const int DW = a.L + M - 1;               // gather window beyond the step, in levels
    const int LV = S + DW;                    // levels held per history table
    double *xch = lds;                                        // [2][2 arrays][2H][kThreads]
    double *eh = xch + 2 * 2 * NS * kThreads;                 // [LV][NT][2][H]: u edges, levels nt-S-DW ..
    double *muh = eh + (size_t)LV * NT * 2 * H;               // [LV][NT][2][H]: mu, levels nt-S ..
    double *gt = muh + (size_t)LV * NT * 2 * H;               // [S][NT][2][H]: gathered mu, levels nt-S ..
    int8_t *kd = reinterpret_cast<int8_t *>(gt + (size_t)S * NT * 2 * H);     // [LV][NT][2]: rows nt-S ..

    const int tid = threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.x * a.CH;
    const int owned = (int)((a.N - c0 < a.CH) ? (a.N - c0) : a.CH);
    const int E = a.RL + owned + S * H;                       // region length
    const int64_t G0 = c0 - a.RL;                             // multiple of PPT
    const int rp0 = tid * PPT;
    const int64_t Gt = G0 + rp0;
    const int64_t tdiv = fdiv(Gt, a.W);
    const int o0 = (int)(Gt - tdiv * a.W);                    // multiple of PPT
    const int tl0 = (int)(tdiv - fdiv(G0, a.W));
    int64_t tp0 = tdiv % a.P;
    if (tp0 < 0) tp0 += a.P;
    const bool in_region = rp0 < E;
    const bool lo_edge = o0 == 0 && in_region;
    const bool hi_edge = o0 + PPT == a.W && in_region;
    const bool owns = rp0 >= a.RL && rp0 < a.RL + owned;
    int64_t gb = Gt % a.N;                                    // a thread's points never straddle the wrap
    if (gb < 0) gb += a.N;
    const Partials<ORDER> pd = partials<ORDER>(a.c1, a.c2);
    const bool stale = a.stale != 0;
    const int64_t F = 2 * a.P;
    const int64_t nlo = a.nt - S;                             // lowest level computed here

    // ---- LDS tables
    {
        int64_t tb = fdiv(G0, a.W) % a.P;
        if (tb < 0) tb += a.P;
        const int nk = LV * NT * 2;
        for (int e = tid; e < nk; e += kThreads) {
            const int side = e & 1;
            const int tl = (e >> 1) % NT;
            const int r = (e >> 1) / NT;
            const int64_t n2 = nlo + r;
            const int64_t tp = (tb + tl) % a.P;
            kd[e] = n2 < a.nsteps_total ? a.delays[n2 * F + 2 * tp + side] : (int8_t)0;
        }
        const int nh = LV * NT * 2 * H;
        for (int e = tid; e < nh; e += kThreads) {
            const int q = e % H;
            const int side = (e / H) & 1;
            const int tl = (e / (2 * H)) % NT;
            const int r = (e / (2 * H)) / NT;
            const int64_t tp = (tb + tl) % a.P;
            const int64_t lev = nlo - DW + r;                 // u edge level
            if (lev >= 0)
                eh[e] = a.ring[((lev * a.P + tp) * 2 + side) * H + q];
            const int64_t n2 = nlo + r;                       // mu level
            if (n2 >= a.nt && n2 < a.nsteps_total) {
                const int64_t ms = n2 % a.Rmu;
                muh[e] = a.mu[((ms * a.P + tp) * 2 + side) * H + q];
            }
        }
    }

    // ---- lambda^{nt} of the thread's points
    double lam[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) lam[j] = in_region ? a.lam_in[gb + j] : 0.0;

    // P_s(u) = dt*(nu*g2[s] - a*g1[s]) for a compile-time slot s
    auto Ps = [&](int s, double u) -> double {
        const double adv = LINEAR ? a.cadv : u;
        return a.dt * (a.nu * pd.g2[s] - adv * pd.g1[s]);
    };

    Acc gacc{0.0, 0.0};
    // one reverse step: level n = nt-1-t from lambda^{n+1} (lam) and u^n (uc);
    // the loads of u^{n-1} go to un
    auto rstep = [&](int t, double (&uc)[PPT], double (&un)[PPT]) {
        const int64_t n = a.nt - 1 - t;
        {   // unconditional (a level inside the segment), so that the wait for uc
            // below leaves these loads in flight
            const int64_t nn = t + 1 < S ? n - 1 : n;
            const double *src = a.seg + (nn - a.seg_n0) * a.N + gb;
#pragma unroll
            for (int j = 0; j < PPT; ++j) un[j] = src[j];
        }
        // ---- exchange lambda^{n+1} and u^n edges with the neighbouring threads
        double *buf = xch + (t & 1) * 2 * NS * kThreads;
#pragma unroll
        for (int q = 0; q < H; ++q) {
            buf[(0 * NS + q) * kThreads + tid] = lam[q];
            buf[(0 * NS + H + q) * kThreads + tid] = lam[PPT - H + q];
            buf[(1 * NS + q) * kThreads + tid] = uc[q];
            buf[(1 * NS + H + q) * kThreads + tid] = uc[PPT - H + q];
        }
        __syncthreads();
        double llo[H], lhi[H], ulo[H], uhi[H];   // raw neighbours: points -H..-1 and PPT..PPT+H-1
#pragma unroll
        for (int q = 0; q < H; ++q) {
            llo[q] = tid > 0 ? buf[(0 * NS + H + q) * kThreads + tid - 1] : 0.0;
            ulo[q] = tid > 0 ? buf[(1 * NS + H + q) * kThreads + tid - 1] : 0.0;
            lhi[q] = tid < kThreads - 1 ? buf[(0 * NS + q) * kThreads + tid + 1] : 0.0;
            uhi[q] = tid < kThreads - 1 ? buf[(1 * NS + q) * kThreads + tid + 1] : 0.0;
        }
        // ---- the LDS values of this step's edge work, all loaded before the
        // first is used so that their latencies overlap: the delays of this
        // tile's faces, and the delays and gathered sums at level n of the
        // neighbours' faces that this thread's edge points feed
        const int krow = (int)(n - nlo);
        const bool lo_src = lo_edge && tid > 0;   // region ends: no source tile in the tables
        const bool hi_src = hi_edge && tid < kThreads - 1;
        int kown[2] = {0, 0}, knb[2] = {1, 1};
        double gth[2][H];
#pragma unroll
        for (int q = 0; q < H; ++q) { gth[0][q] = 0.0; gth[1][q] = 0.0; }
        if (lo_edge) kown[0] = kd[(krow * NT + tl0) * 2 + 0];
        if (hi_edge) kown[1] = kd[(krow * NT + tl0) * 2 + 1];
        if (hi_src) {                             // feeds the next tile's low face
            knb[0] = kd[(krow * NT + tl0 + 1) * 2 + 0];
#pragma unroll
            for (int q = 0; q < H; ++q) gth[0][q] = gt[((krow * NT + tl0 + 1) * 2 + 0) * H + q];
        }
        if (lo_src) {                             // feeds the previous tile's high face
            knb[1] = kd[(krow * NT + tl0 - 1) * 2 + 1];
#pragma unroll
            for (int q = 0; q < H; ++q) gth[1][q] = gt[((krow * NT + tl0 - 1) * 2 + 1) * H + q];
        }
        // ---- u window with the forward AT halo across the tile faces
        double uw[PPT + 2 * H];
#pragma unroll
        for (int q = 0; q < H; ++q) { uw[q] = ulo[q]; uw[PPT + H + q] = uhi[q]; }
#pragma unroll
        for (int j = 0; j < PPT; ++j) uw[H + j] = uc[j];
        if (lo_edge || hi_edge) {
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                if (side == 0 ? !lo_src : !hi_src) continue;
                const int kk = kown[side];
                if (kk > 0) {
                    const int stl = side == 0 ? tl0 - 1 : tl0 + 1;
#pragma unroll
                    for (int q = 0; q < H; ++q) {
                        double vv[3] = {0.0, 0.0, 0.0};
#pragma unroll
                        for (int jj = 0; jj < M; ++jj) {
                            if (jj == 0 || !stale) {
                                const int64_t lev = n - kk - jj;
                                vv[jj] = eh[((((int)(lev - (nlo - DW))) * NT + stl) * 2 + (1 - side)) * H + q];
                            }
                        }
                        const double hv = extrap(kk, stale, vv[0], vv[1], vv[2], M);
                        if (side == 0) uw[q] = hv;
                        else uw[PPT + H + q] = hv;
                    }
                }
            }
        }
        // lambda and raw u at window index i (-H .. PPT+H-1), compile-time i
        auto lat = [&](int i) -> double { return i < 0 ? llo[H + i] : (i >= PPT ? lhi[i - PPT] : lam[i]); };
        auto uat = [&](int i) -> double { return i < 0 ? ulo[H + i] : (i >= PPT ? uhi[i - PPT] : uc[i]); };
        // mu^n of this step for the face a point feeds, from the raw window
        auto mu_lo = [&](int q) -> double {         // face of the next tile, low side: its first h points
            double m = 0.0;
#pragma unroll
            for (int e = 0; e < H; ++e)
                if (e <= q) m += lat(PPT + e) * Ps(q - e, uat(PPT + e));
            return m;
        };
        auto mu_hi = [&](int q) -> double {         // face of the previous tile, high side: its last h points
            double m = 0.0;
#pragma unroll
            for (int e = 0; e < H; ++e)
                if (e <= H - 1 - q) m += lat(-1 - e) * Ps(H + q + e, uat(-1 - e));
            return m;
        };
        double res[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const double u = uc[j];
            double nb[NS];
#pragma unroll
            for (int q = 0; q < H; ++q) { nb[q] = uw[j + q]; nb[H + q] = uw[j + H + 1 + q]; }
            double D1, D2;
            if constexpr (ORDER == 2) {
                D1 = (nb[1] - nb[0]) * a.c1;
                D2 = ((nb[1] - 2.0 * u) + nb[0]) * a.c2;
            } else {
                D1 = (8.0 * (nb[2] - nb[1]) - (nb[3] - nb[0])) * a.c1;
                D2 = ((16.0 * (nb[2] + nb[1]) - 30.0 * u) - (nb[3] + nb[0])) * a.c2;
            }
            const double lg = lam[j];
            const double du = 1.0 + a.dt * (a.nu * pd.g2u - (LINEAR ? 0.0 : D1));
            double acc = lg * du;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int d = (s < H) ? -(H - s) : (s - H + 1);
                const int i = j - d;
                const bool same = (i >= 0 || !lo_edge) && (i < PPT || !hi_edge);
                if (same) acc += lat(i) * Ps(s, uat(i));
            }
            // delayed halo contributions gathered over steps n .. n+L+m-1
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const bool feeds = side == 0 ? (hi_src && j >= PPT - H) : (lo_src && j < H);
                if (!feeds) continue;
                const int q = side == 0 ? j - (PPT - H) : j;
                // later levels' contributions, accumulated newest first by their
                // producers; then this level's own (k = 0: the raw neighbour)
                double g = gth[side][q];
                if (knb[side] == 0)
                    g += hweight(0, stale, 0, M) * (side == 0 ? mu_lo(q) : mu_hi(q));
                acc += g;
            }
            res[j] = acc;
            if (owns) acc_add(gacc, lg * (a.dt * D2));
        }
        // ---- mu^n of this tile's faces: added to the gathered sums of the
        // earlier levels of this launch that it feeds (n-k-j, weight dH/dv_j),
        // and to the ring for later launches
        auto scatter = [&](int side, int q, double m) {
            const int kk = kown[side];
            const int need = (kk == 0 || stale) ? 1 : M;
            for (int jw = 0; jw < need; ++jw) {
                const int64_t nt2 = n - kk - jw;      // level this contribution belongs to
                if (nt2 == n || nt2 < nlo) continue;  // own level: gathered directly
                double &gref = gt[((((int)(nt2 - nlo)) * NT + tl0) * 2 + side) * H + q];
                gref += hweight(kk, stale, jw, M) * m;
            }
        };
        if (lo_edge || hi_edge) {
            const int64_t ms = n % a.Rmu;
#pragma unroll
            for (int q = 0; q < H; ++q) {
                if (lo_edge) {                        // own first h points feed the low face
                    double m = 0.0;
#pragma unroll
                    for (int e = 0; e < H; ++e)
                        if (e <= q) m += lam[e] * Ps(q - e, uc[e]);
                    scatter(0, q, m);
                    if (owns) a.mu[((ms * a.P + tp0) * 2 + 0) * H + q] = m;
                }
                if (hi_edge) {                        // own last h points feed the high face
                    double m = 0.0;
#pragma unroll
                    for (int e = 0; e < H; ++e)
                        if (e <= H - 1 - q) m += lam[PPT - 1 - e] * Ps(H + q + e, uc[PPT - 1 - e]);
                    scatter(1, q, m);
                    if (owns) a.mu[((ms * a.P + tp0) * 2 + 1) * H + q] = m;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < PPT; ++j) lam[j] = res[j];
    };

    double ua[PPT], ub[PPT];
    {
        const double *src = a.seg + (a.nt - 1 - a.seg_n0) * a.N + gb;
#pragma unroll
        for (int j = 0; j < PPT; ++j) ua[j] = src[j];
#pragma unroll
        for (int j = 0; j < PPT; ++j) ub[j] = 0.0;
    }
    __syncthreads();                          // LDS tables ready
    // delayed contributions to the levels of this launch from mu levels
    // written by earlier launches (nt ..), newest first; the launch's own mu
    // levels are added by their producers as they are computed
    {
        const int ng = S * NT * 2 * H;
        for (int e = tid; e < ng; e += kThreads) {
            const int q = e % H;
            const int side = (e / H) & 1;
            const int tl = (e / (2 * H)) % NT;
            const int r = (e / (2 * H)) / NT;
            const int64_t n = nlo + r;
            double g = 0.0;
            int64_t top = n + DW;
            if (top > a.nsteps_total - 1) top = a.nsteps_total - 1;
            for (int64_t n2 = top; n2 >= a.nt && n2 > n; --n2) {
                const int r2 = (int)(n2 - nlo);
                const int kk = kd[(r2 * NT + tl) * 2 + side];
                const int jw = (int)(n2 - n) - kk;
                const int need = (kk == 0 || stale) ? 1 : M;
                if (jw < 0 || jw >= need) continue;
                g += hweight(kk, stale, jw, M) * muh[((r2 * NT + tl) * 2 + side) * H + q];
            }
            gt[e] = g;
        }
    }
    int t = 0;
    for (; t + 2 <= S; t += 2) {
        rstep(t, ua, ub);
        rstep(t + 1, ub, ua);
    }
    if (t < S) rstep(t, ua, ub);

    if (owns) {
#pragma unroll
        for (int j = 0; j < PPT; ++j) a.lam_out[gb + j] = lam[j];
    }
    __shared__ double red[kThreads / 64][2];
    gacc = wave_acc(gacc);
    const int lane = tid & 63, wv = tid >> 6;
    if (lane == 0) { red[wv][0] = gacc.s; red[wv][1] = gacc.c; }
    __syncthreads();
    if (tid == 0) {
        Acc Sg{a.gnu[blockIdx.x * 2], a.gnu[blockIdx.x * 2 + 1]};
        for (int q = 0; q < kThreads / 64; ++q) acc_merge(Sg, Acc{red[q][0], red[q][1]});
        a.gnu[blockIdx.x * 2] = Sg.s;
        a.gnu[blockIdx.x * 2 + 1] = Sg.c;
    }
}

}  // namespace

int adj1d_points_per_block() { return kCHA; }

hipError_t launch_adj1d_fused(const AdjF &a, int order, bool linear, int ppt, int64_t nblocks,
                              size_t lds, hipStream_t st)
{
    dim3 grid((unsigned)nblocks), block(kThreads);
#define AT_AF(O, LI, P) hipLaunchKernelGGL((k_adj1d_fused<O, LI, P>), grid, block, lds, st, a)
    if (ppt != 4 && ppt != 8) return hipErrorInvalidValue;
    if (order == 2) {
        if (linear) { if (ppt == 8) AT_AF(2, true, 8); else AT_AF(2, true, 4); }
        else { if (ppt == 8) AT_AF(2, false, 8); else AT_AF(2, false, 4); }
    } else {
        if (linear) { if (ppt == 8) AT_AF(4, true, 8); else AT_AF(4, true, 4); }
        else { if (ppt == 8) AT_AF(4, false, 8); else AT_AF(4, false, 4); }
    }
#undef AT_AF
    return hipGetLastError();
}

size_t adj1d_fused_lds_bytes(int order, int S, int NT, int L)
{
    const int H = order / 2, M = order == 2 ? 2 : 3;
    const size_t LV = (size_t)S + L + M - 1;
    const size_t dbl = (size_t)2 * 2 * 2 * H * kThreads + 2 * LV * NT * 2 * H +
                       (size_t)S * NT * 2 * H;
    return 8 * dbl + ((LV * NT * 2 + 7) / 8) * 8;
}

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
