// Host side of libat.so: configuration checks, workspace layout, delay set-up,
// launch sequencing (plain, fused, recorded), checkpoints, adjoint sweep,
// snapshots, reductions and the autotuner.  See include/at.h for the contract.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/at.h"
#include "at_internal.h"

using namespace atk;

// 3D hooks (defined in at_step3d.hip)
at_status at3_check(const at_config *c);
uint64_t at3_ring_level_doubles(const at_config *c);

namespace {

thread_local std::string g_err;

at_status fail(at_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define AT_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(AT_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));    \
    } while (0)

constexpr uint64_t kAlign = 256;
constexpr int kWholeVariant = 4;   // 1D: the whole grid in one workgroup
uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    uint64_t delays = 0, ring = 0, red = 0, sync = 0, ckpt = 0, seg = 0, lam = 0, mu = 0, gnu = 0,
             total = 0;
    int64_t nckpt = 0, ngnu = 0;
    int R = 0, Rmu = 0;
};

struct Derived {
    int dim, order, h, m;
    int L;          // delay bound
    int fppt = 16;  // 1D: points per thread of the fused (aligned) launches
    int64_t N;      // total points
    int64_t F;      // faces
    int64_t nb;     // tiles / blocks
    int64_t P, W;   // 1D
    double c1[3], c2[3];
};

// Region of one workgroup: RL points left of the owned chunk, CH owned, s*h
// right.  Aligned form (tile width a multiple of the points per thread): RL
// and CH are multiples of PPT so every thread's points lie in one tile.
struct Region1D {
    bool aligned;
    int ppt;        // points per thread of the kernel that runs it
    int64_t RL, CH;
};

// Points per thread of the fused 1D launches: the most (16, 8, 4) that still
// give every SIMD four waves of the grid and divide the tile width; 16 (the
// unaligned kernel) when none divides it.
int fused_ppt(const Derived &d)
{
    const int opts[3] = {16, 8, 4};
    int pick = 0;
    for (int i = 0; i < 3; ++i) {
        const int p = opts[i];
        if (d.W % p != 0) continue;
        if (pick == 0) pick = p;
        if (d.N >= (int64_t)4 * 1024 * 64 * p) return p;
        pick = p;
    }
    return pick ? pick : 16;
}

at_status derive(const at_config *c, Derived &d)
{
    if (!c) return fail(AT_ERR_ARG, "null configuration");
    if (c->abi_version != AT_ABI_VERSION)
        return fail(AT_ERR_ARG, "abi_version %d, library has %d", c->abi_version, AT_ABI_VERSION);
    if (c->dim != 1 && c->dim != 3) return fail(AT_ERR_ARG, "dim must be 1 or 3");
    if (c->order != 2 && c->order != 4) return fail(AT_ERR_ARG, "order must be 2 or 4");
    if (c->dim == 3 && c->order != 2) return fail(AT_ERR_ARG, "3D stepper is order 2");
    if (c->L < 0 || c->L > 15) return fail(AT_ERR_ARG, "L must be in 0..15");
    if (c->halo_mode != 0 && c->halo_mode != 1) return fail(AT_ERR_ARG, "halo_mode must be 0 or 1");
    if (c->adv_mode != 0 && c->adv_mode != 1) return fail(AT_ERR_ARG, "adv_mode must be 0 or 1");
    if (c->adv_mode == 1 && c->dim != 1) return fail(AT_ERR_ARG, "linear advection is 1D only");
    if (!(c->nu >= 0.0) || !isfinite(c->nu)) return fail(AT_ERR_ARG, "nu must be finite and >= 0");
    if (!(c->dt > 0.0) || !isfinite(c->dt)) return fail(AT_ERR_ARG, "dt must be finite and > 0");
    if (!(c->length > 0.0) || !isfinite(c->length)) return fail(AT_ERR_ARG, "length must be > 0");
    if (c->nsteps_max < 0) return fail(AT_ERR_ARG, "nsteps_max must be >= 0");
    if (c->delay_mode != AT_DELAY_GENERATE && c->delay_mode != AT_DELAY_HOST)
        return fail(AT_ERR_ARG, "unknown delay_mode");
    if (c->delay_mode == AT_DELAY_GENERATE && c->delay_dist != AT_DIST_UNIFORM &&
        c->delay_dist != AT_DIST_HALF_ZERO)
        return fail(AT_ERR_ARG, "unknown delay_dist");
    if (c->delay_mode == AT_DELAY_HOST && !c->delays_host && c->nsteps_max > 0)
        return fail(AT_ERR_ARG, "delays_host is NULL");
    if (c->fuse_steps < 0 || c->fuse_steps > kMaxFuse)
        return fail(AT_ERR_ARG, "fuse_steps must be in 0..%d", kMaxFuse);
    if (c->arith != 0 && c->arith != 1) return fail(AT_ERR_ARG, "arith must be 0 or 1");
    if (c->arith == 1 && c->dim != 1) return fail(AT_ERR_ARG, "arith 1 is 1D only");
    if (c->reserved1 != 0) return fail(AT_ERR_ARG, "reserved1 must be 0");
    if (c->nscalars < 0 || c->nscalars > AT_MAX_SCALARS)
        return fail(AT_ERR_ARG, "nscalars must be in 0..%d", AT_MAX_SCALARS);
    if (c->nscalars > 0 && c->dim != 3) return fail(AT_ERR_ARG, "passive scalars are 3D only");
    for (int s = 0; s < c->nscalars; ++s)
        if (!(c->alpha[s] >= 0.0) || !isfinite(c->alpha[s]))
            return fail(AT_ERR_ARG, "alpha[%d] must be finite and >= 0", s);
    if (c->record) {
        if (c->dim != 1) return fail(AT_ERR_ARG, "record mode (adjoint) is 1D only");
        if (c->ckpt_every < 1) return fail(AT_ERR_ARG, "record mode needs ckpt_every >= 1");
    }
    d.dim = c->dim;
    d.order = c->order;
    d.h = c->order / 2;
    d.m = (c->order == 2) ? 2 : 3;
    d.L = c->L;
    const int naxes = c->dim;
    d.N = 1;
    d.nb = 1;
    for (int a = 0; a < 3; ++a) {
        const int64_t n = c->n[a];
        const int64_t p = c->p[a];
        if (a >= naxes) {
            if (n != 1 || p != 1) return fail(AT_ERR_SHAPE, "unused axis %d must have n = p = 1", a);
            d.c1[a] = d.c2[a] = 0.0;
            continue;
        }
        if (n <= 0 || p <= 0) return fail(AT_ERR_SHAPE, "axis %d: n and p must be positive", a);
        if (n % p != 0) return fail(AT_ERR_SHAPE, "axis %d: n %% p != 0", a);
        if (n / p < 2 * d.h) return fail(AT_ERR_SHAPE, "axis %d: tile width %lld < 2h", a,
                                         (long long)(n / p));
        const double dx = c->length / (double)n;
        if (c->order == 2) { d.c1[a] = 1.0 / (2.0 * dx); d.c2[a] = 1.0 / (dx * dx); }
        else { d.c1[a] = 1.0 / (12.0 * dx); d.c2[a] = 1.0 / (12.0 * (dx * dx)); }
        d.N *= n;
        d.nb *= p;
    }
    d.F = (c->dim == 1 ? 2 : 6) * d.nb;
    d.P = c->p[0];
    d.W = c->n[0] / c->p[0];
    if (d.N > ((int64_t)1 << 40)) return fail(AT_ERR_SHAPE, "grid too large");
    if (c->dim == 3) {
        at_status st = at3_check(c);
        if (st != AT_OK) return st;
    }
    if (d.dim == 1) d.fppt = fused_ppt(d);
    return AT_OK;
}

int max_fuse_1d(const Derived &d);

// ring levels: L+m-1 past levels are read while up to s levels are written
// (s = the largest steps-per-launch this grid allows); record mode keeps every
// level of the run (the adjoint re-reads them).
int ring_levels(const at_config *c, const Derived &d)
{
    // 1D: any steps-per-launch and points-per-thread choice; 3D: a step reads
    // levels n-L-1 .. n and publishes level n+1, and in the weakly-synchronous
    // run a face neighbour up to L steps behind still reads levels down to
    // n-2L-1 while this block writes level n+1: 2L + m + 2 slots keep them apart
    const int smax = d.dim == 1 ? kMaxFuse : c->L + 3;
    int64_t R = c->L + d.m - 1 + smax;
    if (c->record) R = std::max<int64_t>(R, c->nsteps_max + 1);
    return (int)R;
}

}  // namespace

struct at_ctx {
    at_config cfg;
    Derived d;
    Layout lay;
    hipStream_t st;
    int8_t *delays;
    double *ring, *red, *ckpt, *seg, *lam, *mu, *gnu;
    int32_t *sync;   // level counters (1D [P][2], 3D [blocks]), then the error flag
    int64_t n;
    int fuse;
    int variant;     // 3D kernel variant (tile rows, prefetch depth, register budget)
    int adj_fuse = 0;   // reverse steps per adjoint launch: 0 automatic, 1 one-step kernel
    int debug = 0;      // AT_DEBUG_* flags (at_set_debug)
    // graph replay of at_run (at_set_graph): the launch sequence of one call,
    // captured on a private stream and replayed on the context's stream
    int use_graph = 0;
    hipStream_t cap = nullptr;
    hipGraphExec_t gexec = nullptr;
    int64_t g_n0 = -1, g_nsteps = -1;
    const double *g_u = nullptr, *g_s = nullptr;
    int g_fuse = 0, g_variant = -1, g_debug = -1;
    // snapshots taken through this context: device buffer and its step
    std::vector<std::pair<const void *, int64_t>> snaps;
};

namespace {

uint64_t ring_level_doubles(const at_config *c, const Derived &d)
{
    if (d.dim == 1) return (uint64_t)d.P * 2 * d.h;
    return at3_ring_level_doubles(c);
}

int64_t adj_blocks(const Derived &d)
{
    const int64_t per = adj1d_points_per_block();
    return (d.N + per - 1) / per;
}

at_status make_layout(const at_config *c, const Derived &d, Layout &L)
{
    L.R = ring_levels(c, d);
    L.Rmu = c->L + d.m + kMaxFuse;   // levels a fused reverse launch writes and reads stay distinct
    uint64_t off = 0;
    L.delays = off;
    off = align_up(off + (uint64_t)c->nsteps_max * (uint64_t)d.F);
    L.ring = off;
    off = align_up(off + 8ull * (uint64_t)L.R * ring_level_doubles(c, d));
    L.red = off;
    off = align_up(off + 8ull * (kRedBlocks * 6 + 16));
    // level counters of the weakly-synchronous run (1D: [P][2] tile edges;
    // 3D: one per block), then its error flag
    L.sync = off;
    off = align_up(off + 4ull * ((d.dim == 1 ? 2 * (uint64_t)d.P : (uint64_t)d.nb) + 64));
    if (c->record) {
        L.nckpt = c->nsteps_max / c->ckpt_every + 1;
        L.ckpt = off;
        off = align_up(off + 8ull * (uint64_t)L.nckpt * (uint64_t)d.N);
        L.seg = off;
        off = align_up(off + 8ull * (uint64_t)c->ckpt_every * (uint64_t)d.N);
        L.lam = off;
        off = align_up(off + 8ull * 2 * (uint64_t)d.N);
        L.mu = off;
        off = align_up(off + 8ull * (uint64_t)L.Rmu * (uint64_t)d.P * 2 * d.h);
        L.ngnu = (d.N + 255) / 256;   // >= the blocks of any reverse launch (chunks >= 256 points)
        L.gnu = off;
        off = align_up(off + 8ull * 2 * (uint64_t)L.ngnu);
    }
    L.total = off;
    return AT_OK;
}

Region1D region_1d(const Derived &d, int s, bool allow_plain = true);

// Largest steps-per-launch usable for this 1D configuration: the owned chunk
// stays at least half the region (or the whole grid) and the LDS edge
// history fits in 64 KiB.
int max_fuse_1d(const Derived &d)
{
    int best = 1;
    for (int s = 2; s <= kMaxFuse; ++s) {
        const Region1D rg = region_1d(d, s);
        const int reg = kThreads * rg.ppt;
        if (rg.CH < std::min<int64_t>(reg / 2, d.N)) break;
        const int NT = (int)((reg - 1) / d.W + 2);
        if (step1d_lds_bytes(d.order, s, NT, d.L + d.m - 1, rg.ppt, false) > 64 * 1024) break;
        best = s;
    }
    return best;
}

Region1D region_1d(const Derived &d, int s, bool allow_plain)
{
    // single steps use the 8-point-per-thread kernel when the tiles allow it
    // (not in the batched form, whose kernel keeps 16 points per thread)
    const int pplain = step1d_plain_points_per_thread();
    const bool plain = allow_plain && s == 1 && d.W % pplain == 0;
    const int ppt = plain ? pplain : (d.W % d.fppt == 0 ? d.fppt : step1d_points_per_thread());
    const int64_t reg = (int64_t)kThreads * ppt;
    Region1D r;
    r.ppt = ppt;
    r.aligned = d.W % ppt == 0;
    if (r.aligned) {
        r.RL = ((int64_t)s * d.h + ppt - 1) / ppt * ppt;
        r.CH = (reg - r.RL - (int64_t)s * d.h) / ppt * ppt;
    } else {
        r.RL = (int64_t)s * d.h;
        r.CH = reg - 2 * (int64_t)s * d.h;
    }
    if (r.CH > d.N) r.CH = d.N;
    return r;
}

// Points per thread of the whole-grid single-workgroup kernel (1D variant 4)
// for this context, 0 when the grid does not fit one workgroup
int whole_ppt(const at_ctx *c)
{
    const Derived &d = c->d;
    if (d.dim != 1) return 0;
    return step1d_whole_ppt(d.N, d.W, d.P, d.order, c->cfg.L + d.m - 1);
}

at_status launch_1d(at_ctx *c, const double *uin, double *uout, int64_t n0, int s, int publish,
                    double *levels = nullptr)
{
    const Derived &d = c->d;
    if (c->variant == kWholeVariant && !levels) {
        // the whole grid in one workgroup: any number of steps, no rims
        Step1D a{};
        a.uin = uin;
        a.uout = uout;
        a.ring = c->ring;
        a.delays = c->delays;
        a.N = d.N;
        a.P = d.P;
        a.W = d.W;
        a.n0 = n0;
        a.CH = d.N;
        a.s = s;
        a.R = c->lay.R;
        a.NT = (int)d.P;
        a.stale = c->cfg.halo_mode;
        a.publish = publish;
        a.RL = 0;
        a.slot0 = (int32_t)(n0 % a.R);
        a.D = c->cfg.L + d.m - 1;
        a.levels = nullptr;
        a.nu = c->cfg.nu;
        a.dt = c->cfg.dt;
        a.c1 = d.c1[0];
        a.c2 = d.c2[0];
        a.cadv = c->cfg.adv_speed;
        a.A1 = a.dt * a.c1;
        a.A2 = a.dt * (a.nu * a.c2);
        AT_HIP(launch_step1d_whole(a, d.order, c->cfg.adv_mode == 1, c->cfg.arith == 1,
                                   whole_ppt(c), c->st));
        return AT_OK;
    }
    const Region1D rg = region_1d(d, s);
    const int reg = kThreads * rg.ppt;
    Step1D a;
    a.uin = uin;
    a.uout = uout;
    a.ring = c->ring;
    a.delays = c->delays;
    a.N = d.N;
    a.P = d.P;
    a.W = d.W;
    a.n0 = n0;
    a.CH = rg.CH;
    if (a.CH < 1) return fail(AT_ERR_ARG, "fuse_steps %d too large for this stencil", s);
    a.s = s;
    a.R = c->lay.R;
    a.NT = (int)((reg - 1) / d.W + 2);
    a.stale = c->cfg.halo_mode;
    a.publish = publish;
    a.RL = (int32_t)rg.RL;
    a.slot0 = (int32_t)(n0 % a.R);
    a.D = c->cfg.L + d.m - 1;
    a.levels = levels;
    if (levels && !rg.aligned) return fail(AT_ERR_STATE, "level store needs the aligned layout");
    a.nu = c->cfg.nu;
    a.dt = c->cfg.dt;
    a.c1 = d.c1[0];
    a.c2 = d.c2[0];
    a.cadv = c->cfg.adv_speed;
    a.A1 = a.dt * a.c1;
    a.A2 = a.dt * (a.nu * a.c2);
    const int64_t nblocks = (d.N + a.CH - 1) / a.CH;
    AT_HIP(launch_step1d(a, d.order, c->cfg.adv_mode == 1, rg.aligned, c->cfg.arith == 1, rg.ppt,
                         nblocks, c->st));
    return AT_OK;
}

}  // namespace

// 3D launcher (at_step3d.hip)
at_status at3_launch(at_ctx *c, const double *uin, double *uout, int64_t n0, int s, int publish);
at_status at3_publish(at_ctx *c, const double *u, int64_t n);
int at3_max_fuse(const at_ctx *c);
int at3_variants();
bool at3_variant_ok(const at_config *c, int var);
bool at3_is_fused(int var);
int at3_single_variant(const at_config *c, int var);
int64_t at3_ws_capacity(const at_config *c);
at_status at3_launch_ws(at_ctx *ctx, double *u, double *scratch, int64_t n0, int64_t nsteps,
                        int32_t *cnt, int32_t *err, int8_t *delays, int32_t jitter, uint64_t seed,
                        int64_t spin_limit, int *in_scratch);

// accessors used by the 3D translation unit
extern "C++" {
const at_config *at_ctx_cfg(const at_ctx *c) { return &c->cfg; }
double *at_ctx_ring(const at_ctx *c) { return c->ring; }
const int8_t *at_ctx_delays(const at_ctx *c) { return c->delays; }
int at_ctx_R(const at_ctx *c) { return c->lay.R; }
hipStream_t at_ctx_stream(const at_ctx *c) { return c->st; }
void at_ctx_coefs(const at_ctx *c, double *c1, double *c2)
{
    for (int a = 0; a < 3; ++a) { c1[a] = c->d.c1[a]; c2[a] = c->d.c2[a]; }
}
at_status at_fail(at_status st, const char *msg) { return fail(st, "%s", msg); }
int at_ctx_variant(const at_ctx *c) { return c->variant; }
}

namespace {

at_status launch_any(at_ctx *c, const double *uin, double *uout, int64_t n0, int s, int publish)
{
    if (c->d.dim == 1) return launch_1d(c, uin, uout, n0, s, publish);
    return at3_launch(c, uin, uout, n0, s, publish);
}

// doubles in one field: N (1D) or (3 + nscalars) N (3D: velocity, then scalars)
int64_t field_doubles(const at_ctx *c)
{
    return (c->d.dim == 1 ? 1 : 3 + c->cfg.nscalars) * c->d.N;
}

int max_fuse(const at_ctx *c)
{
    return c->d.dim == 1 ? max_fuse_1d(c->d) : at3_max_fuse(c);
}

// Ring levels a later launch may still read once the context has reached
// level n1: 1D, the L + m - 1 levels below n1 (a step n reads levels down to
// n - L - m + 1 and publishes level n itself); 3D, levels n1 - L - 1 .. n1
// (a step reads levels down to n - L - 1, and level n's faces are published
// before it).  Levels below 0 are never read (start-up clamp).
void live_levels(const at_ctx *c, int64_t n1, int64_t *lo, int64_t *hi)
{
    if (c->d.dim == 1) {
        *lo = n1 - (c->cfg.L + c->d.m - 1);
        *hi = n1 - 1;
    } else {
        *lo = n1 - c->cfg.L - 1;
        *hi = n1;
    }
    if (*lo < 0) *lo = 0;
}

// Debug mode AT_DEBUG_POISON_RING: after every launch, every ring slot that
// holds no live level is overwritten with NaN, so a step that read a level it
// must not would carry the NaN into the field.
hipError_t poison_ring(at_ctx *c, int64_t n1)
{
    if (!(c->debug & AT_DEBUG_POISON_RING)) return hipSuccess;
    int64_t lo, hi;
    live_levels(c, n1, &lo, &hi);
    const int64_t R = c->lay.R;
    const int64_t nlive = hi >= lo ? std::min<int64_t>(hi - lo + 1, R) : 0;
    return launch_poison(c->ring, R, (int64_t)ring_level_doubles(&c->cfg, c->d),
                         (int)(lo % R), (int)nlive, c->st);
}

// Clear the whole ring: zeros, or NaN in the poisoning debug mode (no level is
// live before the first step)
hipError_t clear_ring(at_ctx *c)
{
    const double v = (c->debug & AT_DEBUG_POISON_RING) ? __builtin_nan("") : 0.0;
    return launch_fill(c->ring, (int64_t)c->lay.R * (int64_t)ring_level_doubles(&c->cfg, c->d),
                       v, c->st);
}

void drop_graph(at_ctx *c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
    c->g_n0 = c->g_nsteps = -1;
}

// Region of a fused reverse launch of s steps (8 points per thread, aligned)
struct RegionAdj {
    int64_t RL, CH;
    int NT, ppt;
};

// Points per thread of the fused reverse launches (8 or 4: the larger one
// that still gives every SIMD four waves and divides the tile width), 0 when
// neither divides it
int adj_ppt(const Derived &d)
{
    if (d.W % 8 == 0 && d.N >= (int64_t)4 * 1024 * 64 * 8) return 8;
    if (d.W % 4 == 0) return 4;
    return d.W % 8 == 0 ? 8 : 0;
}

RegionAdj region_adj(const Derived &d, int s)
{
    const int ppf = adj_ppt(d);
    const int64_t reg = (int64_t)kThreads * ppf;
    RegionAdj r;
    r.ppt = ppf;
    r.RL = ((int64_t)s * d.h + ppf - 1) / ppf * ppf;
    r.CH = (reg - r.RL - (int64_t)s * d.h) / ppf * ppf;
    if (r.CH > d.N) r.CH = d.N;
    r.NT = (int)((reg - 1) / d.W + 2);
    return r;
}

// Reverse steps per launch: 0 when the tiles do not fit the fused kernel,
// else the most (up to kMaxFuse) that keep the owned chunk at least half the
// region (and 256 points) and the LDS tables within 64 KiB
int adj_fuse_max(const Derived &d, int L)
{
    if (adj_ppt(d) == 0) return 0;
    int best = 0;
    for (int s = 1; s <= kMaxFuse; ++s) {
        const RegionAdj r = region_adj(d, s);
        if (r.CH < std::min<int64_t>(std::max<int64_t>(256, kThreads * r.ppt / 2), d.N)) break;
        if (adj1d_fused_lds_bytes(d.order, s, r.NT, L) > 64 * 1024) break;
        best = s;
    }
    return best;
}

}  // namespace

extern "C" {

int32_t at_abi_version(void) { return AT_ABI_VERSION; }

const char *at_last_error(void) { return g_err.c_str(); }

uint64_t at_config_bytes(void) { return sizeof(at_config); }

at_status at_workspace_bytes(const at_config *cfg, uint64_t *bytes)
{
    Derived d;
    at_status st = derive(cfg, d);
    if (st) return st;
    if (!bytes) return fail(AT_ERR_ARG, "null output");
    Layout L;
    make_layout(cfg, d, L);
    *bytes = L.total;
    return AT_OK;
}

at_status at_init(const at_config *cfg, at_ctx **out)
{
    if (!out) return fail(AT_ERR_ARG, "null output");
    *out = nullptr;
    Derived d;
    at_status st = derive(cfg, d);
    if (st) return st;
    Layout L;
    make_layout(cfg, d, L);
    if (!cfg->workspace) return fail(AT_ERR_ARG, "workspace is NULL");
    if (((uintptr_t)cfg->workspace) % kAlign) return fail(AT_ERR_ARG, "workspace not 256-byte aligned");
    if (cfg->workspace_bytes < L.total)
        return fail(AT_ERR_NOMEM, "workspace %llu bytes, need %llu",
                    (unsigned long long)cfg->workspace_bytes, (unsigned long long)L.total);
    if (cfg->delay_mode == AT_DELAY_HOST) {
        // every entry must satisfy 0 <= k <= min(L, max(0, n - m + 1))
        for (int64_t n = 0; n < cfg->nsteps_max; ++n) {
            int64_t lim = std::min<int64_t>(cfg->L, std::max<int64_t>(0, n - d.m + 1));
            const int8_t *row = cfg->delays_host + n * d.F;
            for (int64_t f = 0; f < d.F; ++f)
                if (row[f] < 0 || row[f] > lim)
                    return fail(AT_ERR_DELAY, "delay k[%lld][%lld] = %d outside 0..%lld",
                                (long long)n, (long long)f, (int)row[f], (long long)lim);
        }
    }
    at_ctx *c = new (std::nothrow) at_ctx;
    if (!c) return fail(AT_ERR_NOMEM, "host allocation failed");
    c->cfg = *cfg;
    c->cfg.delays_host = nullptr;
    c->d = d;
    c->lay = L;
    c->st = (hipStream_t)cfg->stream;
    char *base = (char *)cfg->workspace;
    c->delays = (int8_t *)(base + L.delays);
    c->ring = (double *)(base + L.ring);
    c->red = (double *)(base + L.red);
    c->sync = (int32_t *)(base + L.sync);
    c->ckpt = cfg->record ? (double *)(base + L.ckpt) : nullptr;
    c->seg = cfg->record ? (double *)(base + L.seg) : nullptr;
    c->lam = cfg->record ? (double *)(base + L.lam) : nullptr;
    c->mu = cfg->record ? (double *)(base + L.mu) : nullptr;
    c->gnu = cfg->record ? (double *)(base + L.gnu) : nullptr;
    c->n = 0;
    c->variant = 0;
    if (d.dim == 3)   // the first variant with a build for this component count
        while (!at3_variant_ok(&c->cfg, c->variant)) ++c->variant;
    c->fuse = cfg->fuse_steps > 0 ? std::min(cfg->fuse_steps, max_fuse(c)) : 1;
    if (d.dim == 3 && c->fuse == 2)   // two steps per launch: the two-step kernel
        c->variant = at3_variant_ok(&c->cfg, 15) ? 15 : 16;
    hipError_t e = hipSuccess;
    if (cfg->delay_mode == AT_DELAY_GENERATE)
        e = launch_delays(c->delays, cfg->nsteps_max, d.F, cfg->L, d.m, cfg->delay_dist,
                          cfg->delay_seed, c->st);
    else if (cfg->nsteps_max > 0)
        e = hipMemcpyAsync(c->delays, cfg->delays_host, (size_t)(cfg->nsteps_max * d.F),
                           hipMemcpyHostToDevice, c->st);
    if (e == hipSuccess)
        e = launch_fill(c->ring, (int64_t)L.R * (int64_t)ring_level_doubles(cfg, d), 0.0, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e != hipSuccess) {
        delete c;
        return fail(AT_ERR_HIP, "at_init: %s", hipGetErrorString(e));
    }
    *out = c;
    return AT_OK;
}

void at_free(at_ctx *c)
{
    if (!c) return;
    drop_graph(c);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    delete c;
}

at_status at_set_graph(at_ctx *c, int32_t use_graph)
{
    if (!c) return fail(AT_ERR_ARG, "null context");
    if (use_graph != 0 && use_graph != 1) return fail(AT_ERR_ARG, "use_graph must be 0 or 1");
    c->use_graph = use_graph;
    if (!use_graph) drop_graph(c);
    return AT_OK;
}

at_status at_set_debug(at_ctx *c, int32_t flags)
{
    if (!c) return fail(AT_ERR_ARG, "null context");
    if (flags & ~AT_DEBUG_POISON_RING) return fail(AT_ERR_ARG, "unknown debug flags 0x%x", flags);
    if ((flags & AT_DEBUG_POISON_RING) && c->cfg.record)
        return fail(AT_ERR_STATE, "ring poisoning is not available in record mode (the adjoint "
                                  "re-reads every level)");
    const bool was = c->debug & AT_DEBUG_POISON_RING;
    c->debug = flags;
    if ((flags & AT_DEBUG_POISON_RING) && !was) {
        if (c->n == 0) AT_HIP(clear_ring(c));
        else AT_HIP(poison_ring(c, c->n));
    }
    return AT_OK;
}

at_status at_set_fuse(at_ctx *c, int32_t s)
{
    if (!c) return fail(AT_ERR_ARG, "null context");
    if (s < 1 || s > kMaxFuse) return fail(AT_ERR_ARG, "fuse_steps must be in 1..%d", kMaxFuse);
    const int mf = max_fuse(c);
    if (s > mf) return fail(AT_ERR_ARG, "fuse_steps %d exceeds the limit %d of this grid", s, mf);
    c->fuse = s;
    if (c->d.dim == 3) {   // 3D: the kernel variant follows the steps per launch
        if (s == 2 && !at3_is_fused(c->variant))
            c->variant = at3_variant_ok(&c->cfg, 15) ? 15 : 16;
        if (s == 1) c->variant = at3_single_variant(&c->cfg, c->variant);
    }
    return AT_OK;
}

at_status at_set_adjoint_fuse(at_ctx *c, int32_t s)
{
    if (!c) return fail(AT_ERR_ARG, "null context");
    if (s < 0 || s > kMaxFuse) return fail(AT_ERR_ARG, "adjoint steps per launch must be in 0..%d",
                                           kMaxFuse);
    if (s > 1) {
        if (c->d.dim != 1) return fail(AT_ERR_ARG, "the adjoint is 1D only");
        const int mf = adj_fuse_max(c->d, c->cfg.L);
        if (s > mf)
            return fail(AT_ERR_ARG, "%d reverse steps per launch exceed the limit %d of this grid",
                        s, mf);
    }
    c->adj_fuse = s;
    return AT_OK;
}

at_status at_set_variant(at_ctx *c, int32_t v)
{
    if (!c) return fail(AT_ERR_ARG, "null context");
    const int nv = c->d.dim == 1 ? 5 : at3_variants();
    if (v < 0 || v >= nv) return fail(AT_ERR_ARG, "variant must be in 0..%d", nv - 1);
    if (c->d.dim == 3 && !at3_variant_ok(&c->cfg, v))
        return fail(AT_ERR_ARG, "variant %d needs block widths that are multiples of its tile", v);
    if (c->d.dim == 1 && v == kWholeVariant) {
        if (whole_ppt(c) == 0)
            return fail(AT_ERR_ARG, "variant 4 needs the grid in one workgroup (N <= 256 x 16, "
                                    "N and the tile width multiples of 4)");
        c->variant = v;
        c->fuse = (int)std::min<int64_t>(std::max<int64_t>(c->cfg.nsteps_max, 1), INT32_MAX);
        return AT_OK;
    }
    if (c->d.dim == 1) {
        // 0: automatic; 1, 2, 3: 16, 8, 4 points per thread in fused launches
        const int p = v == 0 ? 0 : (v == 1 ? 16 : (v == 2 ? 8 : 4));
        if (p && c->d.W % p != 0)
            return fail(AT_ERR_ARG, "variant %d needs a tile width divisible by %d", v, p);
        c->d.fppt = p ? p : fused_ppt(c->d);
        c->fuse = std::min(c->fuse, max_fuse(c));
    } else {
        c->fuse = at3_is_fused(v) ? 2 : 1;   // 3D: two-step variants advance two steps per launch
    }
    c->variant = v;
    return AT_OK;
}

at_status at_query(const at_ctx *c, int64_t *n, int32_t *fuse, int32_t *R, int32_t *variant)
{
    if (!c) return fail(AT_ERR_ARG, "null context");
    if (n) *n = c->n;
    if (fuse) *fuse = c->fuse;
    if (R) *R = c->lay.R;
    if (variant) *variant = c->variant;
    return AT_OK;
}

at_status at_step(at_ctx *c, const double *u_in, double *u_out)
{
    if (!c || !u_in || !u_out) return fail(AT_ERR_ARG, "null argument");
    if (u_in == u_out) return fail(AT_ERR_ARG, "u_in and u_out must differ");
    if (c->n + 1 > c->cfg.nsteps_max) return fail(AT_ERR_STATE, "step %lld beyond nsteps_max",
                                                  (long long)c->n);
    if (c->cfg.record && c->n % c->cfg.ckpt_every == 0)
        AT_HIP(launch_copy(c->ckpt + (c->n / c->cfg.ckpt_every) * c->d.N, u_in, c->d.N, c->st));
    if (c->d.dim == 3) {                      // the face values of level n, from u_in
        const at_status sp = at3_publish(c, u_in, c->n);
        if (sp) return sp;
    }
    at_status st = launch_any(c, u_in, u_out, c->n, 1, 1);
    if (st) return st;
    c->n += 1;
    AT_HIP(poison_ring(c, c->n));
    return AT_OK;
}

namespace {

// the launch sequence of at_run on c->st (recorded into a graph when c->st is
// a capturing stream); advances c->n
at_status run_launches(at_ctx *c, double *u, double *scratch, int64_t nsteps)
{
    double *cur = u, *oth = scratch;
    int64_t left = nsteps;
    const int64_t C = c->cfg.ckpt_every;
    if (c->d.dim == 3 && nsteps > 0) {        // the face values of level n, from u
        const at_status sp = at3_publish(c, u, c->n);
        if (sp) return sp;
    }
    while (left > 0) {
        int64_t s = std::min<int64_t>(c->fuse, left);
        if (c->cfg.record) {
            if (c->n % C == 0)
                AT_HIP(launch_copy(c->ckpt + (c->n / C) * c->d.N, cur, c->d.N, c->st));
            s = std::min<int64_t>(s, C - c->n % C);
        }
        // 1D without the edge tape: only the last L + m - 1 levels of a launch
        // reach the ring (the next launch reads no older level)
        at_status st = launch_any(c, cur, oth, c->n, (int)s,
                                  (c->d.dim == 1 && !c->cfg.record) ? 2 : 1);
        if (st) return st;
        std::swap(cur, oth);
        c->n += s;
        left -= s;
        AT_HIP(poison_ring(c, c->n));
    }
    if (cur != u) AT_HIP(launch_copy(u, cur, field_doubles(c), c->st));
    return AT_OK;
}

}  // namespace

at_status at_run(at_ctx *c, double *u, double *scratch, int64_t nsteps)
{
    if (!c || !u || !scratch) return fail(AT_ERR_ARG, "null argument");
    if (u == scratch) return fail(AT_ERR_ARG, "u and scratch must differ");
    if (nsteps < 0) return fail(AT_ERR_ARG, "nsteps < 0");
    if (c->n + nsteps > c->cfg.nsteps_max)
        return fail(AT_ERR_STATE, "run to step %lld beyond nsteps_max %lld",
                    (long long)(c->n + nsteps), (long long)c->cfg.nsteps_max);
    if (!c->use_graph || nsteps == 0) return run_launches(c, u, scratch, nsteps);
    // graph replay: the cached graph applies when it was captured for the same
    // start step, length, fields and launch choices
    if (!(c->gexec && c->g_n0 == c->n && c->g_nsteps == nsteps && c->g_u == u &&
          c->g_s == scratch && c->g_fuse == c->fuse && c->g_variant == c->variant &&
          c->g_debug == c->debug)) {
        drop_graph(c);
        if (!c->cap) AT_HIP(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
        const int64_t n0 = c->n;
        hipStream_t own = c->st;
        c->st = c->cap;
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal);
        at_status st = AT_OK;
        if (e == hipSuccess) {
            st = run_launches(c, u, scratch, nsteps);
            hipError_t e2 = hipStreamEndCapture(c->cap, &g);
            if (e2 != hipSuccess && st == AT_OK) e = e2;
        }
        c->st = own;
        c->n = n0;
        if (st) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return fail(AT_ERR_HIP, "graph capture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            c->gexec = nullptr;
            return fail(AT_ERR_HIP, "graph instantiate: %s", hipGetErrorString(e));
        }
        c->g_n0 = n0;
        c->g_nsteps = nsteps;
        c->g_u = u;
        c->g_s = scratch;
        c->g_fuse = c->fuse;
        c->g_variant = c->variant;
        c->g_debug = c->debug;
    }
    AT_HIP(hipGraphLaunch(c->gexec, c->st));
    c->n += nsteps;
    return AT_OK;
}

at_status at_ws_capacity(const at_ctx *c, int64_t *max_tiles)
{
    if (!c || !max_tiles) return fail(AT_ERR_ARG, "null argument");
    *max_tiles = 0;
    if (c->d.dim == 3) {
        *max_tiles = at3_ws_capacity(&c->cfg);
        return AT_OK;
    }
    *max_tiles = ws1d_max_tiles(c->d.order, c->cfg.adv_mode == 1, c->d.W);
    return AT_OK;
}

at_status at_run_ws(at_ctx *c, double *u, double *scratch, int64_t nsteps, int32_t jitter,
                    uint64_t seed, int64_t spin_limit)
{
    if (!c || !u) return fail(AT_ERR_ARG, "null argument");
    if (c->cfg.record) return fail(AT_ERR_STATE, "the weakly-synchronous run has no record mode");
    if (c->cfg.arith != 0) return fail(AT_ERR_ARG, "the weakly-synchronous run uses arith 0");
    if (c->n != 0) return fail(AT_ERR_STATE, "the weakly-synchronous run starts at step 0");
    if (nsteps < 0 || nsteps > c->cfg.nsteps_max)
        return fail(AT_ERR_ARG, "nsteps must be in 0..nsteps_max");
    if (nsteps >= ((int64_t)1 << 31) - 1) return fail(AT_ERR_ARG, "nsteps too large");
    if (jitter < 0 || jitter > (1 << 20)) return fail(AT_ERR_ARG, "jitter must be in 0..2^20");
    const Derived &d = c->d;
    const int64_t spins = spin_limit > 0 ? spin_limit : ((int64_t)1 << 20);
    if (d.dim == 3) {
        if (!scratch || scratch == u)
            return fail(AT_ERR_ARG, "the 3D weakly-synchronous run needs a scratch field apart from u");
        const int64_t Wx = c->cfg.n[0] / c->cfg.p[0], Wy = c->cfg.n[1] / c->cfg.p[1];
        if (Wx % 64 != 0 || Wy % 8 != 0)
            return fail(AT_ERR_SHAPE, "3D weakly-synchronous run: block widths must be multiples "
                                      "of 64 (x) and 8 (y)");
        const int64_t maxb = at3_ws_capacity(&c->cfg);
        if (d.nb > maxb)
            return fail(AT_ERR_SHAPE, "%lld blocks, but at most %lld workgroups can be resident "
                                      "at once", (long long)d.nb, (long long)maxb);
        if (nsteps == 0) return AT_OK;
        int32_t *err = c->sync + d.nb;
        const at_status sp = at3_publish(c, u, 0);           // level 0's faces, announced below
        if (sp) return sp;
        AT_HIP(launch_ws_init(c->sync, d.nb, 0, err, c->st));
        int in_scratch = 0;
        const at_status st = at3_launch_ws(c, u, scratch, 0, nsteps, c->sync, err, c->delays,
                                           jitter, seed, spins, &in_scratch);
        if (st) return st;
        if (in_scratch) AT_HIP(launch_copy(u, scratch, field_doubles(c), c->st));
        int32_t herr = 0;
        AT_HIP(hipMemcpyAsync(&herr, err, sizeof herr, hipMemcpyDeviceToHost, c->st));
        AT_HIP(hipStreamSynchronize(c->st));
        if (herr != 0)
            return fail(AT_ERR_TIMEOUT, "a wait passed the spin limit; u and the delays are undefined");
        c->n = nsteps;
        return AT_OK;
    }
    int nt = 0, ppt = 0;
    if (!ws1d_shape(d.W, d.h, &nt, &ppt))
        return fail(AT_ERR_SHAPE, "tile width must be 256 q or 64 q with q in {1, 2, 4, 8, 16} "
                                  "(q >= 2 for order 4)");
    const bool linear = c->cfg.adv_mode == 1;
    const int64_t maxt = ws1d_max_tiles(d.order, linear, d.W);
    if (d.P > maxt)
        return fail(AT_ERR_SHAPE, "%lld tiles, but at most %lld workgroups can be resident at once",
                    (long long)d.P, (long long)maxt);
    if (nsteps == 0) return AT_OK;
    int32_t *err = c->sync + 2 * d.P;
    AT_HIP(launch_ws_init(c->sync, 2 * d.P, -1, err, c->st));
    Ws1D a{};
    a.u = u;
    a.ring = c->ring;
    a.cnt = c->sync;
    a.err = err;
    a.delays = c->delays;
    a.P = d.P;
    a.W = d.W;
    a.n0 = 0;
    a.nsteps = nsteps;
    a.spin_limit = spins;
    a.R = c->lay.R;
    a.L = c->cfg.L;
    a.stale = c->cfg.halo_mode;
    a.jitter = jitter;
    a.seed = seed;
    a.coef.nu = c->cfg.nu;
    a.coef.dt = c->cfg.dt;
    a.coef.c1 = d.c1[0];
    a.coef.c2 = d.c2[0];
    a.coef.cadv = c->cfg.adv_speed;
    AT_HIP(launch_ws1d(a, d.order, linear, c->st));
    int32_t herr = 0;
    AT_HIP(hipMemcpyAsync(&herr, err, sizeof herr, hipMemcpyDeviceToHost, c->st));
    AT_HIP(hipStreamSynchronize(c->st));
    if (herr != 0)
        return fail(AT_ERR_TIMEOUT, "a wait passed the spin limit; u and the delays are undefined");
    c->n = nsteps;
    return AT_OK;
}

at_status at_autotune(at_ctx *c, const double *u0, double *t1, double *t2, int32_t trial_steps,
                      int32_t *chosen)
{
    if (!c || !u0 || !t1 || !t2) return fail(AT_ERR_ARG, "null argument");
    if (c->n != 0) return fail(AT_ERR_STATE, "autotune needs a context at step 0");
    if (c->cfg.record) return fail(AT_ERR_STATE, "autotune is not available in record mode");
    if (trial_steps < 1 || trial_steps > c->cfg.nsteps_max)
        return fail(AT_ERR_ARG, "trial_steps must be in 1..nsteps_max");
    // 1D: (points per thread, steps per launch) pairs, the points per thread
    // as the variant (1, 2, 3: 16, 8, 4; those dividing the tile width);
    // 3D: the kernel variant (one or two steps per launch)
    std::vector<std::pair<int, int>> cands;       // (variant, steps per launch)
    if (c->d.dim == 1) {
        const Derived keep = c->d;
        for (int v = 1; v <= 3; ++v) {
            const int p = v == 1 ? 16 : (v == 2 ? 8 : 4);
            if (c->d.W % p != 0) continue;
            c->d.fppt = p;
            const int mf = max_fuse(c);
            for (int s : {1, 2, 3, 4, 6, 8, 10, 12, 16, 20, 24, 32, 40, 48, 56, 64})
                if (s <= mf && (s > 1 || v == 1)) cands.push_back({v, s});   // one step: one kernel
        }
        c->d = keep;
        if (whole_ppt(c) != 0) cands.push_back({kWholeVariant, 0});   // one launch per run
        if (cands.empty()) cands.push_back({c->variant, 1});
    } else {
        for (int v = 0; v < at3_variants(); ++v)
            if (at3_variant_ok(&c->cfg, v)) cands.push_back({v, at3_is_fused(v) ? 2 : 1});
    }
    hipEvent_t e0, e1;
    AT_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(AT_ERR_HIP, "at_autotune: hipEventCreate failed");
    }
    float best_ms = 1e30f;
    std::pair<int, int> best = cands[0];
    const int keep_graph = c->use_graph;
    c->use_graph = 0;                         // time the launches themselves
    at_status st = AT_OK;
    // select a candidate: the variant (1D: points per thread) and steps per launch
    auto choose = [&](std::pair<int, int> vs) {
        if (c->d.dim == 1 && vs.first == kWholeVariant) {
            c->d.fppt = fused_ppt(c->d);          // the regular layout, for the adjoint's rebuild
            c->variant = kWholeVariant;
            c->fuse = (int)std::min<int64_t>(c->cfg.nsteps_max, INT32_MAX);
            return;
        }
        if (c->d.dim == 1) {
            const int p = vs.first == 1 ? 16 : (vs.first == 2 ? 8 : 4);
            c->d.fppt = p;
        }
        c->variant = vs.first;
        c->fuse = vs.second;
    };
    for (size_t i = 0; i < cands.size() && st == AT_OK; ++i) {
        float ms_best = 1e30f;
        for (int rep = 0; rep < 2 && st == AT_OK; ++rep) {
            hipError_t e = clear_ring(c);
            if (e == hipSuccess) e = launch_copy(t1, u0, field_doubles(c), c->st);
            c->n = 0;
            choose(cands[i]);
            if (e == hipSuccess) e = hipEventRecord(e0, c->st);
            if (e == hipSuccess) st = at_run(c, t1, t2, trial_steps);
            if (e == hipSuccess && st == AT_OK) e = hipEventRecord(e1, c->st);
            if (e == hipSuccess && st == AT_OK) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess && st == AT_OK) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess && st == AT_OK)
                st = fail(AT_ERR_HIP, "at_autotune: %s", hipGetErrorString(e));
            ms_best = std::min(ms_best, ms);
        }
        if (st == AT_OK && ms_best < best_ms * 0.98f) { best_ms = ms_best; best = cands[i]; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->use_graph = keep_graph;
    c->n = 0;
    if (st) return st;
    choose(best);
    AT_HIP(clear_ring(c));
    AT_HIP(hipStreamSynchronize(c->st));
    if (chosen) *chosen = c->d.dim == 1 ? c->fuse : best.first;
    return AT_OK;
}

at_status at_delays_copy(const at_ctx *c, int8_t *host_out)
{
    if (!c || !host_out) return fail(AT_ERR_ARG, "null argument");
    AT_HIP(hipMemcpyAsync(host_out, c->delays, (size_t)(c->cfg.nsteps_max * c->d.F),
                          hipMemcpyDeviceToHost, c->st));
    AT_HIP(hipStreamSynchronize(c->st));
    return AT_OK;
}

at_status at_snapshot_bytes(const at_ctx *c, uint64_t *bytes)
{
    if (!c || !bytes) return fail(AT_ERR_ARG, "null argument");
    *bytes = align_up(8ull * field_doubles(c)) +
             align_up(8ull * c->lay.R * ring_level_doubles(&c->cfg, c->d)) + kAlign;
    return AT_OK;
}

at_status at_snapshot(at_ctx *c, const double *u, void *dev_buf)
{
    if (!c || !u || !dev_buf) return fail(AT_ERR_ARG, "null argument");
    const uint64_t nu = field_doubles(c), nr = (uint64_t)c->lay.R * ring_level_doubles(&c->cfg, c->d);
    char *b = (char *)dev_buf;
    AT_HIP(launch_copy((double *)b, u, nu, c->st));
    AT_HIP(launch_copy((double *)(b + align_up(8 * nu)), c->ring, nr, c->st));
    // the step counter, exact below 2^53, written by a kernel (no host buffer
    // has to outlive the call, so nothing waits)
    AT_HIP(launch_fill((double *)(b + align_up(8 * nu) + align_up(8 * nr)), 1, (double)c->n,
                       c->st));
    for (auto &e : c->snaps)
        if (e.first == dev_buf) { e.second = c->n; return AT_OK; }
    c->snaps.emplace_back(dev_buf, c->n);
    return AT_OK;
}

at_status at_restore(at_ctx *c, const void *dev_buf, double *u)
{
    if (!c || !u || !dev_buf) return fail(AT_ERR_ARG, "null argument");
    const uint64_t nu = field_doubles(c), nr = (uint64_t)c->lay.R * ring_level_doubles(&c->cfg, c->d);
    const char *b = (const char *)dev_buf;
    // a buffer this context filled: its step is known on the host; any other
    // buffer: read the step it holds (the only case that waits for the stream)
    int64_t step = -1;
    for (const auto &e : c->snaps)
        if (e.first == dev_buf) step = e.second;
    if (step < 0) {
        double nn = 0.0;
        AT_HIP(hipMemcpyAsync(&nn, b + align_up(8 * nu) + align_up(8 * nr), sizeof nn,
                              hipMemcpyDeviceToHost, c->st));
        AT_HIP(hipStreamSynchronize(c->st));
        if (!(nn >= 0.0) || nn > (double)c->cfg.nsteps_max || nn != floor(nn))
            return fail(AT_ERR_ARG, "buffer does not hold a snapshot of this context");
        step = (int64_t)nn;
    }
    AT_HIP(launch_copy(u, (const double *)b, nu, c->st));
    AT_HIP(launch_copy(c->ring, (const double *)(b + align_up(8 * nu)), nr, c->st));
    c->n = step;
    return AT_OK;
}

at_status at_stats(at_ctx *c, const double *u, double *out4)
{
    if (!c || !u || !out4) return fail(AT_ERR_ARG, "null argument");
    const int64_t n = field_doubles(c);
    AT_HIP(launch_stats(u, n, c->red, out4, c->st));
    return AT_OK;
}

at_status at_loss(at_ctx *c, const double *u, const double *target, double *lam, double *J_dev)
{
    if (!c || !u || !target || !J_dev) return fail(AT_ERR_ARG, "null argument");
    const int64_t n = field_doubles(c);
    AT_HIP(launch_loss(u, target, lam, n, c->red, J_dev, c->st));
    return AT_OK;
}

at_status at_adjoint(at_ctx *c, const double *lambda_T, double *grad_u0, double *grad_nu_dev)
{
    if (!c || !lambda_T || !grad_u0 || !grad_nu_dev) return fail(AT_ERR_ARG, "null argument");
    if (!c->cfg.record) return fail(AT_ERR_STATE, "at_adjoint needs a context in record mode");
    const Derived &d = c->d;
    const int64_t nend = c->n, C = c->cfg.ckpt_every, N = d.N;
    double *lcur = c->lam, *loth = c->lam + N;
    AT_HIP(launch_copy(lcur, lambda_T, N, c->st));
    AT_HIP(launch_fill(c->mu, (int64_t)c->lay.Rmu * d.P * 2 * d.h, 0.0, c->st));
    AT_HIP(launch_fill(c->gnu, 2 * c->lay.ngnu, 0.0, c->st));
    if (nend > 0) {
        for (int64_t a0 = ((nend - 1) / C) * C; a0 >= 0; a0 -= C) {
            const int64_t a1 = std::min(a0 + C, nend);
            AT_HIP(launch_copy(c->seg, c->ckpt + (a0 / C) * N, N, c->st));
            // rebuild levels a0+1 .. a1-1: fused launches that also store every
            // intermediate level (aligned layout), else one launch per step
            const bool fused = region_1d(d, 2).aligned;
            const int sr = fused ? max_fuse(c) : 1;
            for (int64_t n = a0; n + 1 < a1;) {
                const int s = (int)std::min<int64_t>(sr, a1 - 1 - n);
                at_status st = launch_1d(c, c->seg + (n - a0) * N, c->seg + (n + s - a0) * N, n, s,
                                         0, s > 1 ? c->seg + (n - a0) * N : nullptr);
                if (st) return st;
                n += s;
            }
            const int smax = adj_fuse_max(d, c->cfg.L);
            const int sadj = c->adj_fuse == 0 ? smax : (c->adj_fuse == 1 ? 0 : c->adj_fuse);
            for (int64_t nt = a1; sadj > 0 && nt > a0;) {
                const int s = (int)std::min<int64_t>(sadj, nt - a0);
                const RegionAdj rg = region_adj(d, s);
                AdjF f;
                f.lam_in = lcur;
                f.lam_out = loth;
                f.seg = c->seg;
                f.ring = c->ring;
                f.mu = c->mu;
                f.delays = c->delays;
                f.gnu = c->gnu;
                f.N = N;
                f.P = d.P;
                f.W = d.W;
                f.CH = rg.CH;
                f.nt = nt;
                f.seg_n0 = a0;
                f.nsteps_total = nend;
                f.S = s;
                f.Rmu = c->lay.Rmu;
                f.L = c->cfg.L;
                f.stale = c->cfg.halo_mode;
                f.RL = (int32_t)rg.RL;
                f.NT = rg.NT;
                f.nu = c->cfg.nu;
                f.dt = c->cfg.dt;
                f.c1 = d.c1[0];
                f.c2 = d.c2[0];
                f.cadv = c->cfg.adv_speed;
                const int64_t nblocks = (N + rg.CH - 1) / rg.CH;   // <= ngnu (CH >= 256)
                AT_HIP(launch_adj1d_fused(f, d.order, c->cfg.adv_mode == 1, rg.ppt, nblocks,
                                          adj1d_fused_lds_bytes(d.order, s, rg.NT, c->cfg.L),
                                          c->st));
                std::swap(lcur, loth);
                nt -= s;
            }
            for (int64_t n = a1 - 1; sadj == 0 && n >= a0; --n) {
                Adj1D a;
                a.lam_in = lcur;
                a.lam_out = loth;
                a.u = c->seg + (n - a0) * N;
                a.ring = c->ring;
                a.mu = c->mu;
                a.delays = c->delays;
                a.gnu = c->gnu;
                a.N = N;
                a.P = d.P;
                a.W = d.W;
                a.n = n;
                a.nsteps_total = nend;
                a.R = c->lay.R;
                a.Rmu = c->lay.Rmu;
                a.L = c->cfg.L;
                a.stale = c->cfg.halo_mode;
                a.mslot0 = (int32_t)(n % a.Rmu);
                a.pad0 = 0;
                a.nu = c->cfg.nu;
                a.dt = c->cfg.dt;
                a.c1 = d.c1[0];
                a.c2 = d.c2[0];
                a.cadv = c->cfg.adv_speed;
                AT_HIP(launch_adj1d(a, d.order, c->cfg.adv_mode == 1, adj_blocks(d), c->st));
                std::swap(lcur, loth);
            }
        }
    }
    AT_HIP(launch_copy(grad_u0, lcur, N, c->st));
    AT_HIP(launch_gnu_final(c->gnu, c->lay.ngnu, grad_nu_dev, c->st));
    return AT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched form: independent 1D instances advanced by shared launches
// ---------------------------------------------------------------------------

struct at_batch {
    int count = 0, order = 2;
    bool linear = false, fma = false;
    hipStream_t st = nullptr;
    std::vector<at_config> cfg;
    std::vector<Derived> d;
    std::vector<int> R;
    std::vector<int8_t *> delays;
    std::vector<double *> ring;
    std::vector<int64_t> ring_doubles;
    int64_t nsteps_max = 0;   // smallest over the instances
    int max_fuse = 1, fuse = 1;
    int ppt = 16;             // points per thread of the batched kernel (16, 8 or 4)
    int variant = 0;          // 0 automatic (16), 1, 2, 3: 16, 8, 4 points per thread
    int mf_ppt[3] = {1, 1, 1};   // steps-per-launch limit for 16, 8, 4 points per thread
    int64_t n = 0;
    // device tables (two slots: the run's s and its tail)
    Step1D *desc_dev[2] = {nullptr, nullptr};
    int2 *tbl_dev[2] = {nullptr, nullptr};
    int64_t tbl_cap = 0;
    int slot_s[2] = {0, 0};
    int64_t slot_blocks[2] = {0, 0};
    size_t slot_lds[2] = {0, 0};
    uint64_t slot_key[2] = {0, 0};
    std::vector<Step1D> hdesc[2];
    std::vector<int2> htbl[2];
    // cached graph of one whole run, captured on a private stream (the
    // caller's stream may be the null stream, which cannot be captured)
    hipStream_t cap = nullptr;
    bool has_graph = false;
    hipGraphExec_t gexec = nullptr;
    int64_t g_n0 = -1, g_nsteps = -1;
    int g_fuse = 0, g_ppt = 0;
    uint64_t g_key = 0;
};

namespace {

uint64_t ptr_key(double *const *u, double *const *s, int count)
{
    uint64_t h = 1469598103934665603ULL;
    for (int j = 0; j < count; ++j) {
        h = (h ^ (uint64_t)(uintptr_t)u[j]) * 1099511628211ULL;
        h = (h ^ (uint64_t)(uintptr_t)s[j]) * 1099511628211ULL;
    }
    return h;
}

void drop_graph(at_batch *b)
{
    if (b->has_graph) (void)hipGraphExecDestroy(b->gexec);
    b->has_graph = false;
    b->gexec = nullptr;
}

at_status batch_tables(at_batch *b, int slot, int s, double *const *u, double *const *scr,
                       uint64_t key)
{
    const uint64_t k2 = key ^ ((uint64_t)s * 0x9E3779B97F4A7C15ULL) ^
                        ((uint64_t)b->ppt * 0xD1B54A32D192ED03ULL);
    if (b->slot_s[slot] == s && b->slot_key[slot] == k2) return AT_OK;
    drop_graph(b);    // a cached graph reads these tables
    const int reg = kThreads * b->ppt;
    std::vector<Step1D> &D = b->hdesc[slot];
    std::vector<int2> &T = b->htbl[slot];
    D.resize(b->count);
    T.clear();
    size_t lds = 0;
    for (int j = 0; j < b->count; ++j) {
        Derived d = b->d[j];
        d.fppt = b->ppt;
        const Region1D rg = region_1d(d, s, false);
        Step1D &a = D[j];
        a.uin = u[j];
        a.uout = scr[j];
        a.ring = b->ring[j];
        a.delays = b->delays[j];
        a.N = d.N;
        a.P = d.P;
        a.W = d.W;
        a.n0 = 0;
        a.CH = rg.CH;
        a.s = s;
        a.R = b->R[j];
        a.NT = (int)((reg - 1) / d.W + 2);
        a.stale = b->cfg[j].halo_mode;
        a.publish = 2;        // no edge tape: the last D levels of a launch
        a.RL = (int32_t)rg.RL;
        a.slot0 = 0;          // set per launch by the batched kernel
        a.D = b->cfg[j].L + d.m - 1;
        a.levels = nullptr;
        a.nu = b->cfg[j].nu;
        a.dt = b->cfg[j].dt;
        a.c1 = d.c1[0];
        a.c2 = d.c2[0];
        a.cadv = b->cfg[j].adv_speed;
        a.A1 = a.dt * a.c1;
        a.A2 = a.dt * (a.nu * a.c2);
        const int64_t nch = (d.N + rg.CH - 1) / rg.CH;
        for (int64_t c = 0; c < nch; ++c) T.push_back(make_int2(j, (int)c));
        lds = std::max(lds, step1d_lds_bytes(b->order, s, a.NT, a.D, b->ppt, true));
    }
    if ((int64_t)T.size() > b->tbl_cap) return fail(AT_ERR_STATE, "batch block table overflow");
    AT_HIP(hipStreamSynchronize(b->st));
    AT_HIP(hipMemcpyAsync(b->desc_dev[slot], D.data(), D.size() * sizeof(Step1D),
                          hipMemcpyHostToDevice, b->st));
    AT_HIP(hipMemcpyAsync(b->tbl_dev[slot], T.data(), T.size() * sizeof(int2),
                          hipMemcpyHostToDevice, b->st));
    AT_HIP(hipStreamSynchronize(b->st));
    b->slot_s[slot] = s;
    b->slot_key[slot] = k2;
    b->slot_blocks[slot] = (int64_t)T.size();
    b->slot_lds[slot] = lds;
    return AT_OK;
}

// the launches of one run (recorded into a graph when capturing)
at_status batch_launches(at_batch *b, int64_t n0, int64_t nsteps, double *const *u,
                         double *const *scr, hipStream_t stream)
{
    int flip = 0;
    int64_t done = 0;
    while (done < nsteps) {
        const int s = (int)std::min<int64_t>(b->fuse, nsteps - done);
        const int slot = s == b->slot_s[0] ? 0 : 1;
        AT_HIP(launch_step1d_batch(b->desc_dev[slot], b->tbl_dev[slot], b->slot_blocks[slot],
                                   b->order, b->linear, b->fma, b->ppt, n0 + done, flip,
                                   b->slot_lds[slot], stream));
        flip ^= 1;
        done += s;
    }
    if (flip)
        for (int j = 0; j < b->count; ++j)
            AT_HIP(launch_copy(u[j], scr[j], b->d[j].N, stream));
    return AT_OK;
}

}  // namespace

extern "C" {

static at_status batch_layout(const at_config *cfgs, int32_t count, std::vector<Derived> &ds,
                              std::vector<uint64_t> &off_delays, std::vector<uint64_t> &off_ring,
                              std::vector<int> &Rs, uint64_t &off_desc, uint64_t &off_tbl,
                              int64_t &tbl_cap, int &smax, int (&mf_ppt)[3], uint64_t &total)
{
    if (!cfgs || count < 1) return fail(AT_ERR_ARG, "batch needs at least one configuration");
    ds.resize(count);
    off_delays.resize(count);
    off_ring.resize(count);
    Rs.resize(count);
    smax = kMaxFuse;
    for (int j = 0; j < count; ++j) {
        at_status st = derive(&cfgs[j], ds[j]);
        if (st) return fail(st, "instance %d: %s", j, g_err.c_str());
        ds[j].fppt = step1d_points_per_thread();        // the batched kernel's layout
        if (cfgs[j].dim != 1) return fail(AT_ERR_ARG, "instance %d: batched form is 1D", j);
        if (cfgs[j].record) return fail(AT_ERR_ARG, "instance %d: record mode not batched", j);
        if (cfgs[j].order != cfgs[0].order || cfgs[j].adv_mode != cfgs[0].adv_mode ||
            cfgs[j].arith != cfgs[0].arith)
            return fail(AT_ERR_ARG, "instance %d: all instances share order, adv_mode and arith", j);
        if (ds[j].W % step1d_points_per_thread() != 0)
            return fail(AT_ERR_SHAPE, "instance %d: tile width %lld is not a multiple of %d", j,
                        (long long)ds[j].W, step1d_points_per_thread());
        smax = std::min(smax, max_fuse_1d(ds[j]));
    }
    // steps-per-launch limit for each points-per-thread choice (16 gives the
    // largest regions, so the rings sized for it serve every choice)
    const int ppts[3] = {16, 8, 4};
    for (int i = 0; i < 3; ++i) {
        mf_ppt[i] = kMaxFuse;
        for (int j = 0; j < count; ++j) {
            Derived d = ds[j];
            d.fppt = ppts[i];
            mf_ppt[i] = std::min(mf_ppt[i], max_fuse_1d(d));
        }
        mf_ppt[i] = std::min(mf_ppt[i], smax);
    }
    uint64_t off = 0;
    tbl_cap = 0;
    for (int j = 0; j < count; ++j) {
        Rs[j] = cfgs[j].L + ds[j].m - 1 + smax;
        off_delays[j] = off;
        off = align_up(off + (uint64_t)cfgs[j].nsteps_max * (uint64_t)ds[j].F);
        off_ring[j] = off;
        off = align_up(off + 8ull * (uint64_t)Rs[j] * (uint64_t)ds[j].P * 2 * ds[j].h);
        int64_t chmin = ds[j].N;
        for (int i = 0; i < 3; ++i) {
            Derived d = ds[j];
            d.fppt = ppts[i];
            for (int s = 1; s <= mf_ppt[i]; ++s)
                chmin = std::min<int64_t>(chmin, region_1d(d, s, false).CH);
        }
        tbl_cap += (ds[j].N + chmin - 1) / chmin;
    }
    off_desc = off;
    off = align_up(off + 2ull * count * sizeof(Step1D));
    off_tbl = off;
    off = align_up(off + 2ull * (uint64_t)tbl_cap * sizeof(int2));
    total = off;
    return AT_OK;
}

at_status at_batch_workspace_bytes(const at_config *cfgs, int32_t count, uint64_t *bytes)
{
    if (!bytes) return fail(AT_ERR_ARG, "null output");
    std::vector<Derived> ds;
    std::vector<uint64_t> od, orr;
    std::vector<int> Rs;
    uint64_t odesc, otbl, total;
    int64_t cap;
    int smax, mfp[3];
    at_status st = batch_layout(cfgs, count, ds, od, orr, Rs, odesc, otbl, cap, smax, mfp, total);
    if (st) return st;
    *bytes = total;
    return AT_OK;
}

at_status at_batch_init(const at_config *cfgs, int32_t count, void *workspace,
                        uint64_t workspace_bytes, at_batch **out)
{
    if (!out) return fail(AT_ERR_ARG, "null output");
    *out = nullptr;
    std::vector<Derived> ds;
    std::vector<uint64_t> od, orr;
    std::vector<int> Rs;
    uint64_t odesc, otbl, total;
    int64_t cap;
    int smax, mfp[3];
    at_status st = batch_layout(cfgs, count, ds, od, orr, Rs, odesc, otbl, cap, smax, mfp, total);
    if (st) return st;
    if (!workspace || ((uintptr_t)workspace) % kAlign)
        return fail(AT_ERR_ARG, "workspace NULL or not 256-byte aligned");
    if (workspace_bytes < total)
        return fail(AT_ERR_NOMEM, "workspace %llu bytes, need %llu",
                    (unsigned long long)workspace_bytes, (unsigned long long)total);
    for (int j = 0; j < count; ++j) {
        const at_config *c = &cfgs[j];
        if (c->delay_mode != AT_DELAY_HOST) continue;
        for (int64_t n = 0; n < c->nsteps_max; ++n) {
            const int64_t lim = std::min<int64_t>(c->L, std::max<int64_t>(0, n - ds[j].m + 1));
            for (int64_t f = 0; f < ds[j].F; ++f) {
                const int k = c->delays_host[n * ds[j].F + f];
                if (k < 0 || k > lim)
                    return fail(AT_ERR_DELAY, "instance %d: delay k[%lld][%lld] = %d outside 0..%lld",
                                j, (long long)n, (long long)f, k, (long long)lim);
            }
        }
    }
    at_batch *b = new (std::nothrow) at_batch;
    if (!b) return fail(AT_ERR_NOMEM, "host allocation failed");
    char *base = (char *)workspace;
    b->count = count;
    b->order = cfgs[0].order;
    b->linear = cfgs[0].adv_mode == 1;
    b->fma = cfgs[0].arith == 1;
    b->st = (hipStream_t)cfgs[0].stream;
    b->cfg.assign(cfgs, cfgs + count);
    b->d = ds;
    b->R = Rs;
    for (int i = 0; i < 3; ++i) b->mf_ppt[i] = mfp[i];
    b->ppt = 16;
    b->max_fuse = mfp[0];
    b->fuse = cfgs[0].fuse_steps > 0 ? std::min<int>(cfgs[0].fuse_steps, b->max_fuse) : 1;
    b->nsteps_max = cfgs[0].nsteps_max;
    b->tbl_cap = cap;
    for (int s = 0; s < 2; ++s) {
        b->desc_dev[s] = (Step1D *)(base + odesc + (uint64_t)s * count * sizeof(Step1D));
        b->tbl_dev[s] = (int2 *)(base + otbl + (uint64_t)s * cap * sizeof(int2));
    }
    hipError_t e = hipSuccess;
    for (int j = 0; j < count && e == hipSuccess; ++j) {
        const at_config *c = &cfgs[j];
        b->cfg[j].delays_host = nullptr;
        b->nsteps_max = std::min<int64_t>(b->nsteps_max, c->nsteps_max);
        b->delays.push_back((int8_t *)(base + od[j]));
        b->ring.push_back((double *)(base + orr[j]));
        b->ring_doubles.push_back((int64_t)Rs[j] * ds[j].P * 2 * ds[j].h);
        if (c->delay_mode == AT_DELAY_GENERATE)
            e = launch_delays(b->delays[j], c->nsteps_max, ds[j].F, c->L, ds[j].m, c->delay_dist,
                              c->delay_seed, b->st);
        else if (c->nsteps_max > 0)
            e = hipMemcpyAsync(b->delays[j], c->delays_host, (size_t)(c->nsteps_max * ds[j].F),
                               hipMemcpyHostToDevice, b->st);
        if (e == hipSuccess) e = launch_fill(b->ring[j], b->ring_doubles[j], 0.0, b->st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->st);
    if (e != hipSuccess) {
        delete b;
        return fail(AT_ERR_HIP, "at_batch_init: %s", hipGetErrorString(e));
    }
    *out = b;
    return AT_OK;
}

void at_batch_free(at_batch *b)
{
    if (!b) return;
    drop_graph(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
}

at_status at_batch_set_fuse(at_batch *b, int32_t s)
{
    if (!b) return fail(AT_ERR_ARG, "null batch");
    if (s < 1 || s > b->max_fuse)
        return fail(AT_ERR_ARG, "fuse_steps must be in 1..%d for this batch", b->max_fuse);
    b->fuse = s;
    return AT_OK;
}

at_status at_batch_set_variant(at_batch *b, int32_t v)
{
    if (!b) return fail(AT_ERR_ARG, "null batch");
    if (v < 0 || v > 3) return fail(AT_ERR_ARG, "batch variant must be in 0..3");
    const int idx = v <= 1 ? 0 : v - 1;               // 16, 8, 4 points per thread
    b->variant = v;
    b->ppt = idx == 0 ? 16 : (idx == 1 ? 8 : 4);
    b->max_fuse = b->mf_ppt[idx];
    b->fuse = std::min(b->fuse, b->max_fuse);
    b->slot_s[0] = b->slot_s[1] = 0;                  // tables are rebuilt for the new layout
    drop_graph(b);
    return AT_OK;
}

at_status at_batch_reset(at_batch *b)
{
    if (!b) return fail(AT_ERR_ARG, "null batch");
    for (int j = 0; j < b->count; ++j)
        AT_HIP(launch_fill(b->ring[j], b->ring_doubles[j], 0.0, b->st));
    b->n = 0;
    return AT_OK;
}

at_status at_batch_run(at_batch *b, double *const *u, double *const *scr, int64_t nsteps,
                       int32_t use_graph)
{
    if (!b || !u || !scr) return fail(AT_ERR_ARG, "null argument");
    if (nsteps < 0) return fail(AT_ERR_ARG, "nsteps < 0");
    if (b->n + nsteps > b->nsteps_max)
        return fail(AT_ERR_STATE, "batch run to step %lld beyond nsteps_max %lld",
                    (long long)(b->n + nsteps), (long long)b->nsteps_max);
    for (int j = 0; j < b->count; ++j)
        if (!u[j] || !scr[j] || u[j] == scr[j]) return fail(AT_ERR_ARG, "instance %d: bad fields", j);
    if (nsteps == 0) return AT_OK;
    const uint64_t key = ptr_key(u, scr, b->count);
    if (use_graph && b->has_graph && b->g_n0 == b->n && b->g_nsteps == nsteps &&
        b->g_fuse == b->fuse && b->g_ppt == b->ppt && b->g_key == key) {
        AT_HIP(hipGraphLaunch(b->gexec, b->st));
        b->n += nsteps;
        return AT_OK;
    }
    at_status st = batch_tables(b, 0, b->fuse, u, scr, key);
    if (st) return st;
    const int tail = (int)(nsteps % b->fuse);
    if (tail && nsteps > b->fuse) {
        st = batch_tables(b, 1, tail, u, scr, key);
        if (st) return st;
    } else if (tail) {
        st = batch_tables(b, 0, tail, u, scr, key);    // a single short launch
        if (st) return st;
    }
    if (!use_graph) {
        st = batch_launches(b, b->n, nsteps, u, scr, b->st);
        if (st) return st;
        b->n += nsteps;
        return AT_OK;
    }
    drop_graph(b);
    if (!b->cap) AT_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    hipGraph_t g;
    AT_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    st = batch_launches(b, b->n, nsteps, u, scr, b->cap);
    hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (st) return st;
    if (e != hipSuccess) return fail(AT_ERR_HIP, "graph capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(AT_ERR_HIP, "graph instantiate: %s", hipGetErrorString(e));
    b->has_graph = true;
    b->g_n0 = b->n;
    b->g_nsteps = nsteps;
    b->g_fuse = b->fuse;
    b->g_ppt = b->ppt;
    b->g_key = key;
    AT_HIP(hipGraphLaunch(b->gexec, b->st));
    b->n += nsteps;
    return AT_OK;
}

at_status at_batch_autotune(at_batch *b, double *const *u0, double *const *t1,
                            double *const *t2, int32_t trial_steps, int32_t *chosen)
{
    if (!b || !u0 || !t1 || !t2) return fail(AT_ERR_ARG, "null argument");
    if (b->n != 0) return fail(AT_ERR_STATE, "autotune needs a batch at step 0");
    if (trial_steps < 1 || trial_steps > b->nsteps_max)
        return fail(AT_ERR_ARG, "trial_steps must be in 1..nsteps_max");
    static const int cands[] = {1, 2, 3, 4, 6, 8, 10, 12, 16, 20, 24, 32, 40, 48, 56, 64};
    hipEvent_t e0, e1;
    AT_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(AT_ERR_HIP, "at_batch_autotune: hipEventCreate failed");
    }
    // points per thread (variants 1, 2, 3: 16, 8, 4) and steps per launch
    float best_ms = 1e30f;
    int best_s = 1, best_v = 1;
    at_status st = AT_OK;
    for (int v = 1; v <= 3 && st == AT_OK; ++v) {
        st = at_batch_set_variant(b, v);
        // largest steps per launch first: a smaller count must be 2% faster to
        // replace it (fewer launches, and fewer launch tails, on a near tie)
        for (int ci = (int)(sizeof(cands) / sizeof(cands[0])) - 1; ci >= 0; --ci) {
            const int s = cands[ci];
            if (st != AT_OK) break;
            if (s > b->max_fuse) continue;
            float ms_best = 1e30f;
            for (int rep = 0; rep < 2 && st == AT_OK; ++rep) {
                st = at_batch_reset(b);
                hipError_t e = hipSuccess;
                for (int j = 0; j < b->count && st == AT_OK && e == hipSuccess; ++j)
                    e = launch_copy(t1[j], u0[j], b->d[j].N, b->st);
                b->fuse = s;
                if (st == AT_OK && e == hipSuccess) e = hipEventRecord(e0, b->st);
                if (st == AT_OK && e == hipSuccess) st = at_batch_run(b, t1, t2, trial_steps, 0);
                if (st == AT_OK && e == hipSuccess) e = hipEventRecord(e1, b->st);
                if (st == AT_OK && e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (st == AT_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess && st == AT_OK)
                    st = fail(AT_ERR_HIP, "at_batch_autotune: %s", hipGetErrorString(e));
                ms_best = std::min(ms_best, ms);
            }
            if (st == AT_OK && ms_best < best_ms * 0.98f) {
                best_ms = ms_best;
                best_s = s;
                best_v = v;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) { b->n = 0; return st; }
    st = at_batch_set_variant(b, best_v);
    if (st) return st;
    st = at_batch_reset(b);
    if (st) return st;
    AT_HIP(hipStreamSynchronize(b->st));
    b->fuse = best_s;
    if (chosen) *chosen = best_s;
    return AT_OK;
}

at_status at_batch_query(const at_batch *b, int64_t *n, int32_t *fuse, int32_t *max_fuse,
                         int32_t *variant)
{
    if (!b) return fail(AT_ERR_ARG, "null batch");
    if (n) *n = b->n;
    if (fuse) *fuse = b->fuse;
    if (max_fuse) *max_fuse = b->max_fuse;
    if (variant) *variant = b->variant;
    return AT_OK;
}

}  // extern "C"
