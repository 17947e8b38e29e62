/*
 * at.h -- C ABI of libat.so, the MI355X (gfx950) stepper for explicit
 * time-marching of viscous Burgers' equation with asynchrony-tolerant (AT)
 * finite differences at subdomain boundaries, after Aditya, Gysi,
 * Kwasniewski, Hoefler, Donzis and Chen, "A scalable weakly-synchronous
 * algorithm for solving partial differential equations" (arXiv:1911.05769).
 *
 * The method (paper sections 2, 3 and 5.2):
 *   * The grid is split into P subdomains ("processing elements" in the
 *     paper, tiles of one device-resident grid here).  A point whose stencil
 *     reaches into another tile reads that tile's edge through a halo whose
 *     value may lag the current level n by a delay k, 0 <= k <= L
 *     (section 2).  Delays are prescribed per directed face and per step.
 *   * The halo value is extrapolated in time from the m most recent
 *     available levels n-k, n-k-1, ... of the neighbour's edge (the AT
 *     schemes, section 2, Eqs. (1)-(2): weights (k+1, -k) for m = 2).  The
 *     stencil itself is the standard central one (section 5.2 splits AT into
 *     "halo approximation" and "unchanged stencil").  Order 4 uses m = 3
 *     (quadratic Newton extrapolation in time; the paper defers the 4th-order
 *     coefficients to another article).
 *   * Central differences, forward Euler (section 3.2), for
 *     u_t + u u_x = nu u_xx (1D) and u_i,t + u_j d_j u_i = nu d_j d_j u_i (3D
 *     vector, section 3.1, Eq. (4)), periodic domain of side `length`; in 3D
 *     optionally with passive scalars phi_s,t + u_j d_j phi_s =
 *     alpha_s d_j d_j phi_s (the second line of Eq. (4)), each advected by
 *     the velocity and carried through the same AT halos.
 *   * The neighbour edges of past levels live in a circular buffer ("ring")
 *     of R levels, the analogue of the paper's circular receive buffers of
 *     T entries (section 5.2, Algorithm 2, Table 1).
 *
 * Conventions for every call:
 *   * All field pointers (u, scratch, lambda, gradients, targets, outputs of
 *     reductions) are DEVICE pointers to contiguous binary64 arrays owned by
 *     the caller.  1D fields are double[n0].  3D fields are
 *     double[3 + nscalars][nz][ny][nx] (component-major, x fastest:
 *     u_x, u_y, u_z, then the scalars).
 *   * The caller also owns the workspace (device memory of at least
 *     at_workspace_bytes() bytes, 256-byte aligned).  The library never
 *     allocates or frees device memory.  The opaque handles (at_ctx,
 *     at_batch) hold host-side state only.
 *   * Calls are asynchronous on the stream given in the configuration unless
 *     stated otherwise; results meant for the host are written to device
 *     memory.  Calls on one context must not overlap.
 *   * Every call returns an at_status; on failure it changes nothing it
 *     documents as output, and at_last_error() returns a message.  No call
 *     aborts or throws.
 */
#ifndef AT_H
#define AT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AT_ABI_VERSION 4
#define AT_MAX_SCALARS 4      /* passive scalars a 3D context may carry         */

typedef enum {
    AT_OK = 0,
    AT_ERR_ARG = -1,     /* invalid argument or configuration field        */
    AT_ERR_SHAPE = -2,   /* n % p != 0, tile narrower than the stencil, ... */
    AT_ERR_DELAY = -3,   /* a delay outside 0..min(L, max(0, n-m+1))       */
    AT_ERR_HIP = -4,     /* a HIP runtime call failed (message kept)       */
    AT_ERR_NOMEM = -5,   /* workspace too small                            */
    AT_ERR_STATE = -6,   /* call not valid in the context's current state  */
    AT_ERR_TIMEOUT = -7  /* a bounded wait of the weakly-synchronous run gave up */
} at_status;

/* Delay sources and distributions. */
#define AT_DELAY_GENERATE 0   /* k[n][f] from the counter-based generator      */
#define AT_DELAY_HOST 1       /* k[n][f] copied from delays_host (validated)   */
#define AT_DIST_UNIFORM 0     /* k uniform on {0..L}                           */
#define AT_DIST_HALF_ZERO 1   /* k = 0 with probability 1/2, else {1..L}       */

typedef struct at_config {
    int32_t abi_version;      /* must equal AT_ABI_VERSION                        */
    int32_t dim;              /* 1 (scalar) or 3 (vector, 3 components + scalars) */
    int64_t n[3];             /* points per axis x, y, z (1D: n[1] = n[2] = 1)    */
    int32_t p[3];             /* tiles per axis (1D: p[1] = p[2] = 1)             */
    int32_t order;            /* 2 or 4 (3D: 2); halo width h = order / 2,
                                 extrapolation levels m = 2 (order 2), 3 (order 4) */
    int32_t L;                /* maximum delay, 0..15 (section 2)                 */
    int32_t halo_mode;        /* 0: AT extrapolation; 1: standard scheme on the
                                 delayed level n-k (the paper's negative control)  */
    int32_t adv_mode;         /* 0: Burgers u u_x; 1 (1D only): linear
                                 advection c u_x with c = adv_speed                */
    double nu;                /* viscosity, >= 0                                  */
    double dt;                /* time step, > 0, constant for the run             */
    double length;            /* side of the periodic domain (dx = length / n)    */
    double adv_speed;         /* c for adv_mode 1                                 */
    int32_t delay_mode;       /* AT_DELAY_GENERATE or AT_DELAY_HOST               */
    int32_t delay_dist;       /* AT_DIST_* (generate mode)                        */
    uint64_t delay_seed;      /* generator seed (generate mode)                   */
    const int8_t *delays_host;/* host array int8[nsteps_max][F] (host mode);
                                 F = 2*p[0] (1D) or 6*p[0]*p[1]*p[2] (3D);
                                 face f = 2*tile + side (1D), 6*block + 2*axis +
                                 side (3D), side 0 = low, 1 = high; the block
                                 index is (bz*p[1] + by)*p[0] + bx               */
    int64_t nsteps_max;       /* steps the context may advance in total          */
    int32_t record;           /* 1: keep what at_adjoint needs (1D only)          */
    int32_t ckpt_every;       /* record mode: checkpoint interval C >= 1          */
    int32_t fuse_steps;       /* steps per launch s (1 = one launch per step);
                                 0 = let at_autotune choose (default 1 until then) */
    int32_t arith;            /* 0: each formula evaluated in the fixed order
                                 with separate roundings (bit-identical to a
                                 reference evaluating the same order);
                                 1 (1D only): fused multiply-adds with dt*c1 and
                                 dt*nu*c2 folded, u' = u + A2*T2 - (a*A1)*T1 --
                                 fewer instructions, same binary64 precision,
                                 results differ in the last bits */
    int32_t nscalars;         /* 3D: passive scalars 0..AT_MAX_SCALARS (1D: 0)    */
    int32_t reserved1;        /* must be 0                                        */
    double alpha[AT_MAX_SCALARS]; /* diffusivity of each scalar, finite, >= 0;
                                 entries past nscalars are ignored               */
    void *stream;             /* hipStream_t for all work of this context         */
    void *workspace;          /* device memory owned by the caller                */
    uint64_t workspace_bytes;
} at_config;

typedef struct at_ctx at_ctx;

/* Bytes of device workspace needed by `cfg` (the workspace fields are
 * ignored).  Host-only; no device work. */
at_status at_workspace_bytes(const at_config *cfg, uint64_t *bytes);

/* Validate `cfg`, lay out the workspace, fill the delay array k[n][f]
 * (section 2; generate mode: SplitMix64 output of seed + gamma*(1 + n*F + f),
 * mapped to the distribution, then clamped to min(k, max(0, n - m + 1)) so no
 * level below 0 is read -- the start-up synchrony of Algorithm 2; host mode:
 * copied after checking every entry against that bound, AT_ERR_DELAY if one
 * fails) and clear the ring.  The context starts at step n = 0.  Synchronises
 * the stream once before returning. */
at_status at_init(const at_config *cfg, at_ctx **out);

/* Release the handle (host memory only; the workspace stays the caller's). */
void at_free(at_ctx *ctx);

/* One step n -> n+1 in the one-launch-per-step form: reads u_in (level n),
 * writes u_out (level n+1) and the ring.  1D: the step publishes level n's
 * tile edges.  3D: the call first copies level n's block faces from u_in to
 * the ring, and the step publishes level n+1's (a run does the copy once).
 * u_in and u_out must not overlap.  AT_ERR_STATE past nsteps_max. */
at_status at_step(at_ctx *ctx, const double *u_in, double *u_out);

/* Advance nsteps steps from the current level held in u; the result is left
 * in u.  scratch is a second field of the same size.  Steps are fused s at a
 * time (fuse_steps or the autotuned value); results are bit-identical for
 * every s.  A 1D launch of s steps writes to the ring the tile edges of its
 * last L + m - 1 levels (the levels a later step reads; earlier ones stay in
 * the launch's LDS history), or of every level in record mode, where the ring
 * is the adjoint's edge tape.  Record mode also stores a checkpoint of u
 * every ckpt_every steps, counted from n = 0. */
at_status at_run(at_ctx *ctx, double *u, double *scratch, int64_t nsteps);

/* Weakly-synchronous run with EMERGENT delays (paper section 5.2, Algorithm 2;
 * the AT halos of section 2, Eqs. (1)-(2)).  From step 0, arith 0, no record
 * mode.  Each tile (1D) or block (3D) is one workgroup that advances without
 * any global barrier: after each step it writes its edges / block faces into
 * the ring with device-coherent stores and then announces the level on a
 * counter; before step n it reads the neighbours' newest announced level t
 * and uses the delay k = n - min(t, n) per face, waiting only while k would
 * exceed min(L, max(0, n - m + 1)).  The delays actually used are stored in
 * the context's delay array in place of the prescribed ones (at_delays_copy
 * returns them), so a replay with those delays (the oracle, or a fresh
 * context in host-delay mode) reproduces u exactly.
 *   u          device field, level 0 in, level nsteps out
 *   scratch    3D: a second device field of the same size (not u); 1D: unused
 *   jitter     0: none; J > 0: before each step a tile idles a pseudo-random
 *              0..J units of about 128 clocks (hash of seed, tile, step),
 *              emulating uneven arrival
 *   spin_limit polls of a counter before a wait gives up (<= 0: 2^20)
 * Requirements: 1D: tile width W = 256 q or 64 q with q in {1, 2, 4, 8, 16}
 * (q >= 2 for order 4; one workgroup of 256 threads, or of one wave, per
 * tile); 3D: block widths multiples of 64 (x) and 8 (y).  All tiles or
 * blocks must be resident at once (else AT_ERR_SHAPE: the launch is
 * cooperative; at_ws_capacity gives the limit).  Synchronous: returns after
 * the run.  AT_ERR_TIMEOUT if a wait gave up: every workgroup then leaves
 * early, u and the delays are undefined and the step count stays 0.  On
 * success the context is at step nsteps and may continue with at_step /
 * at_run. */
at_status at_run_ws(at_ctx *ctx, double *u, double *scratch, int64_t nsteps, int32_t jitter,
                    uint64_t seed, int64_t spin_limit);

/* The largest tile (1D) or block (3D) count for which at_run_ws can run this
 * context's configuration on the current device (all resident at once), or 0
 * when its tile or block shape is not one at_run_ws supports. */
at_status at_ws_capacity(const at_ctx *ctx, int64_t *max_tiles);

/* Graph replay of at_run: 1 captures the launch sequence of an at_run call
 * into a HIP graph (on a private stream the library creates; no launch runs
 * during the capture) and replays it on the context's stream; the graph is
 * kept and replayed again while a later call has the same start step, step
 * count, fields, steps per launch, kernel variant and debug flags (for
 * example a run restarted from the same snapshot), and captured anew
 * otherwise.  0 (default): launches are issued one by one.  Results are
 * bit-identical either way.  The graph removes the per-launch host cost of
 * the one-launch-per-step form on small grids. */
at_status at_set_graph(at_ctx *ctx, int32_t use_graph);

/* Debug aids.  AT_DEBUG_POISON_RING: after every launch, every ring slot that
 * no later step may read is overwritten with NaN (1D: levels below n - L -
 * m + 1 once level n is reached; 3D: below n - L - 1), and the ring starts
 * filled with NaN instead of zeros, so a step reading a level outside the
 * window that the delay bound L allows (section 2) would carry a NaN into
 * the field.  Results are unchanged when the indexing is right.  Costs one
 * pass over the ring per launch.  Not available in record mode
 * (AT_ERR_STATE): the adjoint re-reads every level. */
#define AT_DEBUG_POISON_RING 1
at_status at_set_debug(at_ctx *ctx, int32_t flags);

/* Choose the launch shape -- 1D: points per thread (the variant, 16, 8 or 4
 * among those dividing the tile width) together with steps per launch s, and
 * the whole-grid variant 4 where the grid fits one workgroup; 3D:
 * the kernel variant (including the two-step variants) -- nothing that
 * changes results -- by timing `trial_steps` steps from u0 for each
 * candidate; requires n == 0 and leaves the context at n = 0 with the ring
 * cleared.  u0 is not modified; t1 and t2 are two scratch fields.
 * Synchronises the stream.  *chosen receives s (1D; nsteps_max for variant
 * 4) or the variant (3D); at_query returns both. */
at_status at_autotune(at_ctx *ctx, const double *u0, double *t1, double *t2,
                      int32_t trial_steps, int32_t *chosen);

/* Kernel variant of a 3D context (results are bit-identical for every
 * variant; at_autotune picks one for 3D contexts): 0..5 LDS-tiled with
 * per-point halos (tile rows, prefetch depth, register budget), 6..8 and
 * 12..14 LDS-tiled with halos in the tile rims and 1 to 4 planes prefetched
 * (block widths multiples of the tile, AT_ERR_ARG otherwise), 9..11
 * barrier-free column march, 15 and 16 two steps per launch (levels n ->
 * n+2 in one z-march of 64 x 8 or 64 x 4 tiles: each workgroup recomputes
 * level n+1 on a one-point rim around its tile as the neighbouring block
 * would, and takes it from the ring's AT levels where the step-(n+1) delay
 * is positive; block widths multiples of 64 in x and of the tile rows in y).
 * Choosing 15 or 16 sets the steps per launch to 2 (a run's odd last step
 * and at_step use a one-step variant); choosing another sets it to 1, and
 * at_set_fuse(ctx, 2) selects 15 (or 16).  1D contexts: 0 automatic; 1, 2, 3 for 16, 8
 * and 4 points per thread in the fused launches (the tile width must be
 * divisible by it, AT_ERR_ARG otherwise); 4 for the whole periodic grid in
 * one workgroup of 256 threads (N <= 256 x 16, with N and the tile width
 * multiples of the 4, 8 or 16 points a thread holds, AT_ERR_ARG otherwise):
 * no rim is recomputed, the neighbour exchange wraps around the workgroup,
 * and one launch advances a whole at_run call (choosing it sets the steps
 * per launch to nsteps_max; at_set_fuse can lower it); every choice gives the
 * same bits. */
at_status at_set_variant(at_ctx *ctx, int32_t variant);

/* Current step n, steps per launch in use, ring levels R, kernel variant
 * (at_set_variant; chosen by at_autotune).  Any output may be NULL. */
at_status at_query(const at_ctx *ctx, int64_t *n, int32_t *fuse_steps, int32_t *ring_levels,
                   int32_t *variant);

/* Copy the delay array (int8[nsteps_max][F], after the clamp) to host memory.
 * Synchronous. */
at_status at_delays_copy(const at_ctx *ctx, int8_t *host_out);

/* Snapshot / restore of the full stepper state (the field u at the current
 * step, the ring and n).  at_snapshot_bytes gives the device buffer size.
 * Both are asynchronous on the context's stream.  at_restore of a buffer that
 * this context filled by at_snapshot (recognised by its address) takes the
 * step from the context; any other buffer is read once on the host to find
 * its step, which waits for the stream, and AT_ERR_ARG if it holds none. */
at_status at_snapshot_bytes(const at_ctx *ctx, uint64_t *bytes);
at_status at_snapshot(at_ctx *ctx, const double *u, void *dev_buf);
at_status at_restore(at_ctx *ctx, const void *dev_buf, double *u);

/* Reductions over a field of the context's size, written to device memory
 * (wave64 shuffles, compensated per-workgroup partials, fixed-order final
 * pass): out4[0] = max |u|, NaN as soon as one value is NaN; out4[1] = mean u;
 * out4[2] = sum |u|; out4[3] = the number of values that are not finite
 * (NaN or +-inf), as a double.  A run that has become unstable (the AT
 * extrapolation with large delays can amplify, section 2) shows up as
 * out4[3] > 0 instead of a finite maximum. */
at_status at_stats(at_ctx *ctx, const double *u, double *out4);

/* at_stats without a context, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops): the same
 * kernels and the same four outputs as at_stats, for n doubles at u
 * (1 <= n <= AT_NOALLOC_MAX_POINTS, AT_ERR_ARG otherwise), launched on
 * `stream` (a hipStream_t; NULL for the null stream) of the current device.
 * The per-workgroup partials live in a static device array of 1024 x 6
 * doubles (48 KiB) that each GPU the library runs on keeps until the process
 * ends; its address is looked up once per device on the first call there.
 * Nothing is allocated or freed.  Every call on one GPU shares that array,
 * so calls that can overlap on one GPU (other streams, other threads) race
 * and must be ordered by the caller.  Asynchronous; out4 is device memory. */
#define AT_NOALLOC_MAX_POINTS ((int64_t)1 << 40)
at_status at_stats_noalloc(const double *u, int64_t n, double *out4, void *stream);

/* Final-time misfit J = 0.5 * sum (u - target)^2 into *J_dev, and
 * lambda = u - target (= dJ/du) into lam (may be NULL). */
at_status at_loss(at_ctx *ctx, const double *u, const double *target, double *lam,
                  double *J_dev);

/* Discrete adjoint of the recorded run (record mode, 1D): given
 * lambda_T = dJ/du at the current step n_end (run from n = 0), writes
 * dJ/du0 into grad_u0 and dJ/dnu into *grad_nu_dev (dt held fixed).  Replays
 * the same delays; recomputes each checkpoint segment of ckpt_every steps in
 * reverse order.  The context stays at n_end. */
at_status at_adjoint(at_ctx *ctx, const double *lambda_T, double *grad_u0, double *grad_nu_dev);

/* ---------------------------------------------------------------------- */
/* Batched form: many independent 1D instances of uneven size advanced by */
/* the same launches.                                                      */
/* ---------------------------------------------------------------------- */
typedef struct at_batch at_batch;

/* cfgs[0..count-1] are 1D configurations (record = 0) that all share one
 * order, one adv_mode and one stream (the first one's), with tile widths that
 * are multiples of 16 (AT_ERR_SHAPE otherwise).  Each instance keeps its own
 * n, p, nu, dt, L, delays (generated or host) and ring.  Instance workspace
 * fields are ignored; the batch uses the single workspace given here, of at
 * least at_batch_workspace_bytes() bytes.  All instances share the step
 * counter, which starts at 0; a run may not pass the smallest nsteps_max. */
at_status at_batch_workspace_bytes(const at_config *cfgs, int32_t count, uint64_t *bytes);
at_status at_batch_init(const at_config *cfgs, int32_t count, void *workspace,
                        uint64_t workspace_bytes, at_batch **out);
void at_batch_free(at_batch *b);

/* Advance every instance by nsteps; u_dev[j] / scratch_dev[j] are host
 * arrays of device pointers for instance j; results are left in u_dev[j].
 * use_graph = 1 captures the launch sequence in a HIP graph and replays it. */
at_status at_batch_run(at_batch *b, double *const *u_dev, double *const *scratch_dev,
                       int64_t nsteps, int32_t use_graph);

/* Clear every instance's ring and set the shared step counter to 0
 * (asynchronous; the caller reloads the fields). */
at_status at_batch_reset(at_batch *b);

/* Shared step counter, steps per launch in use and its upper limit (for the
 * points per thread in use), and the batch's variant. */
at_status at_batch_query(const at_batch *b, int64_t *n, int32_t *fuse_steps, int32_t *max_fuse,
                         int32_t *variant);

/* Points per thread of the batched kernel: 0 (default) and 1: 16, 2: 8,
 * 3: 4.  Fewer points per thread make shorter regions (more workgroups, more
 * redundant rim work per point).  Steps per launch are lowered to the limit
 * of the new layout if needed.  Every choice gives the same bits. */
at_status at_batch_set_variant(at_batch *b, int32_t variant);

/* Choose the batch's points per thread and steps per launch by timing (same
 * contract as at_autotune, per batch); *chosen receives the steps per
 * launch, at_batch_query both.  Steps per launch are tried largest first, and
 * a smaller count replaces a larger one only when it is 2% faster. */
at_status at_batch_autotune(at_batch *b, double *const *u_dev, double *const *t1,
                            double *const *t2, int32_t trial_steps, int32_t *chosen);
at_status at_batch_set_fuse(at_batch *b, int32_t fuse_steps);
at_status at_set_fuse(at_ctx *ctx, int32_t fuse_steps);

/* Reverse steps per launch of at_adjoint.  0 (default): as many as the grid
 * allows (fused reverse launches need a tile width that is a multiple of 4,
 * else one step per launch); 1: one reverse step per launch; 2..64: at most
 * that many per launch (AT_ERR_ARG beyond this grid's limit).  Every setting
 * gives the same lambda bits; dJ/dnu is summed in a different grouping. */
at_status at_set_adjoint_fuse(at_ctx *ctx, int32_t steps);

/* Size of at_config as compiled into the library (bindings check their
 * copy of the layout against it). */
uint64_t at_config_bytes(void);

/* Thread-local message of the last failure in this thread ("" if none). */
const char *at_last_error(void);

/* AT_ABI_VERSION of the loaded library. */
int32_t at_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* AT_H */
