/*
 * at_oracle.c -- plain, slow CPU oracle for the asynchrony-tolerant (AT)
 * explicit Burgers stepper of Aditya, Gysi, Kwasniewski, Hoefler, Donzis and
 * Chen, "A scalable weakly-synchronous algorithm for solving partial
 * differential equations" (arXiv:1911.05769).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library. It shares no code,
 * header, table or helper with the GPU library, and the GPU library never
 * calls it.
 *
 * What it computes (paper passages in brackets):
 *   * Delays (section 2): the halo values of a subdomain face may lag the
 *     current level n by k levels, 0 <= k <= L.  Here k is prescribed per
 *     directed face and per step by a counter-based generator (SplitMix64,
 *     Steele, Lea & Flood, OOPSLA 2014) and clamped during start-up so that
 *     no level before 0 is ever read (the WS algorithm enforces synchrony
 *     while its circular buffers fill: Algorithm 2, section 5.2).
 *   * AT halo approximation (section 2, Eqs. (1)-(2); section 5.2 splits AT
 *     into a halo approximation and the unchanged stencil): the halo value is
 *     extrapolated in time from the m most recent available levels n-k,
 *     n-k-1, ... of the neighbour's edge.  For m = 2 the weights are (k+1, -k)
 *     exactly as printed in Eqs. (1)-(2).  For the 4th-order scheme, whose
 *     coefficients the paper defers to another article, this oracle reads AT
 *     as quadratic (m = 3) Newton backward extrapolation in time -- a reading,
 *     "parity unpinned" against the paper itself, pinned instead by the k = 0
 *     reduction, exactness on quadratic-in-time data and the truncation order.
 *   * Standard central differences at interior points, forward Euler in time
 *     (section 3.2), for viscous Burgers u_t + u u_x = nu u_xx in 1D and the
 *     3D vector form u_i,t + u_j d_j u_i = nu d_j d_j u_i (section 3.1,
 *     Eq. (4)), periodic domain, optionally with passive scalars
 *     phi_t + u_j d_j phi = alpha d_j d_j phi (the second line of Eq. (4)).
 *   * The paper's verification problem, linear advection-diffusion
 *     u_t + c u_x = nu u_xx (section 3.2), and the "standard scheme on
 *     delayed data" configuration (halo = stale level n-k, no extrapolation)
 *     that the paper uses as the negative control of Figure 2.
 *   * A discrete adjoint (reverse-mode derivative) of the 1D stepper, by
 *     brute force: every forward level is stored, every partial derivative is
 *     scattered in reverse order.
 *
 * Floating point: IEEE binary64, compile with -ffp-contract=off; the
 * arithmetic order of each formula is written out below and is part of the
 * specification.  Nothing here is blocked, fused or reordered.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_ERR_ARG -1
#define OR_ERR_SHAPE -2
#define OR_ERR_DELAY -3
#define OR_ERR_NOMEM -5
#define OR_MAX_SCALARS 4

/* ------------------------------------------------------------------------ */
/* Delays                                                                    */
/* ------------------------------------------------------------------------ */

/* SplitMix64 output function applied to the state seed + gamma * c, with the
 * published golden-ratio increment gamma and the published finaliser.  c is
 * the 1-based counter of the (step, face) pair. */
static uint64_t or_splitmix(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + 0x9E3779B97F4A7C15ULL * c;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t or_splitmix_sequence(uint64_t seed, int64_t count, uint64_t *out)
{
    for (int64_t i = 0; i < count; ++i) out[i] = or_splitmix(seed, (uint64_t)(i + 1));
    return (uint64_t)count;
}

/* Raw delay for (step n, face f) before the start-up clamp.
 * dist 0: k uniform on {0..L};  dist 1: k = 0 with probability 1/2, else
 * uniform on {1..L}.  Both map 32 random bits to a range by a multiply-shift. */
static int or_raw_delay(uint64_t z, int L, int dist)
{
    uint64_t hi = z >> 32, lo = z & 0xFFFFFFFFULL;
    if (dist == 0) return (int)((hi * (uint64_t)(L + 1)) >> 32);
    if (L == 0 || lo < 0x80000000ULL) return 0;
    return 1 + (int)((hi * (uint64_t)L) >> 32);
}

/* Largest delay allowed at step n: at most L, and no level below 0 may be
 * touched by an m-level extrapolation (levels n-k .. n-k-m+1). */
static int or_kmax_at(int64_t n, int L, int m)
{
    int64_t lim = n - m + 1;
    if (lim < 0) lim = 0;
    return (int)(lim < L ? lim : L);
}

int or_delays(int64_t nsteps, int64_t nfaces, int L, int m, int dist, uint64_t seed,
              int8_t *k)
{
    if (nsteps < 0 || nfaces <= 0 || L < 0 || L > 15 || m < 1 || (dist != 0 && dist != 1))
        return OR_ERR_ARG;
    for (int64_t n = 0; n < nsteps; ++n) {
        int km = or_kmax_at(n, L, m);
        for (int64_t f = 0; f < nfaces; ++f) {
            uint64_t z = or_splitmix(seed, (uint64_t)(1 + n * nfaces + f));
            int kk = or_raw_delay(z, L, dist);
            k[n * nfaces + f] = (int8_t)(kk < km ? kk : km);
        }
    }
    return OR_OK;
}

int or_check_delays(int64_t nsteps, int64_t nfaces, int L, int m, const int8_t *k)
{
    for (int64_t n = 0; n < nsteps; ++n) {
        int km = or_kmax_at(n, L, m);
        for (int64_t f = 0; f < nfaces; ++f) {
            int kk = k[n * nfaces + f];
            if (kk < 0 || kk > km) return OR_ERR_DELAY;
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Halo approximation (section 2, Eqs. (1)-(2); section 5.2)                 */
/* ------------------------------------------------------------------------ */

/* v[j] = value of the source point at level n-kk-j, j = 0..m-1.
 * halo_mode 0: AT extrapolation to level n;  1: stale value v[0].
 *   m = 2:  H = v0 + kk*(v0 - v1)            == (kk+1) v0 - kk v1
 *   m = 3:  H = (v0 + kk*d1) + w2*(d1 - (v1 - v2)),  d1 = v0 - v1,
 *           w2 = kk(kk+1)/2  (Newton backward form through three levels). */
double or_halo(int kk, int m, int halo_mode, const double *v)
{
    if (kk == 0 || halo_mode == 1) return v[0];
    double dk = (double)kk;
    double d1 = v[0] - v[1];
    if (m == 2) return v[0] + dk * d1;
    double w2 = 0.5 * dk * (dk + 1.0);
    return (v[0] + dk * d1) + w2 * (d1 - (v[1] - v[2]));
}

/* dH/dv_j for the same three cases (used by the adjoint). */
static void or_halo_weights(int kk, int m, int halo_mode, double *w)
{
    w[0] = 1.0; w[1] = 0.0; w[2] = 0.0;
    if (kk == 0 || halo_mode == 1) return;
    double dk = (double)kk;
    if (m == 2) { w[0] = 1.0 + dk; w[1] = -dk; return; }
    double w2 = 0.5 * dk * (dk + 1.0);
    w[0] = (1.0 + dk) + w2;
    w[1] = -dk - 2.0 * w2;
    w[2] = w2;
}

/* ------------------------------------------------------------------------ */
/* Central differences (section 3.2)                                         */
/* ------------------------------------------------------------------------ */

typedef struct { double c1, c2; } or_coef;

/* order 2:  D1 = (r1 - l1) c1,  c1 = 1/(2 dx);  D2 = ((r1 - 2u) + l1) c2,  c2 = 1/dx^2
 * order 4:  D1 = (8(r1 - l1) - (r2 - l2)) c1,  c1 = 1/(12 dx);
 *           D2 = ((16(r1 + l1) - 30u) - (r2 + l2)) c2,  c2 = 1/(12 dx^2) */
static or_coef or_coefs(int order, double dx)
{
    or_coef c;
    if (order == 2) { c.c1 = 1.0 / (2.0 * dx); c.c2 = 1.0 / (dx * dx); }
    else            { c.c1 = 1.0 / (12.0 * dx); c.c2 = 1.0 / (12.0 * (dx * dx)); }
    return c;
}

/* nb[0..h-1] = left neighbours l_h..l_1 (nb[h-1] = l1), nb[h..2h-1] = r1..r_h */
static void or_derivs(int order, or_coef c, double u, const double *nb, double *D1, double *D2)
{
    if (order == 2) {
        double l1 = nb[0], r1 = nb[1];
        *D1 = (r1 - l1) * c.c1;
        *D2 = ((r1 - 2.0 * u) + l1) * c.c2;
    } else {
        double l2 = nb[0], l1 = nb[1], r1 = nb[2], r2 = nb[3];
        *D1 = (8.0 * (r1 - l1) - (r2 - l2)) * c.c1;
        *D2 = ((16.0 * (r1 + l1) - 30.0 * u) - (r2 + l2)) * c.c2;
    }
}

/* dD1/dnb, dD2/dnb (same slot order as nb), dD2/du */
static void or_deriv_partials(int order, or_coef c, double *g1, double *g2, double *g2u)
{
    if (order == 2) {
        g1[0] = -c.c1; g1[1] = c.c1;
        g2[0] = c.c2;  g2[1] = c.c2;
        *g2u = -2.0 * c.c2;
    } else {
        g1[0] = c.c1;  g1[1] = -8.0 * c.c1; g1[2] = 8.0 * c.c1; g1[3] = -c.c1;
        g2[0] = -c.c2; g2[1] = 16.0 * c.c2; g2[2] = 16.0 * c.c2; g2[3] = -c.c2;
        *g2u = -30.0 * c.c2;
    }
}

static int64_t or_mod(int64_t a, int64_t b) { int64_t r = a % b; return r < 0 ? r + b : r; }

/* ------------------------------------------------------------------------ */
/* 1D stepper                                                                */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t N, P, W;
    int order, h, m, L, halo_mode, adv_mode;
    double nu, dt, adv_speed;
    or_coef c;
} or_p1;

static int or_setup1d(or_p1 *p, int64_t N, int64_t P, int order, int L, int halo_mode,
                      int adv_mode, double nu, double dt, double length, double adv_speed)
{
    if (N <= 0 || P <= 0 || (order != 2 && order != 4) || L < 0 || L > 15) return OR_ERR_ARG;
    if (halo_mode < 0 || halo_mode > 1 || adv_mode < 0 || adv_mode > 1) return OR_ERR_ARG;
    if (!(nu >= 0.0) || !(dt > 0.0) || !(length > 0.0)) return OR_ERR_ARG;
    if (N % P != 0) return OR_ERR_SHAPE;
    p->N = N; p->P = P; p->W = N / P; p->order = order; p->h = order / 2; p->m = p->h + 1;
    if (p->W < 2 * p->h) return OR_ERR_SHAPE;
    p->L = L; p->halo_mode = halo_mode; p->adv_mode = adv_mode;
    p->nu = nu; p->dt = dt; p->adv_speed = adv_speed;
    p->c = or_coefs(order, length / (double)N);
    return OR_OK;
}

/* Value seen by point i (tile t = i / W) at stencil offset d at step n.
 * hist(lev) returns the full-grid array of level lev. */
#define OR_HIST(lev) (hist[(lev) % nh])

static double or_nb1d(const or_p1 *p, double *const *hist, int64_t nh, const int8_t *krow,
                      int64_t n, int64_t i, int d, int *face, int64_t *src)
{
    int64_t t = i / p->W, lo = t * p->W, hi = lo + p->W;
    int64_t j = i + d;
    const double *un = OR_HIST(n);
    *face = -1; *src = -1;
    if (j >= lo && j < hi) return un[j];
    int side = (j < lo) ? 0 : 1;
    int64_t s = or_mod(j, p->N);        /* source point, in the neighbouring tile */
    int f = (int)(2 * t + side);
    int kk = krow[f];
    double v[3] = {0.0, 0.0, 0.0};
    int need = (kk == 0 || p->halo_mode == 1) ? 1 : p->m;
    for (int q = 0; q < need; ++q) v[q] = OR_HIST(n - kk - q)[s];
    *face = f; *src = s;
    return or_halo(kk, p->m, p->halo_mode, v);
}

static void or_step1d(const or_p1 *p, double *const *hist, int64_t nh, const int8_t *krow,
                      int64_t n, double *out)
{
    const double *un = OR_HIST(n);
    #pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < p->P; ++t) {
        for (int64_t i = t * p->W; i < (t + 1) * p->W; ++i) {
            double nb[4];
            int face; int64_t src;
            for (int q = 0; q < p->h; ++q) {
                nb[q] = or_nb1d(p, hist, nh, krow, n, i, -(p->h - q), &face, &src);
                nb[p->h + q] = or_nb1d(p, hist, nh, krow, n, i, q + 1, &face, &src);
            }
            double u = un[i], D1, D2;
            or_derivs(p->order, p->c, u, nb, &D1, &D2);
            double a = p->adv_mode ? p->adv_speed : u;
            double F = p->nu * D2 - a * D1;
            out[i] = u + p->dt * F;
        }
    }
}

int or_run1d(int64_t N, int64_t P, int order, int L, int halo_mode, int adv_mode,
             double nu, double dt, double length, double adv_speed,
             const int8_t *k, int64_t nsteps, const double *u0, double *uT)
{
    or_p1 p;
    int st = or_setup1d(&p, N, P, order, L, halo_mode, adv_mode, nu, dt, length, adv_speed);
    if (st) return st;
    if (nsteps < 0) return OR_ERR_ARG;
    if (or_check_delays(nsteps, 2 * P, L, p.m, k)) return OR_ERR_DELAY;
    /* keep the last L+m levels plus the one being written, as full grids */
    int64_t nh = L + p.m + 1;
    double **hist = (double **)calloc((size_t)nh, sizeof(double *));
    if (!hist) return OR_ERR_NOMEM;
    for (int64_t q = 0; q < nh; ++q) {
        hist[q] = (double *)malloc((size_t)N * sizeof(double));
        if (!hist[q]) { for (int64_t r = 0; r < q; ++r) free(hist[r]); free(hist); return OR_ERR_NOMEM; }
    }
    memcpy(hist[0], u0, (size_t)N * sizeof(double));
    for (int64_t n = 0; n < nsteps; ++n)
        or_step1d(&p, hist, nh, k + n * 2 * P, n, hist[(n + 1) % nh]);
    memcpy(uT, hist[nsteps % nh], (size_t)N * sizeof(double));
    for (int64_t q = 0; q < nh; ++q) free(hist[q]);
    free(hist);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* 1D discrete adjoint (reverse mode, brute force)                           */
/* ------------------------------------------------------------------------ */

static void neumaier_add(double *s, double *comp, double x)
{
    double t = *s + x;
    if (fabs(*s) >= fabs(x)) *comp += (*s - t) + x;
    else                     *comp += (x - t) + *s;
    *s = t;
}

/* Given lamT = dJ/du(T) for a run of nsteps from u0, returns lam0 = dJ/du0 and
 * gnu = dJ/dnu, with dt held fixed.  All nsteps+1 forward levels are stored;
 * the adjoint of every level is accumulated in a full array, in reverse step
 * order, point by point in increasing index, neighbour slots in stencil order. */
int or_adjoint1d(int64_t N, int64_t P, int order, int L, int halo_mode, int adv_mode,
                 double nu, double dt, double length, double adv_speed,
                 const int8_t *k, int64_t nsteps, const double *u0, const double *lamT,
                 double *lam0, double *gnu)
{
    or_p1 p;
    int st = or_setup1d(&p, N, P, order, L, halo_mode, adv_mode, nu, dt, length, adv_speed);
    if (st) return st;
    if (nsteps < 0) return OR_ERR_ARG;
    if (or_check_delays(nsteps, 2 * P, L, p.m, k)) return OR_ERR_DELAY;
    int64_t nl = nsteps + 1;
    double **U = (double **)calloc((size_t)nl, sizeof(double *));
    double **A = (double **)calloc((size_t)nl, sizeof(double *));
    if (!U || !A) { free(U); free(A); return OR_ERR_NOMEM; }
    int ok = 1;
    for (int64_t q = 0; q < nl && ok; ++q) {
        U[q] = (double *)malloc((size_t)N * sizeof(double));
        A[q] = (double *)calloc((size_t)N, sizeof(double));
        if (!U[q] || !A[q]) ok = 0;
    }
    if (!ok) {
        for (int64_t q = 0; q < nl; ++q) { free(U[q]); free(A[q]); }
        free(U); free(A); return OR_ERR_NOMEM;
    }
    memcpy(U[0], u0, (size_t)N * sizeof(double));
    /* forward: U is a full history, so hist = U with nh = nl */
    for (int64_t n = 0; n < nsteps; ++n)
        or_step1d(&p, U, nl, k + n * 2 * P, n, U[n + 1]);
    memcpy(A[nsteps], lamT, (size_t)N * sizeof(double));
    double gs = 0.0, gc = 0.0;
    double g1[4], g2[4], g2u;
    or_deriv_partials(order, p.c, g1, g2, &g2u);
    int h = p.h;
    for (int64_t n = nsteps - 1; n >= 0; --n) {
        const int8_t *krow = k + n * 2 * P;
        const double *un = U[n];
        for (int64_t i = 0; i < N; ++i) {
            double lam = A[n + 1][i];
            double nb[4]; int face[4]; int64_t src[4];
            for (int q = 0; q < h; ++q) {
                nb[q] = or_nb1d(&p, U, nl, krow, n, i, -(h - q), &face[q], &src[q]);
                nb[h + q] = or_nb1d(&p, U, nl, krow, n, i, q + 1, &face[h + q], &src[h + q]);
            }
            double u = un[i], D1, D2;
            or_derivs(order, p.c, u, nb, &D1, &D2);
            double a = adv_mode ? adv_speed : u;
            /* u' = u + dt*(nu*D2 - a*D1) */
            double du = 1.0 + dt * (nu * g2u - (adv_mode ? 0.0 : D1));
            A[n][i] += lam * du;
            for (int s = 0; s < 2 * h; ++s) {
                double g = lam * (dt * (nu * g2[s] - a * g1[s]));
                int d = (s < h) ? -(h - s) : (s - h + 1);
                if (face[s] < 0) { A[n][i + d] += g; continue; }
                int kk = krow[face[s]];
                double w[3];
                or_halo_weights(kk, p.m, halo_mode, w);
                int need = (kk == 0 || halo_mode == 1) ? 1 : p.m;
                for (int q = 0; q < need; ++q) A[n - kk - q][src[s]] += g * w[q];
            }
            neumaier_add(&gs, &gc, lam * (dt * D2));
        }
    }
    memcpy(lam0, A[0], (size_t)N * sizeof(double));
    *gnu = gs + gc;
    for (int64_t q = 0; q < nl; ++q) { free(U[q]); free(A[q]); }
    free(U); free(A);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* 3D vector stepper (order 2, 7-point stencil per axis), with passive        */
/* scalars phi_k: phi_t + u_j d_j phi = alpha_k d_j d_j phi (section 3.1, the  */
/* second line of Eq. (4)); a scalar is one more component that the velocity   */
/* advects, with its own diffusivity                                           */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t n[3], P[3], W[3], npt;
    int L, m, halo_mode;
    int nc;                   /* components: 3 velocity + passive scalars */
    double nu, dt;
    double kappa[3 + OR_MAX_SCALARS];   /* diffusivity per component (nu, then alpha_k) */
    or_coef c[3];
} or_p3;

/* u layout: [comp][z][y][x], x fastest.  Block b = (bz*Py + by)*Px + bx,
 * face f = 6b + 2a + s with axis a in {x,y,z}, side s (0 low, 1 high). */
static double or_nb3d(const or_p3 *p, double *const *hist, int64_t nh, const int8_t *krow,
                      int64_t n, int comp, const int64_t *x, int a, int d)
{
    int64_t blk[3], y[3];
    for (int e = 0; e < 3; ++e) { blk[e] = x[e] / p->W[e]; y[e] = x[e]; }
    int64_t j = x[a] + d, lo = blk[a] * p->W[a], hi = lo + p->W[a];
    y[a] = or_mod(j, p->n[a]);
    int64_t off = (int64_t)comp * p->npt + (y[2] * p->n[1] + y[1]) * p->n[0] + y[0];
    if (j >= lo && j < hi) return OR_HIST(n)[off];
    int side = (j < lo) ? 0 : 1;
    int64_t b = (blk[2] * p->P[1] + blk[1]) * p->P[0] + blk[0];
    int kk = krow[6 * b + 2 * a + side];
    double v[3] = {0.0, 0.0, 0.0};
    int need = (kk == 0 || p->halo_mode == 1) ? 1 : p->m;
    for (int q = 0; q < need; ++q) v[q] = OR_HIST(n - kk - q)[off];
    return or_halo(kk, p->m, p->halo_mode, v);
}

static void or_step3d(const or_p3 *p, double *const *hist, int64_t nh, const int8_t *krow,
                      int64_t n, double *out)
{
    const double *un = OR_HIST(n);
    #pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < p->n[2]; ++z) {
        for (int64_t yy = 0; yy < p->n[1]; ++yy) {
            for (int64_t xx = 0; xx < p->n[0]; ++xx) {
                int64_t x[3] = {xx, yy, z};
                int64_t at = (z * p->n[1] + yy) * p->n[0] + xx;
                double vel[3] = {un[at], un[p->npt + at], un[2 * p->npt + at]};
                for (int comp = 0; comp < p->nc; ++comp) {
                    double u = un[(int64_t)comp * p->npt + at];
                    double D1[3], D2[3];
                    for (int a = 0; a < 3; ++a) {
                        double l1 = or_nb3d(p, hist, nh, krow, n, comp, x, a, -1);
                        double r1 = or_nb3d(p, hist, nh, krow, n, comp, x, a, +1);
                        D1[a] = (r1 - l1) * p->c[a].c1;
                        D2[a] = ((r1 - 2.0 * u) + l1) * p->c[a].c2;
                    }
                    double lap = (D2[0] + D2[1]) + D2[2];
                    double adv = (vel[0] * D1[0] + vel[1] * D1[1]) + vel[2] * D1[2];
                    double F = p->kappa[comp] * lap - adv;
                    out[(int64_t)comp * p->npt + at] = u + p->dt * F;
                }
            }
        }
    }
}

int or_run3ds(const int64_t *nxyz, const int64_t *pxyz, int nscalars, const double *alpha,
              int L, int halo_mode, double nu, double dt, double length, const int8_t *k,
              int64_t nsteps, const double *u0, double *uT)
{
    or_p3 p;
    if (L < 0 || L > 15 || halo_mode < 0 || halo_mode > 1) return OR_ERR_ARG;
    if (nscalars < 0 || nscalars > OR_MAX_SCALARS || (nscalars > 0 && !alpha)) return OR_ERR_ARG;
    p.nc = 3 + nscalars;
    for (int c = 0; c < 3; ++c) p.kappa[c] = nu;
    for (int c = 0; c < nscalars; ++c) {
        if (!(alpha[c] >= 0.0)) return OR_ERR_ARG;
        p.kappa[3 + c] = alpha[c];
    }
    if (!(nu >= 0.0) || !(dt > 0.0) || !(length > 0.0) || nsteps < 0) return OR_ERR_ARG;
    int64_t nb = 1;
    for (int a = 0; a < 3; ++a) {
        if (nxyz[a] <= 0 || pxyz[a] <= 0) return OR_ERR_ARG;
        if (nxyz[a] % pxyz[a] != 0) return OR_ERR_SHAPE;
        p.n[a] = nxyz[a]; p.P[a] = pxyz[a]; p.W[a] = nxyz[a] / pxyz[a];
        if (p.W[a] < 2) return OR_ERR_SHAPE;
        p.c[a] = or_coefs(2, length / (double)nxyz[a]);
        nb *= pxyz[a];
    }
    p.npt = p.n[0] * p.n[1] * p.n[2];
    p.L = L; p.m = 2; p.halo_mode = halo_mode; p.nu = nu; p.dt = dt;
    if (or_check_delays(nsteps, 6 * nb, L, p.m, k)) return OR_ERR_DELAY;
    int64_t nh = L + p.m + 1;
    double **hist = (double **)calloc((size_t)nh, sizeof(double *));
    if (!hist) return OR_ERR_NOMEM;
    for (int64_t q = 0; q < nh; ++q) {
        hist[q] = (double *)malloc((size_t)(p.nc * p.npt) * sizeof(double));
        if (!hist[q]) { for (int64_t r = 0; r < q; ++r) free(hist[r]); free(hist); return OR_ERR_NOMEM; }
    }
    memcpy(hist[0], u0, (size_t)(p.nc * p.npt) * sizeof(double));
    for (int64_t n = 0; n < nsteps; ++n)
        or_step3d(&p, hist, nh, k + n * 6 * nb, n, hist[(n + 1) % nh]);
    memcpy(uT, hist[nsteps % nh], (size_t)(p.nc * p.npt) * sizeof(double));
    for (int64_t q = 0; q < nh; ++q) free(hist[q]);
    free(hist);
    return OR_OK;
}

int or_run3d(const int64_t *nxyz, const int64_t *pxyz, int L, int halo_mode,
             double nu, double dt, double length, const int8_t *k, int64_t nsteps,
             const double *u0, double *uT)
{
    return or_run3ds(nxyz, pxyz, 0, NULL, L, halo_mode, nu, dt, length, k, nsteps, u0, uT);
}

/* ------------------------------------------------------------------------ */
/* Reductions (serial order, Neumaier-compensated sums)                      */
/* ------------------------------------------------------------------------ */

/* out[0] = max|u|, out[1] = mean(u), out[2] = sum |u|, out[3] = the number of
 * values that are not finite.  The maximum is NaN as soon as one value is
 * NaN (a NaN compares false with everything, so a plain running maximum would
 * skip it and report a finite maximum for a field that has blown up). */
void or_stats(int64_t n, const double *u, double *out)
{
    double mx = 0.0, s = 0.0, c = 0.0, a = 0.0, ac = 0.0;
    int64_t bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        double v = fabs(u[i]);
        if (isnan(v)) mx = v;
        else if (v > mx) mx = v;
        if (!isfinite(u[i])) ++bad;
        neumaier_add(&s, &c, u[i]);
        neumaier_add(&a, &ac, v);
    }
    out[0] = mx;
    out[1] = (s + c) / (double)n;
    out[2] = a + ac;
    out[3] = (double)bad;
}

/* J = 0.5 * sum (u - target)^2 ; lam = u - target (= dJ/du) */
double or_loss(int64_t n, const double *u, const double *target, double *lam)
{
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double d = u[i] - target[i];
        if (lam) lam[i] = d;
        neumaier_add(&s, &c, 0.5 * (d * d));
    }
    return s + c;
}

/* Threads of the OpenMP loops (timing of the baseline only; the results do
 * not depend on it: no loop reduces across tiles). */
void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
