// 3D vector stepper of libat.so for gfx950.
//
// Method: u_i,t + u_j d_j u_i = nu d_j d_j u_i (paper section 3.1, Eq. (4)),
// i, j over x, y, z, plus passive scalars phi_s,t + u_j d_j phi_s =
// alpha_s d_j d_j phi_s (the second line of Eq. (4)): NC = 3 + nscalars
// components, component c diffused with kappa_c (nu for the velocity, alpha_s
// for the scalars) and advected by the velocity, on a periodic grid split
// into Px x Py x Pz blocks,
// second-order central differences and forward Euler (section 3.2).  A point
// on a block face reads its neighbour across the face through an AT halo:
// the neighbour block's face value extrapolated in time from levels n-k and
// n-k-1 (section 2, Eqs. (1)-(2): H = v0 + k*(v0 - v1)), with the delay k
// prescribed per directed face and per step.  With k = 0 the halo is the
// neighbour's current value.  Fixed evaluation order (contraction off):
//   D1_a = (r - l)*c1_a,  D2_a = ((r - 2u) + l)*c2_a       for a = x, y, z
//   lap = (D2_x + D2_y) + D2_z,  adv = (u_x*D1_x + u_y*D1_y) + u_z*D1_z
//   u' = u + dt*(kappa_c*lap - adv)
//
// Layout: fields double[NC][nz][ny][nx] (x fastest).  Ring level: per block,
// faces x-low, x-high, y-low, y-high, z-low, z-high, each [NC][plane] with the
// plane indexed (z, y) for x-faces, (z, x) for y-faces, (y, x) for z-faces.
//
// Work decomposition (2.5D): a workgroup of 64 x 8 threads owns a 64 x 8 x-y
// tile (one point per thread) and marches through ZC planes in z.  Each
// thread keeps the z-1, z, z+1 values (NC components) in registers and has
// planes z+2 and z+3 in flight; the current plane with one-point rims sits in a
// double-buffered LDS tile for the x and y neighbours (one barrier per
// plane).  Block faces inside the tile are handled per point (any block
// width >= 2).
#include "../../include/at.h"
#include "at_internal.h"
#include "at_ws.h"

at_status at_fail(at_status st, const char *msg);
struct at_ctx;
const at_config *at_ctx_cfg(const at_ctx *c);
double *at_ctx_ring(const at_ctx *c);
const int8_t *at_ctx_delays(const at_ctx *c);
int at_ctx_R(const at_ctx *c);
hipStream_t at_ctx_stream(const at_ctx *c);
void at_ctx_coefs(const at_ctx *c, double *c1, double *c2);
int at_ctx_variant(const at_ctx *c);

namespace atk {

struct Step3D {
    const double *uin;
    double *uout;
    double *ring;
    const int8_t *delays;
    int64_t nx, ny, nz, npt;
    int32_t Px, Py, Pz, Wx, Wy, Wz;
    int64_t F;                // faces
    int64_t level;            // doubles per ring level
    int64_t bstride;          // doubles per block in a ring level
    int64_t foff[6];          // face offsets within a block
    int64_t psz[3];           // plane sizes of x-, y-, z-faces
    int64_t n;
    int32_t R, stale, publish, ZC;
    int32_t slot0;            // n mod R
    int32_t nc;               // components: 3 + passive scalars
    double dt, c1[3], c2[3];
    double kappa[3 + AT_MAX_SCALARS];   // diffusivity per component
};

namespace {

constexpr int TX = 64;        // tile width in x (one wave64 per row)
constexpr int kZB = 64;       // z-blocks one chunk of the aligned kernel may span

// waves per SIMD a variant asks for; from 6 components on scaled down for
// the larger register footprint (measured at 512^3: the unscaled bound is
// faster up to 5 components, the scaled one above)
constexpr int waves_for(int minw, int nc) { return nc <= 5 ? minw : (minw * 3 / nc > 0 ? minw * 3 / nc : 1); }

__device__ __forceinline__ int wrap32(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// TY rows per tile (= waves per workgroup, one row per thread); PF planes
// prefetched ahead (1 or 2); MINW waves per SIMD the register budget allows.
template <int TY, int PF, int MINW, int NC>
__global__ __launch_bounds__(TX * TY, waves_for(MINW, NC)) void k_step3d(Step3D A)
{
    __shared__ double pl[2][NC][TY + 2][TX + 2];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int nx = (int)A.nx, ny = (int)A.ny, nz = (int)A.nz;
    const int X0 = blockIdx.x * TX, Y0 = blockIdx.y * TY;
    const int Z0 = blockIdx.z * A.ZC;
    const int Z1 = (Z0 + A.ZC < nz) ? Z0 + A.ZC : nz;
    const int wx = (nx - X0 < TX) ? nx - X0 : TX;
    const int hy = (ny - Y0 < TY) ? ny - Y0 : TY;
    const int x = X0 + tx, y = Y0 + ty;
    const bool act = tx < wx && ty < hy;
    const int plane = nx * ny;
    const int bx = x / A.Wx, lx = x - bx * A.Wx;
    const int by = y / A.Wy, ly = y - by * A.Wy;
    const double *U0 = A.uin;
    const int64_t npt = A.npt;
    // rim loads of this thread (lanes 0/1: x rims of its row; waves 0/1: y rims)
    const bool xrim = tx < 2 && ty < hy;
    const int xs = tx == 0 ? wrap32(X0 - 1, nx) : wrap32(X0 + wx, nx);
    const int xcol = tx == 0 ? 0 : wx + 1;
    const bool yrim = ty < 2 && tx < wx;
    const int ys = ty == 0 ? wrap32(Y0 - 1, ny) : wrap32(Y0 + hy, ny);
    const int yrow = ty == 0 ? 0 : hy + 1;
    const int col = y * nx + x;

    auto ld3 = [&](int off, double *v, bool on) {
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = on ? U0[c * npt + off] : 0.0;
    };
    // register pipeline: planes z-1, z, z+1 in use, z+2 (and z+3 when PF = 2)
    // in flight; rims of plane z+1 (and z+2) in flight
    double zm[NC], zc[NC], zp[NC], zq[NC], zr[NC], rx[NC], ry[NC], rx2[NC], ry2[NC];
    ld3(wrap32(Z0 - 1, nz) * plane + col, zm, act);
    ld3(Z0 * plane + col, zc, act);
    ld3(wrap32(Z0 + 1, nz) * plane + col, zp, act);
    if (PF == 2) ld3(wrap32(Z0 + 2, nz) * plane + col, zq, act && Z0 + 1 < Z1);
    ld3(Z0 * plane + y * nx + xs, rx, xrim);
    ld3(Z0 * plane + ys * nx + x, ry, yrim);
    // plane Z0 into buffer 0
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if (act) pl[0][c][ty + 1][tx + 1] = zc[c];
        if (xrim) pl[0][c][ty + 1][xcol] = rx[c];
        if (yrim) pl[0][c][yrow][tx + 1] = ry[c];
    }
    {   // rims of plane Z0 + 1 (and Z0 + 2)
        const int zo = wrap32(Z0 + 1, nz) * plane;
        ld3(zo + y * nx + xs, rx, xrim && Z0 + 1 < Z1);
        ld3(zo + ys * nx + x, ry, yrim && Z0 + 1 < Z1);
        if (PF == 2) {
            const int zo2 = wrap32(Z0 + 2, nz) * plane;
            ld3(zo2 + y * nx + xs, rx2, xrim && Z0 + 2 < Z1);
            ld3(zo2 + ys * nx + x, ry2, yrim && Z0 + 2 < Z1);
        }
    }
    const int8_t *krow = A.delays + A.n * A.F;
    const int64_t slot = A.slot0 + 1 == A.R ? 0 : A.slot0 + 1;   // level n+1 is published

    int bz = Z0 / A.Wz, lz = Z0 - bz * A.Wz;
    int kbz = -1, kc[6] = {0, 0, 0, 0, 0, 0};
    for (int z = Z0; z < Z1; ++z, ++lz) {
        if (lz == A.Wz) { lz = 0; ++bz; }
        const int buf = (z - Z0) & 1;
        const bool more = z + 1 < Z1;
        if (PF == 2) ld3(wrap32(z + 3, nz) * plane + col, zr, act && z + 2 < Z1);
        else ld3(wrap32(z + 2, nz) * plane + col, zq, act && more);
        __syncthreads();
        if (act) {
            const int64_t b = ((int64_t)bz * A.Py + by) * A.Px + bx;
            if (bz != kbz) {          // face delays of this block: reloaded only at block changes
                kbz = bz;
                kc[0] = lx == 0 ? krow[6 * b + 0] : 0;
                kc[1] = lx == A.Wx - 1 ? krow[6 * b + 1] : 0;
                kc[2] = ly == 0 ? krow[6 * b + 2] : 0;
                kc[3] = ly == A.Wy - 1 ? krow[6 * b + 3] : 0;
                kc[4] = krow[6 * b + 4];
                kc[5] = krow[6 * b + 5];
            }
            const int kxl = kc[0], kxh = kc[1], kyl = kc[2], kyh = kc[3];
            const int kzl = lz == 0 ? kc[4] : 0;
            const int kzh = lz == A.Wz - 1 ? kc[5] : 0;
            const int px = lz * A.Wy + ly, py = lz * A.Wx + lx, pz = ly * A.Wx + lx;
            // neighbours: x/y from the LDS tile, z from registers
            double nb[6][NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                nb[0][c] = pl[buf][c][ty + 1][tx];
                nb[1][c] = pl[buf][c][ty + 1][tx + 2];
                nb[2][c] = pl[buf][c][ty][tx + 1];
                nb[3][c] = pl[buf][c][ty + 2][tx + 1];
                nb[4][c] = zm[c];
                nb[5][c] = zp[c];
            }
            // AT halo values across the block faces this point touches
            const int kf[6] = {kxl, kxh, kyl, kyh, kzl, kzh};
#pragma unroll
            for (int f = 0; f < 6; ++f) {
                const int kk = kf[f];
                if (kk > 0) {
                    const int a = f >> 1, sd = f & 1;
                    int n0 = bx, n1 = by, n2 = bz;
                    if (a == 0) n0 = wrap32(bx + (sd ? 1 : -1), A.Px);
                    else if (a == 1) n1 = wrap32(by + (sd ? 1 : -1), A.Py);
                    else n2 = wrap32(bz + (sd ? 1 : -1), A.Pz);
                    const int pos = a == 0 ? px : (a == 1 ? py : pz);
                    const int64_t off = (((int64_t)n2 * A.Py + n1) * A.Px + n0) * A.bstride +
                                        A.foff[2 * a + (1 - sd)] + pos;
                    int s0 = A.slot0 - kk, s1 = A.slot0 - kk - 1;     // levels n-k, n-k-1
                    if (s0 < 0) s0 += A.R;
                    if (s1 < 0) s1 += A.R;
                    const double *r0 = A.ring + s0 * A.level + off;
                    const double *r1 = A.ring + s1 * A.level + off;
                    const double dk = (double)kk;
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        const double v0 = r0[c * A.psz[a]];
                        nb[f][c] = A.stale ? v0 : v0 + dk * (v0 - r1[c * A.psz[a]]);
                    }
                }
            }
            const double ux = zc[0], uy = zc[1], uz = zc[2];
            double *out = A.uout + (int64_t)z * plane + col;
            double ov[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double u = zc[c];
                const double xl = nb[0][c], xr = nb[1][c], yl = nb[2][c], yh = nb[3][c];
                const double zl = nb[4][c], zh = nb[5][c];
                const double D1x = (xr - xl) * A.c1[0], D2x = ((xr - 2.0 * u) + xl) * A.c2[0];
                const double D1y = (yh - yl) * A.c1[1], D2y = ((yh - 2.0 * u) + yl) * A.c2[1];
                const double D1z = (zh - zl) * A.c1[2], D2z = ((zh - 2.0 * u) + zl) * A.c2[2];
                const double lap = (D2x + D2y) + D2z;
                const double adv = (ux * D1x + uy * D1y) + uz * D1z;
                ov[c] = u + A.dt * (A.kappa[c] * lap - adv);
                out[c * A.npt] = ov[c];
            }
            // publish the level-(n+1) values of points on block faces
            const bool onface = lx == 0 || lx == A.Wx - 1 || ly == 0 || ly == A.Wy - 1 ||
                                lz == 0 || lz == A.Wz - 1;
            if (A.publish && onface) {
                double *base = A.ring + slot * A.level + b * A.bstride;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const double u = ov[c];
                    if (lx == 0) base[A.foff[0] + c * A.psz[0] + px] = u;
                    if (lx == A.Wx - 1) base[A.foff[1] + c * A.psz[0] + px] = u;
                    if (ly == 0) base[A.foff[2] + c * A.psz[1] + py] = u;
                    if (ly == A.Wy - 1) base[A.foff[3] + c * A.psz[1] + py] = u;
                    if (lz == 0) base[A.foff[4] + c * A.psz[2] + pz] = u;
                    if (lz == A.Wz - 1) base[A.foff[5] + c * A.psz[2] + pz] = u;
                }
            }
        }
        if (more) {
            // plane z+1 into the other buffer (its readers finished before the barrier)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if (act) pl[buf ^ 1][c][ty + 1][tx + 1] = zp[c];
                if (xrim) pl[buf ^ 1][c][ty + 1][xcol] = rx[c];
                if (yrim) pl[buf ^ 1][c][yrow][tx + 1] = ry[c];
            }
            if (PF == 2) {                                            // rims of plane z+3
                const int zo = wrap32(z + 3, nz) * plane;
#pragma unroll
                for (int c = 0; c < NC; ++c) { rx[c] = rx2[c]; ry[c] = ry2[c]; }
                ld3(zo + y * nx + xs, rx2, xrim && z + 3 < Z1);
                ld3(zo + ys * nx + x, ry2, yrim && z + 3 < Z1);
            } else {                                                  // rims of plane z+2
                const int zo = wrap32(z + 2, nz) * plane;
                ld3(zo + y * nx + xs, rx, xrim && z + 2 < Z1);
                ld3(zo + ys * nx + x, ry, yrim && z + 2 < Z1);
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            zm[c] = zc[c]; zc[c] = zp[c]; zp[c] = zq[c];
            if (PF == 2) zq[c] = zr[c];
        }
    }
}


// One neighbour value of all NC components for a tile rim or a z face.
// Across a block face it comes from the ring: levels n-k and n-k-1 of the
// neighbour block's face (k = 0: level n, which the previous step published
// there, contiguous along the face); inside a block, from the field (loaded
// twice from the same address).  Every lane of a role issues the same 2 NC
// loads whatever k is, so the wait counts stay static and no later wait
// drains the planes in flight.
template <int NC>
struct NbC {
    double a[NC];             // level n-k (or the field)
    double b[NC];             // level n-k-1 (or a repeat of a)
    int k;
};

template <int NC, bool COH = false>
__device__ __forceinline__ NbC<NC> load_nbc(const double *ring, const double *field, bool face,
                                            int k, bool stale, int64_t oring0, int64_t oring1,
                                            int64_t cring, int64_t ofield, int64_t cfield)
{
    const double *p0 = face ? ring + oring0 : field + ofield;
    const double *p1 = (k > 0 && !stale) ? ring + oring1 : p0;
    const int64_t cs = face ? cring : cfield;
    NbC<NC> r;
    r.k = k;
#pragma unroll
    for (int c = 0; c < NC; ++c) r.a[c] = COH ? ld_coherent(p0 + c * cs) : p0[c * cs];
#pragma unroll
    for (int c = 0; c < NC; ++c) r.b[c] = COH ? ld_coherent(p1 + c * cs) : p1[c * cs];
    return r;
}

// AT value H = v0 + k (v0 - v1) (Eq. (1), m = 2); the raw value when k = 0
// and the level n-k value itself in the stale-halo mode
__device__ __forceinline__ double at_h(int k, bool stale, double v0, double v1)
{
    return (k > 0 && !stale) ? v0 + (double)k * (v0 - v1) : v0;
}

// Aligned variant: block widths are multiples of the tile (Wx % 64 == 0,
// Wy % TY == 0), so block faces can only lie on the tile's rims (x, y) or on
// whole planes (z).  Wave 0 computes the x-rim halo values of the next plane
// (lanes 0..2TY-1), waves 0 and 1 the y-rim rows, and every thread the z
// neighbour of the next plane, all one plane ahead; the AT value replaces the
// raw neighbour in the LDS rim (or the z register) and every point then runs
// the same branch-free stencil (the split of section 5.2).  The face delays
// of the chunk are copied to LDS first, and every load inside the march is
// consumed one plane after it is issued.
//
// The march of one 64 x TY tile (corner X0, Y0) through planes Z0 .. Z1-1,
// reading level n from U0 and writing level n+1 to uout; sl0 is the ring slot
// of level n, kdl the LDS delay table of the z-blocks from bz0 on (6 per
// z-block; the prescribed form fills it here from the delay array).  WS (the weakly-synchronous run): ring values move with
// device-coherent loads and stores, and the z neighbour across a block face
// comes from the ring whatever k is (the neighbour block's field may already
// hold another level).
template <int TY, int PF, int NC, bool WS>
__device__ __forceinline__ void march3d(const Step3D &A, const double *const U0,
                                        double *const uout, const int sl0,
                                        double (*pl)[NC][TY + 2][TX + 2], int8_t *kdl,
                                        const int X0, const int Y0, const int Z0, const int Z1,
                                        const int bz0)
{
    static_assert(PF == 1 || PF == 2, "plane queue of 2 or 3 slots");
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int nx = (int)A.nx, ny = (int)A.ny, nz = (int)A.nz;
    const int x = X0 + tx, y = Y0 + ty;
    const int plane = nx * ny;
    const int col = y * nx + x;
    const int Wx = A.Wx, Wy = A.Wy, Wz = A.Wz;
    const int bx = X0 / Wx, by = Y0 / Wy;             // one block per tile in x and y
    const int lx = x - bx * Wx, ly = y - by * Wy;
    const bool fxl = X0 % Wx == 0, fxh = (X0 + TX) % Wx == 0;    // tile edges on block faces
    const bool fyl = Y0 % Wy == 0, fyh = (Y0 + TY) % Wy == 0;
    const int64_t npt = A.npt;
    const bool stale = A.stale != 0;
    const int64_t Py = A.Py, Px = A.Px, bstride = A.bstride, level = A.level;
    const int R = A.R;
    if (!WS) {   // face delays of the z-blocks of this chunk (the WS caller fills kdl itself)
        const int nzb = (Z1 - 1) / Wz - bz0 + 1;          // <= kZB (host bounds ZC)
        const int t = ty * TX + tx;
        const int8_t *krow = A.delays + A.n * A.F;
        if (t < 6 * nzb) {
            const int64_t b = ((int64_t)(bz0 + t / 6) * Py + by) * Px + bx;
            kdl[t] = krow[6 * b + t % 6];
        }
    }

    // rim roles, at most one per lane: waves 0 and 1 the low / high y-rim
    // rows, lanes 0..2TY-1 of wave 2 the x rims (row tx/2, low / high side
    // by tx&1); a role fixes the face, the neighbour block, the position in
    // the face plane, the field column and the LDS slot of the rim value
    const bool y_role = ty < 2;
    const bool x_role = ty == 2 && tx < 2 * TY;
    const bool rim_role = y_role || x_role;
    int r_fidx = 0, r_lzmul = 0, r_lds = 0;
    bool r_face = false;
    int64_t r_blk = 0, r_foff = 0, r_pos = 0, r_cring = 0, r_field = 0;
    if (y_role) {
        r_fidx = 2 + ty;
        r_face = ty ? fyh : fyl;
        r_blk = (int64_t)bx + (int64_t)wrap32(by + (ty ? 1 : -1), A.Py) * Px;
        r_foff = ty ? A.foff[2] : A.foff[3];
        r_pos = lx;
        r_lzmul = Wx;
        r_cring = A.psz[1];
        r_field = (int64_t)(ty ? wrap32(Y0 + TY, ny) : wrap32(Y0 - 1, ny)) * nx + x;
        r_lds = (ty ? TY + 1 : 0) * (TX + 2) + tx + 1;
    } else if (x_role) {
        const int row = tx >> 1, side = tx & 1;
        r_fidx = side;
        r_face = side ? fxh : fxl;
        r_blk = (int64_t)wrap32(bx + (side ? 1 : -1), A.Px) + (int64_t)by * Px;
        r_foff = side ? A.foff[0] : A.foff[1];
        r_pos = (Y0 + row) - by * Wy;
        r_lzmul = Wy;
        r_cring = A.psz[0];
        r_field = (int64_t)(Y0 + row) * nx + (side ? wrap32(X0 + TX, nx) : wrap32(X0 - 1, nx));
        r_lds = (row + 1) * (TX + 2) + (side ? TX + 1 : 0);
    }
    const int64_t z_blk = (int64_t)bx + (int64_t)by * Px;
    const int64_t zlo_foff = A.foff[5], zhi_foff = A.foff[4];
    const int64_t psz0 = A.psz[0], psz1 = A.psz[1], psz2 = A.psz[2];
    const int64_t PyPx = Py * Px;
    auto lvl = [=](int back) -> int64_t {
        int q = sl0 - back;
        if (q < 0) q += R;
        return (int64_t)q * level;
    };

    // planes z-1 and z in registers; planes z+1 .. z+PF in a queue of PF+1
    // register slots that rotates by renaming (the loop is unrolled PF+1
    // times): a slot whose load is still in flight is never copied
    double zm[NC], zc[NC];
    double qa[NC], qb[NC], qc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) zm[c] = U0[c * npt + wrap32(Z0 - 1, nz) * plane + col];
#pragma unroll
    for (int c = 0; c < NC; ++c) zc[c] = U0[c * npt + Z0 * plane + col];
    {
        const int o = wrap32(Z0 + 1, nz) * plane + col;
#pragma unroll
        for (int c = 0; c < NC; ++c) qa[c] = U0[c * npt + o];
    }
    if (PF == 2) {
        const int o = wrap32(Z0 + 2, nz) * plane + col;
#pragma unroll
        for (int c = 0; c < NC; ++c) qb[c] = U0[c * npt + o];
    }
    __syncthreads();                                      // kdl ready

    // loads of plane p's rim values, consumed one plane later
    NbC<NC> rr{};
    auto issue = [&](int p) {
        const int bz = p / Wz, lz = p - bz * Wz;
        if (rim_role) {
            const int k = r_face ? kdl[6 * (bz - bz0) + r_fidx] : 0;
            const int64_t off = (r_blk + (int64_t)bz * PyPx) * bstride + r_foff +
                                (int64_t)lz * r_lzmul + r_pos;
            rr = load_nbc<NC, WS>(A.ring, U0, r_face, k, stale, lvl(k) + off, lvl(k + 1) + off,
                                  r_cring, (int64_t)p * plane + r_field, npt);
        }
    };
    // plane p's rim values into LDS buffer bf
    auto finish_rims = [&](int bf) {
        if (rim_role) {
#pragma unroll
            for (int c = 0; c < NC; ++c)
                (&pl[bf][c][0][0])[r_lds] = at_h(rr.k, stale, rr.a[c], rr.b[c]);
        }
    };
    // z neighbour of plane p across a block face (uniform over the tile):
    // loads issued at the start of the step before, consumed at its end
    NbC<NC> zr{};
    int zside = 0;
    bool zface = false;
    auto issue_z = [&](int p) {
        const int bz = p / Wz, lz = p - bz * Wz;
        zside = lz == 0 ? 0 : 1;
        zface = lz == 0 || lz == Wz - 1;
        const int k = zface ? kdl[6 * (bz - bz0) + 4 + zside] : 0;
        zr.k = k;
        if (k > 0 || (WS && zface)) {
            const int nbz = wrap32(bz + (zside ? 1 : -1), A.Pz);
            const int64_t off = (z_blk + (int64_t)nbz * PyPx) * bstride +
                                (zside ? zhi_foff : zlo_foff) + ly * Wx + lx;
            zr = load_nbc<NC, WS>(A.ring, U0, true, k, stale, lvl(k) + off, lvl(k + 1) + off, psz2,
                                  0, npt);
        }
    };

    double hz[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) hz[c] = 0.0;
    bool hz_lo = false, hz_hi = false;      // plane's z neighbour replaced by hz (low / high)
    auto take_z = [&]() {
        hz_lo = hz_hi = false;
        if (zr.k > 0 || (WS && zface)) {
#pragma unroll
            for (int c = 0; c < NC; ++c) hz[c] = at_h(zr.k, stale, zr.a[c], zr.b[c]);
            hz_lo = zside == 0;
            hz_hi = zside == 1;
        }
    };
    issue_z(Z0);
    issue(Z0);
#pragma unroll
    for (int c = 0; c < NC; ++c) pl[0][c][ty + 1][tx + 1] = zc[c];
    finish_rims(0);
    take_z();
    if (Z0 + 1 < Z1) issue(Z0 + 1);
    const int64_t slot = sl0 + 1 == A.R ? 0 : sl0 + 1;   // level n+1 is published
    const double c10 = A.c1[0], c11 = A.c1[1], c12 = A.c1[2];
    const double c20 = A.c2[0], c21 = A.c2[1], c22 = A.c2[2];
    const double dt = A.dt;

    int bz = Z0 / Wz, lz = Z0 - bz * Wz;
    // one plane: znx holds plane z+1 (complete), zld receives plane z+1+PF
    auto body = [&](int z, double (&znx)[NC], double (&zld)[NC]) {
        if (lz == Wz) { lz = 0; ++bz; }
        const int buf = (z - Z0) & 1;
        const bool more = z + 1 < Z1;
        {
            const int o = wrap32(z + 1 + PF, nz) * plane + col;   // past Z1: unused, in bounds
#pragma unroll
            for (int c = 0; c < NC; ++c) zld[c] = U0[c * npt + o];
        }
        if (more) issue_z(z + 1);
        __syncthreads();
        const double ux = zc[0], uy = zc[1], uz = zc[2];
        double *out = uout + (int64_t)z * plane + col;
        double ov[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double u = zc[c];
            const double zmc = zm[c];
            const double hzc = hz[c];
            const double xl = pl[buf][c][ty + 1][tx], xh = pl[buf][c][ty + 1][tx + 2];
            const double yl = pl[buf][c][ty][tx + 1], yh = pl[buf][c][ty + 2][tx + 1];
            const double zl = hz_lo ? hzc : zmc;
            const double zh = hz_hi ? hzc : znx[c];
            const double D1x = (xh - xl) * c10, D2x = ((xh - 2.0 * u) + xl) * c20;
            const double D1y = (yh - yl) * c11, D2y = ((yh - 2.0 * u) + yl) * c21;
            const double D1z = (zh - zl) * c12, D2z = ((zh - 2.0 * u) + zl) * c22;
            const double lap = (D2x + D2y) + D2z;
            const double adv = (ux * D1x + uy * D1y) + uz * D1z;
            ov[c] = u + dt * (A.kappa[c] * lap - adv);
            __builtin_nontemporal_store(ov[c], &out[c * npt]);
        }
        // publish the level-(n+1) values of points on block faces
        if (A.publish && (lx == 0 || lx == Wx - 1 || ly == 0 || ly == Wy - 1 || lz == 0 ||
                          lz == Wz - 1)) {
            double *base = A.ring + slot * level + (((int64_t)bz * Py + by) * Px + bx) * bstride;
            const int px = lz * Wy + ly, py = lz * Wx + lx, pz = ly * Wx + lx;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double u = ov[c];
                if constexpr (WS) {
                    if (lx == 0) st_coherent(&base[A.foff[0] + c * psz0 + px], u);
                    if (lx == Wx - 1) st_coherent(&base[A.foff[1] + c * psz0 + px], u);
                    if (ly == 0) st_coherent(&base[A.foff[2] + c * psz1 + py], u);
                    if (ly == Wy - 1) st_coherent(&base[A.foff[3] + c * psz1 + py], u);
                    if (lz == 0) st_coherent(&base[A.foff[4] + c * psz2 + pz], u);
                    if (lz == Wz - 1) st_coherent(&base[A.foff[5] + c * psz2 + pz], u);
                } else {
                    if (lx == 0) base[A.foff[0] + c * psz0 + px] = u;
                    if (lx == Wx - 1) base[A.foff[1] + c * psz0 + px] = u;
                    if (ly == 0) base[A.foff[2] + c * psz1 + py] = u;
                    if (ly == Wy - 1) base[A.foff[3] + c * psz1 + py] = u;
                    if (lz == 0) base[A.foff[4] + c * psz2 + pz] = u;
                    if (lz == Wz - 1) base[A.foff[5] + c * psz2 + pz] = u;
                }
            }
        }
        if (more) {
            // plane z+1: interior, rims and z neighbour (loads issued one plane ago)
#pragma unroll
            for (int c = 0; c < NC; ++c) pl[buf ^ 1][c][ty + 1][tx + 1] = znx[c];
            finish_rims(buf ^ 1);
            take_z();
            if (z + 2 < Z1) issue(z + 2);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) { zm[c] = zc[c]; zc[c] = znx[c]; }
        ++lz;
    };
    int z = Z0;
    if (PF == 1) {
        for (; z + 2 <= Z1; z += 2) {
            body(z, qa, qb);
            body(z + 1, qb, qa);
        }
        if (z < Z1) body(z, qa, qb);
    } else {
        for (; z + 3 <= Z1; z += 3) {
            body(z, qa, qc);
            body(z + 1, qb, qa);
            body(z + 2, qc, qb);
        }
        if (z < Z1) body(z++, qa, qc);
        if (z < Z1) body(z, qb, qa);
    }
}

template <int TY, int MINW, int PF, int NC>
__global__ __launch_bounds__(TX * TY, waves_for(MINW, NC)) void k_step3d_aligned(Step3D A)
{
    __shared__ double pl[2][NC][TY + 2][TX + 2];
    __shared__ int8_t kdl[6 * kZB];
    const int X0 = blockIdx.x * TX, Y0 = blockIdx.y * TY;
    const int Z0 = blockIdx.z * A.ZC;
    const int Z1 = (Z0 + A.ZC < (int)A.nz) ? Z0 + A.ZC : (int)A.nz;
    const int bz0 = Z0 / A.Wz;
    march3d<TY, PF, NC, false>(A, A.uin, A.uout, A.slot0, pl, kdl, X0, Y0, Z0, Z1, bz0);
}

// ---------------------------------------------------------------------------
// Two steps per launch (levels n -> n+2) for block shapes that are multiples
// of the 64 x TY tile in x and y.
//
// A workgroup of 66 x (TY + 2) threads marches one 64 x TY tile through the
// planes of a z-chunk.  Thread (ex, ey), ex in [-1, 64], ey in [-1, TY], owns
// one point of the tile widened by one point on every side.  For each plane z
// it computes level n+1 at that point exactly as the block that owns the
// point would: with that block's delays, AT halo values across that block's
// faces (section 2, Eqs. (1)-(2)) and the raw neighbour values elsewhere.
// The threads of the 64 x TY interior then compute level n+2 one plane behind
// (plane z - 1).  Their x/y neighbours come from an LDS plane of level n+1:
// across a face of the tile's block it holds the neighbour block's own level
// n+1 value when the step-(n+1) delay is 0 (computed here, redundantly) and
// the AT value from the ring levels n+1-k, n-k when it is not.  Their z
// neighbours come from the level-n+1 values of the planes before and after,
// or from the ring the same way.  Every point update is the single-step
// kernel's own sequence of operations, so two fused steps give the bits of
// two single steps.
//
// LDS: level n of plane z on the tile widened by two (double-buffered, one
// barrier per plane), level n+1 as the interior reads it (double-buffered),
// and the delays of steps n and n+1 of the blocks around the tile for every
// z-block row the chunk touches.  Each thread issues its own ring loads (AT
// halos) for the next plane at the end of a plane, next to the field load of
// the plane after next, so no load is waited on in the plane that issues it.
// Levels n+1 and n+2 of the interior points on block faces are published to
// the ring (slots n+1 and n+2).
constexpr int kF2X = TX + 2;    // threads per row of the widened tile
constexpr int kZB2 = 16;        // z-block rows the delay table of a fused chunk may span

template <int TY, int NC>
struct F2Lds {
    double a[2][NC][TY + 4][TX + 4];     // level n of a plane, tile widened by two
    double b[2][NC][TY + 2][TX + 2];     // level n+1 of a plane as the interior reads it
    int8_t kd[kZB2][2][3][3][6];         // delays: z-block row, step, x / y block offset, face
};

template <int TY, int NC>
constexpr size_t f2_lds() { return sizeof(F2Lds<TY, NC>); }

__device__ __forceinline__ int fdiv32(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
__device__ __forceinline__ int pmod32(int a, int b) { const int r = a % b; return r < 0 ? r + b : r; }

// an AT halo value in flight: levels n-k-? of a neighbour face, NC components
template <int NC>
struct F2Cross {
    double a[NC], b[NC];
    int k;          // 0: no substitution
    int side;       // which neighbour it replaces (0 low, 1 high)
};

template <int TY, int NC>
__global__ __launch_bounds__(kF2X * (TY + 2)) void k_step3d_f2(Step3D A)
{
    __shared__ F2Lds<TY, NC> sh;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int t = ty * kF2X + tx;
    constexpr int NT = kF2X * (TY + 2);
    const int ex = tx - 1, ey = ty - 1;
    const int nx = (int)A.nx, ny = (int)A.ny, nz = (int)A.nz;
    const int Wx = A.Wx, Wy = A.Wy, Wz = A.Wz;
    const int Px = A.Px, Py = A.Py, Pz = A.Pz;
    const int X0 = blockIdx.x * TX, Y0 = blockIdx.y * TY;
    const int Z0 = blockIdx.z * A.ZC;
    const int Z1 = (Z0 + A.ZC < nz) ? Z0 + A.ZC : nz;
    // offsets in doubles fit in 32 bits for the shapes this kernel accepts
    // (NC x points and the ring below 2^31: at3_variant_ok), so addresses are
    // a uniform base plus one 32-bit register
    const int plane = nx * ny;
    const int npt = (int)A.npt;
    const int level = (int)A.level, bstride = (int)A.bstride;
    const int ps0 = (int)A.psz[0], ps1 = (int)A.psz[1], ps2 = (int)A.psz[2];
    const bool stale = A.stale != 0;
    const int R = A.R;
    const int sl0 = A.slot0;
    const double *U0 = A.uin;

    // this thread's point (ex, ey) of the widened tile and its block
    const int x = wrap32(X0 + ex, nx), y = wrap32(Y0 + ey, ny);
    const int col = y * nx + x;
    const int bxp = x / Wx, byp = y / Wy;
    const int lxp = x - bxp * Wx, lyp = y - byp * Wy;
    const int bx = X0 / Wx, by = Y0 / Wy;                 // the tile's block in x and y
    const int bxo = bxp == bx ? 0 : (ex < 0 ? -1 : 1);    // the point's block, relative
    const int byo = byp == by ? 0 : (ey < 0 ? -1 : 1);
    const bool interior = ex >= 0 && ex < TX && ey >= 0 && ey < TY;
    const bool xlo = lxp == 0, xhi = lxp == Wx - 1;       // on its block's faces (x, y)
    const bool ylo = lyp == 0, yhi = lyp == Wy - 1;
    // rim points next to the interior across a face of the tile's block: that
    // face (its level-n+1 slot then holds what the interior reads across it)
    int rface = -1;
    if (ey >= 0 && ey < TY) {
        if (ex == -1 && X0 % Wx == 0) rface = 0;
        if (ex == TX && (X0 + TX) % Wx == 0) rface = 1;
    }
    if (ex >= 0 && ex < TX) {
        if (ey == -1 && Y0 % Wy == 0) rface = 2;
        if (ey == TY && (Y0 + TY) % Wy == 0) rface = 3;
    }
    // the point of the outer ring (tile widened by two, minus the widened by
    // one) this thread loads, if any: rows -2 and TY+1, then columns -2, TX+1
    constexpr int NOUT = 2 * (TX + 4) + 2 * (TY + 2);
    int ox = 0, oy = 0;
    const bool has_out = t < NOUT;
    if (has_out) {
        if (t < 2 * (TX + 4)) {
            oy = t < TX + 4 ? -2 : TY + 1;
            ox = t % (TX + 4) - 2;
        } else {
            const int o2 = t - 2 * (TX + 4);
            ox = o2 < TY + 2 ? -2 : TX + 1;
            oy = o2 % (TY + 2) - 1;
        }
    }
    // every thread issues the outer-ring load (those without an outer point
    // reload their own), so the count of loads in flight is the same in every
    // wave and every wait in the march can leave the newer loads in flight
    const int ocol = has_out ? wrap32(Y0 + oy, ny) * nx + wrap32(X0 + ox, nx) : col;

    // ---- delays of steps n and n+1 of the 3 x 3 blocks around the tile's
    // block, for each z-block row of planes Z0-1 .. Z1
    const int zb_first = fdiv32(Z0 - 1, Wz);
    const int nzb = fdiv32(Z1, Wz) - zb_first + 1;        // <= kZB2 (host bounds ZC)
    {
        int8_t *kflat = &sh.kd[0][0][0][0][0];
        for (int e = t; e < nzb * 108; e += NT) {
            const int f = e % 6, yo1 = (e / 6) % 3, xo1 = (e / 18) % 3, s = (e / 54) & 1;
            const int j = e / 108;
            const int64_t b = ((int64_t)pmod32(zb_first + j, Pz) * Py + pmod32(by + yo1 - 1, Py)) *
                                  Px + pmod32(bx + xo1 - 1, Px);
            kflat[e] = A.delays[(A.n + s) * A.F + 6 * b + f];
        }
    }
    // ring slot (offset in doubles) of level n + d, |d| <= L + 2 < R
    auto slot = [&](int d) -> int {
        int q = sl0 + d;
        if (q < 0) q += R;
        if (q >= R) q -= R;
        return q * level;
    };
    // offsets of the faces this thread's ring reads use, picked once with
    // constant indices (a per-lane index into the argument block would be a
    // memory load); the neighbour blocks across its x / y faces
    const int fo_x = (int)(xlo ? A.foff[1] : A.foff[0]);  // the x neighbour's face towards it
    const int fo_y = (int)(ylo ? A.foff[3] : A.foff[2]);
    const int fo_zl = (int)A.foff[5], fo_zh = (int)A.foff[4];
    int fo_r = 0;                                         // rim: face rface ^ 1 of its block
    if (rface == 0) fo_r = (int)A.foff[1];
    if (rface == 1) fo_r = (int)A.foff[0];
    if (rface == 2) fo_r = (int)A.foff[3];
    if (rface == 3) fo_r = (int)A.foff[2];
    const int cs_r = rface >= 2 ? ps1 : ps0;
    // loads of an AT halo value: levels n+d-k and n+d-k-1 of the face at
    // offset fo of block (qx, qy, qz), position pos (components cs apart)
    auto cross_load = [&](F2Cross<NC> &cr, int k, int side, int d, int qx, int qy, int qz,
                          int fo, int pos, int cs) {
        cr.k = k;
        cr.side = side;
        if (k > 0) {
            const int fb = ((qz * Py + qy) * Px + qx) * bstride + fo + pos;
            const double *p0 = A.ring + (unsigned)(slot(d - k) + fb);
            const double *p1 = A.ring + (unsigned)((stale ? slot(d - k) : slot(d - k - 1)) + fb);
#pragma unroll
            for (int c = 0; c < NC; ++c) cr.a[c] = p0[(unsigned)(c * cs)];
#pragma unroll
            for (int c = 0; c < NC; ++c) cr.b[c] = p1[(unsigned)(c * cs)];
        }
    };

    auto zneighbour = [&](int bz, bool lo) -> int {
        return lo ? (bz == 0 ? Pz - 1 : bz - 1) : (bz == Pz - 1 ? 0 : bz + 1);
    };
    // position of plane zi along z: wrapped z, block row (wrapped), local z,
    // row of the delay table (recomputed where used: fewer values live)
    struct PlaneZ { int zw, bz, lz, j; };
    auto planez = [&](int zi) -> PlaneZ {
        PlaneZ p;
        p.zw = wrap32(zi, nz);
        p.bz = p.zw / Wz;
        p.lz = p.zw - p.bz * Wz;
        p.j = fdiv32(zi, Wz) - zb_first;
        return p;
    };

    F2Cross<NC> cx{}, cy{}, cz{}, cs{};
    // the ring loads needed in the iteration of plane zi (p = its position,
    // q = that of plane zi-1): the AT halos of level n at this thread's point
    // of plane zi (x, y, z faces of the point's block); for a rim point, what
    // the interior reads across the tile block's face at level n+1; for an
    // interior point, the AT halo of level n+1 across a z face at plane zi-1
    // (whose level n+2 it computes)
    auto issue_cross = [&](int zi) {
        cx.k = cy.k = cz.k = cs.k = 0;
        const PlaneZ p = planez(zi);
        const int8_t *kp = &sh.kd[p.j][0][bxo + 1][byo + 1][0];
        if (xlo || xhi) {
            const int qbx = xlo ? (bxp == 0 ? Px - 1 : bxp - 1) : (bxp == Px - 1 ? 0 : bxp + 1);
            cross_load(cx, kp[xlo ? 0 : 1], xlo ? 0 : 1, 0, qbx, byp, p.bz, fo_x,
                       p.lz * Wy + lyp, ps0);
        }
        if (ylo || yhi) {
            const int qby = ylo ? (byp == 0 ? Py - 1 : byp - 1) : (byp == Py - 1 ? 0 : byp + 1);
            cross_load(cy, kp[ylo ? 2 : 3], ylo ? 0 : 1, 0, bxp, qby, p.bz, fo_y,
                       p.lz * Wx + lxp, ps1);
        }
        if (p.lz == 0 || p.lz == Wz - 1) {
            const bool lo = p.lz == 0;
            cross_load(cz, kp[lo ? 4 : 5], lo ? 0 : 1, 0, bxp, byp, zneighbour(p.bz, lo),
                       lo ? fo_zl : fo_zh, lyp * Wx + lxp, ps2);
        }
        if (rface >= 0) {
            const int pos = rface < 2 ? p.lz * Wy + lyp : p.lz * Wx + lxp;
            cross_load(cs, sh.kd[p.j][1][1][1][rface], rface & 1, 1, bxp, byp, p.bz, fo_r, pos,
                       cs_r);
        } else if (interior && zi - 1 >= Z0) {
            const PlaneZ q = planez(zi - 1);
            if (!(q.lz == 0 || q.lz == Wz - 1)) return;
            const bool lo = q.lz == 0;
            cross_load(cs, sh.kd[q.j][1][1][1][lo ? 4 : 5], lo ? 0 : 1, 1, bx, by,
                       zneighbour(q.bz, lo), lo ? fo_zl : fo_zh, lyp * Wx + lxp, ps2);
        }
    };

    // ---- prologue: level n of planes Z0-2, Z0-1, Z0 at this point; plane
    // Z0-1 (widened by two) into LDS; outer ring of plane Z0 in flight
    double qm[NC], qc[NC], qa[NC], qb[NC], ov[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) qm[c] = U0[(unsigned)(c * npt + wrap32(Z0 - 2, nz) * plane + col)];
#pragma unroll
    for (int c = 0; c < NC; ++c) qc[c] = U0[(unsigned)(c * npt + wrap32(Z0 - 1, nz) * plane + col)];
#pragma unroll
    for (int c = 0; c < NC; ++c) qa[c] = U0[(unsigned)(c * npt + wrap32(Z0, nz) * plane + col)];
#pragma unroll
    for (int c = 0; c < NC; ++c) ov[c] = U0[(unsigned)(c * npt + wrap32(Z0 - 1, nz) * plane + ocol)];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        sh.a[0][c][ey + 2][ex + 2] = qc[c];
        if (has_out) sh.a[0][c][oy + 2][ox + 2] = ov[c];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) ov[c] = U0[(unsigned)(c * npt + wrap32(Z0, nz) * plane + ocol)];
    __syncthreads();                                      // delay table ready
    issue_cross(Z0 - 1);

    const double c10 = A.c1[0], c11 = A.c1[1], c12 = A.c1[2];
    const double c20 = A.c2[0], c21 = A.c2[1], c22 = A.c2[2];
    const double dt = A.dt;
    const int s1 = slot(1), s2 = slot(2);                 // ring slots of levels n+1, n+2
    double h1[NC], h2[NC];                                // level n+1 of planes z-1, z-2
#pragma unroll
    for (int c = 0; c < NC; ++c) h1[c] = h2[c] = 0.0;

    // publish a value of the tile's block at (lx, ly, lz) of block row bzb
    auto publish = [&](int sl, int bzb, int lzb, const double (&v)[NC]) {
        if (!(xlo || xhi || ylo || yhi || lzb == 0 || lzb == Wz - 1)) return;
        const int base = sl + ((bzb * Py + by) * Px + bx) * bstride;
        const int px = lzb * Wy + lyp, py = lzb * Wx + lxp, pz = lyp * Wx + lxp;
        double *R0 = A.ring;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (xlo) R0[(unsigned)(base + (int)A.foff[0] + c * ps0 + px)] = v[c];
            if (xhi) R0[(unsigned)(base + (int)A.foff[1] + c * ps0 + px)] = v[c];
            if (ylo) R0[(unsigned)(base + (int)A.foff[2] + c * ps1 + py)] = v[c];
            if (yhi) R0[(unsigned)(base + (int)A.foff[3] + c * ps1 + py)] = v[c];
            if (lzb == 0) R0[(unsigned)(base + (int)A.foff[4] + c * ps2 + pz)] = v[c];
            if (lzb == Wz - 1) R0[(unsigned)(base + (int)A.foff[5] + c * ps2 + pz)] = v[c];
        }
    };

    // one plane z: qp holds level n of plane z+1 (complete), qn receives
    // plane z+2.  The field and outer-ring loads are unconditional (in bounds
    // past the chunk), so the wait counts are static; the ring loads of the
    // next plane go out last.  (One body per iteration: the queue rotates by
    // copies at the end of a plane, which wait only for the load issued at
    // its start.)
    auto body = [&](int z, double (&qp)[NC], double (&qn)[NC]) {
        const int buf = (z - (Z0 - 1)) & 1;
        {
            const int o = wrap32(z + 2, nz) * plane + col;   // past Z1 + 1: unused, in bounds
#pragma unroll
            for (int c = 0; c < NC; ++c) qn[c] = U0[(unsigned)(c * npt + o)];
        }
        __syncthreads();
        // ---- level n+1 at this point of plane z
        double l1[NC];
        {
            const double ux = qc[0], uy = qc[1], uz = qc[2];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double u = qc[c];
                double xl = sh.a[buf][c][ey + 2][ex + 1], xh = sh.a[buf][c][ey + 2][ex + 3];
                double yl = sh.a[buf][c][ey + 1][ex + 2], yh = sh.a[buf][c][ey + 3][ex + 2];
                double zl = qm[c], zh = qp[c];
                if (cx.k > 0) {
                    const double hv = at_h(cx.k, stale, cx.a[c], cx.b[c]);
                    if (cx.side) xh = hv; else xl = hv;
                }
                if (cy.k > 0) {
                    const double hv = at_h(cy.k, stale, cy.a[c], cy.b[c]);
                    if (cy.side) yh = hv; else yl = hv;
                }
                if (cz.k > 0) {
                    const double hv = at_h(cz.k, stale, cz.a[c], cz.b[c]);
                    if (cz.side) zh = hv; else zl = hv;
                }
                const double D1x = (xh - xl) * c10, D2x = ((xh - 2.0 * u) + xl) * c20;
                const double D1y = (yh - yl) * c11, D2y = ((yh - 2.0 * u) + yl) * c21;
                const double D1z = (zh - zl) * c12, D2z = ((zh - 2.0 * u) + zl) * c22;
                const double lap = (D2x + D2y) + D2z;
                const double adv = (ux * D1x + uy * D1y) + uz * D1z;
                l1[c] = u + dt * (A.kappa[c] * lap - adv);
            }
        }
        // the step-(n+1) AT value of this plane (rim: what the interior reads
        // here; interior: its z neighbour across a face)
        double hs[NC];
        const int hs_k = cs.k, hs_side = cs.side;
#pragma unroll
        for (int c = 0; c < NC; ++c) hs[c] = hs_k > 0 ? at_h(hs_k, stale, cs.a[c], cs.b[c]) : 0.0;
        // what the interior reads here at level n+1
#pragma unroll
        for (int c = 0; c < NC; ++c)
            sh.b[buf][c][ey + 1][ex + 1] = (rface >= 0 && hs_k > 0) ? hs[c] : l1[c];
        const bool own = interior && z >= Z0 && z < Z1;
        if (own) {
            const PlaneZ p = planez(z);
            publish(s1, p.bz, p.lz, l1);
        }
        // ---- level n+2 at this point of plane z-1
        if (interior && z - 1 >= Z0) {
            const int zz = z - 1;
            const int pb = buf ^ 1;
            double l2[NC];
            const double ux = h1[0], uy = h1[1], uz = h1[2];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double u = h1[c];
                const double xl = sh.b[pb][c][ey + 1][ex], xh = sh.b[pb][c][ey + 1][ex + 2];
                const double yl = sh.b[pb][c][ey][ex + 1], yh = sh.b[pb][c][ey + 2][ex + 1];
                double zl = h2[c], zh = l1[c];
                if (hs_k > 0) {
                    if (hs_side) zh = hs[c]; else zl = hs[c];
                }
                const double D1x = (xh - xl) * c10, D2x = ((xh - 2.0 * u) + xl) * c20;
                const double D1y = (yh - yl) * c11, D2y = ((yh - 2.0 * u) + yl) * c21;
                const double D1z = (zh - zl) * c12, D2z = ((zh - 2.0 * u) + zl) * c22;
                const double lap = (D2x + D2y) + D2z;
                const double adv = (ux * D1x + uy * D1y) + uz * D1z;
                l2[c] = u + dt * (A.kappa[c] * lap - adv);
            }
            double *out = A.uout;
            const int oo = zz * plane + col;
#pragma unroll
            for (int c = 0; c < NC; ++c)
                __builtin_nontemporal_store(l2[c], &out[(unsigned)(c * npt + oo)]);
            const PlaneZ p = planez(zz);
            publish(s2, p.bz, p.lz, l2);
        }
        // ---- level n of plane z+1 into the other LDS buffer; the outer ring
        // of plane z+2
        if (z + 1 <= Z1) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                sh.a[buf ^ 1][c][ey + 2][ex + 2] = qp[c];
                if (has_out) sh.a[buf ^ 1][c][oy + 2][ox + 2] = ov[c];
            }
        }
        // rotate the plane queue (the load of plane z+2 was issued at the start
        // of this plane) before the next loads go out
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            qm[c] = qc[c];
            qc[c] = qp[c];
            qp[c] = qn[c];
            h2[c] = h1[c];
            h1[c] = l1[c];
        }
        {
            const int o = wrap32(z + 2, nz) * plane + ocol;  // past Z1: unused, in bounds
#pragma unroll
            for (int c = 0; c < NC; ++c) ov[c] = U0[(unsigned)(c * npt + o)];
        }
        if (z + 1 <= Z1) issue_cross(z + 1);                // ring loads of the next plane
    };
    for (int z = Z0 - 1; z <= Z1; ++z) body(z, qa, qb);
}

// Weakly-synchronous 3D run (emergent delays; paper section 5.2, Algorithm 2):
// one workgroup per block, all blocks resident at once (cooperative launch).
// Before step n, lanes 0..5 poll the level counters of the six face
// neighbours; face f then uses the delay k = n - min(t_f, n), waiting only
// while k would exceed min(L, max(0, n - 1)), and records it.  The block
// marches its tiles through level n (ring reads device-coherent), publishes
// level n+1's faces with device-coherent stores during the march, and
// announces n+1 on its own counter once every store has completed.  Every
// wait is bounded (spin limit, error flag), so every wave reaches the end.
struct Ws3D {
    int32_t *cnt;             // newest announced level per block: [nb]
    int32_t *err;             // 0, or 1 once a wait passed the spin limit
    int8_t *delays;           // delays used, recorded: k[n][6 nb]
    int64_t n0, nsteps, spin_limit;
    int32_t L, jitter;
    uint64_t seed;
};

constexpr int kWsTY = 8;      // tile rows of the weakly-synchronous 3D kernel

template <int NC>
__global__ __launch_bounds__(TX * kWsTY, 4) void k_ws3d(Step3D A, Ws3D W)
{
    __shared__ double pl[2][NC][kWsTY + 2][TX + 2];
    __shared__ int8_t kdl[6];
    __shared__ int s_stop;
    const int t = threadIdx.y * TX + threadIdx.x;
    const int64_t b = blockIdx.x;
    const int bx = (int)(b % A.Px), by = (int)((b / A.Px) % A.Py);
    const int bz = (int)(b / ((int64_t)A.Px * A.Py));
    int64_t q = b;                                    // lanes 0..5: the neighbour across face t
    if (t < 6) {
        const int a = t >> 1, sd = t & 1;
        int nbx = bx, nby = by, nbz = bz;
        if (a == 0) nbx = wrap32(bx + (sd ? 1 : -1), A.Px);
        else if (a == 1) nby = wrap32(by + (sd ? 1 : -1), A.Py);
        else nbz = wrap32(bz + (sd ? 1 : -1), A.Pz);
        q = ((int64_t)nbz * A.Py + nby) * A.Px + nbx;
    }
    if (t == 0) s_stop = 0;
    __syncthreads();
    const double *cur = A.uin;
    double *nxt = A.uout;
    const int ntx = A.Wx / TX, nty = A.Wy / kWsTY;
    for (int64_t n = W.n0; n < W.n0 + W.nsteps; ++n) {
        ws_idle(W.jitter, W.seed, b, n);
        if (t < 6) {
            const int64_t kmax = min((int64_t)W.L, max((int64_t)0, n - 1));
            const int32_t got = ws_wait(W.cnt + q, (int32_t)(n - kmax), W.err, W.spin_limit);
            if (got == -2) {
                s_stop = 1;
            } else {
                const int k = (int)(n - min((int64_t)got, n));
                kdl[t] = (int8_t)k;
                W.delays[n * A.F + 6 * b + t] = (int8_t)k;
            }
        }
        __syncthreads();
        if (s_stop) break;
        const int sl0 = (int)(n % A.R);
        for (int i = 0; i < ntx; ++i)
            for (int j = 0; j < nty; ++j)
                march3d<kWsTY, 1, NC, true>(A, cur, nxt, sl0, pl, kdl, bx * A.Wx + i * TX,
                                            by * A.Wy + j * kWsTY, bz * A.Wz, bz * A.Wz + A.Wz,
                                            bz);
        __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();                              // every face store of level n+1 completed
        if (t == 0)
            __hip_atomic_store(W.cnt + b, (int32_t)(n + 1), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        const double *was = cur;
        cur = nxt;
        nxt = const_cast<double *>(was);
    }
}

// Barrier-free variant: every thread marches its (x, y) column through the
// z range with the z-1, z, z+1 values in registers (plane z+2 in flight) and
// reads its x and y neighbours straight from global memory (L1/L2 hits: the
// same rows are the neighbouring threads' own loads).  No LDS, no barrier, so
// each wave advances on its own and many loads are in flight per wave.
template <int TY, int NC>
__global__ __launch_bounds__(TX * TY) void k_step3d_direct(Step3D A)
{
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int nx = (int)A.nx, ny = (int)A.ny, nz = (int)A.nz;
    const int X0 = blockIdx.x * TX, Y0 = blockIdx.y * TY;
    const int Z0 = blockIdx.z * A.ZC;
    const int Z1 = (Z0 + A.ZC < nz) ? Z0 + A.ZC : nz;
    const int x = X0 + tx, y = Y0 + ty;
    if (x >= nx || y >= ny) return;            // no barrier below: idle threads may leave
    const int plane = nx * ny;
    const int col = y * nx + x;
    const int xm = (x == 0 ? nx : x) - 1, xp = (x + 1 == nx ? 0 : x + 1);
    const int ym = (y == 0 ? ny : y) - 1, yp = (y + 1 == ny ? 0 : y + 1);
    const int bx = x / A.Wx, lx = x - bx * A.Wx;
    const int by = y / A.Wy, ly = y - by * A.Wy;
    const double *U0 = A.uin;
    auto U = [&](int c, int off) -> double { return U0[(int64_t)c * A.npt + off]; };
    double zm[NC], zc[NC], zp[NC], zq[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        zm[c] = U(c, wrap32(Z0 - 1, nz) * plane + col);
        zc[c] = U(c, Z0 * plane + col);
        zp[c] = U(c, wrap32(Z0 + 1, nz) * plane + col);
    }
    const int8_t *krow = A.delays + A.n * A.F;
    const int64_t slot = A.slot0 + 1 == A.R ? 0 : A.slot0 + 1;   // level n+1 is published
    int bz = Z0 / A.Wz, lz = Z0 - bz * A.Wz;
    int kbz = -1, kc[6] = {0, 0, 0, 0, 0, 0};
    for (int z = Z0; z < Z1; ++z, ++lz) {
        if (lz == A.Wz) { lz = 0; ++bz; }
        const bool more = z + 1 < Z1;
        const int po = z * plane;
        double nb[6][NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            zq[c] = more ? U(c, wrap32(z + 2, nz) * plane + col) : 0.0;
            nb[0][c] = U(c, po + y * nx + xm);
            nb[1][c] = U(c, po + y * nx + xp);
            nb[2][c] = U(c, po + ym * nx + x);
            nb[3][c] = U(c, po + yp * nx + x);
            nb[4][c] = zm[c];
            nb[5][c] = zp[c];
        }
        const int64_t b = ((int64_t)bz * A.Py + by) * A.Px + bx;
        if (bz != kbz) {              // face delays of this block: reloaded only at block changes
            kbz = bz;
            kc[0] = lx == 0 ? krow[6 * b + 0] : 0;
            kc[1] = lx == A.Wx - 1 ? krow[6 * b + 1] : 0;
            kc[2] = ly == 0 ? krow[6 * b + 2] : 0;
            kc[3] = ly == A.Wy - 1 ? krow[6 * b + 3] : 0;
            kc[4] = krow[6 * b + 4];
            kc[5] = krow[6 * b + 5];
        }
        const int kf[6] = {kc[0], kc[1], kc[2], kc[3], lz == 0 ? kc[4] : 0,
                           lz == A.Wz - 1 ? kc[5] : 0};
        const int px = lz * A.Wy + ly, py = lz * A.Wx + lx, pz = ly * A.Wx + lx;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            const int kk = kf[f];
            if (kk > 0) {
                const int a = f >> 1, sd = f & 1;
                int n0 = bx, n1 = by, n2 = bz;
                if (a == 0) n0 = wrap32(bx + (sd ? 1 : -1), A.Px);
                else if (a == 1) n1 = wrap32(by + (sd ? 1 : -1), A.Py);
                else n2 = wrap32(bz + (sd ? 1 : -1), A.Pz);
                const int pos = a == 0 ? px : (a == 1 ? py : pz);
                const int64_t off = (((int64_t)n2 * A.Py + n1) * A.Px + n0) * A.bstride +
                                    A.foff[2 * a + (1 - sd)] + pos;
                int s0 = A.slot0 - kk, s1 = A.slot0 - kk - 1;
                if (s0 < 0) s0 += A.R;
                if (s1 < 0) s1 += A.R;
                const double *r0 = A.ring + s0 * A.level + off;
                const double *r1 = A.ring + s1 * A.level + off;
                const double dk = (double)kk;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const double v0 = r0[c * A.psz[a]];
                    nb[f][c] = A.stale ? v0 : v0 + dk * (v0 - r1[c * A.psz[a]]);
                }
            }
        }
        const double ux = zc[0], uy = zc[1], uz = zc[2];
        double *out = A.uout + (int64_t)po + col;
        double ov[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double u = zc[c];
            const double xl = nb[0][c], xr = nb[1][c], yl = nb[2][c], yh = nb[3][c];
            const double zl = nb[4][c], zh = nb[5][c];
            const double D1x = (xr - xl) * A.c1[0], D2x = ((xr - 2.0 * u) + xl) * A.c2[0];
            const double D1y = (yh - yl) * A.c1[1], D2y = ((yh - 2.0 * u) + yl) * A.c2[1];
            const double D1z = (zh - zl) * A.c1[2], D2z = ((zh - 2.0 * u) + zl) * A.c2[2];
            const double lap = (D2x + D2y) + D2z;
            const double adv = (ux * D1x + uy * D1y) + uz * D1z;
            ov[c] = u + A.dt * (A.kappa[c] * lap - adv);
            out[c * A.npt] = ov[c];
        }
        if (A.publish && (lx == 0 || lx == A.Wx - 1 || ly == 0 || ly == A.Wy - 1 || lz == 0 ||
                          lz == A.Wz - 1)) {
            double *base = A.ring + slot * A.level + b * A.bstride;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double u = ov[c];
                if (lx == 0) base[A.foff[0] + c * A.psz[0] + px] = u;
                if (lx == A.Wx - 1) base[A.foff[1] + c * A.psz[0] + px] = u;
                if (ly == 0) base[A.foff[2] + c * A.psz[1] + py] = u;
                if (ly == A.Wy - 1) base[A.foff[3] + c * A.psz[1] + py] = u;
                if (lz == 0) base[A.foff[4] + c * A.psz[2] + pz] = u;
                if (lz == A.Wz - 1) base[A.foff[5] + c * A.psz[2] + pz] = u;
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) { zm[c] = zc[c]; zc[c] = zp[c]; zp[c] = zq[c]; }
    }
}

// Level n's block-face values from the field into ring slot n mod R (the
// steps read the faces of the current level from the ring; a run starts by
// publishing them once)
__global__ __launch_bounds__(256) void k3_publish(Step3D A)
{
    const int64_t nlev = A.level;
    const int64_t slot = A.slot0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nlev;
         e += (int64_t)gridDim.x * 256) {
        const int64_t b = e / A.bstride;
        const int64_t rem = e - b * A.bstride;
        int f = 5;
        while (f > 0 && rem < A.foff[f]) --f;
        const int ax = f >> 1;
        const int64_t r2 = rem - A.foff[f];
        const int c = (int)(r2 / A.psz[ax]);
        const int64_t pos = r2 - c * A.psz[ax];
        const int bx = (int)(b % A.Px), by = (int)((b / A.Px) % A.Py), bz = (int)(b / (A.Px * A.Py));
        int lx, ly, lz;
        if (ax == 0) { lz = (int)(pos / A.Wy); ly = (int)(pos - (int64_t)lz * A.Wy); lx = (f & 1) ? A.Wx - 1 : 0; }
        else if (ax == 1) { lz = (int)(pos / A.Wx); lx = (int)(pos - (int64_t)lz * A.Wx); ly = (f & 1) ? A.Wy - 1 : 0; }
        else { ly = (int)(pos / A.Wx); lx = (int)(pos - (int64_t)ly * A.Wx); lz = (f & 1) ? A.Wz - 1 : 0; }
        const int64_t x = (int64_t)bx * A.Wx + lx, y = (int64_t)by * A.Wy + ly,
                      z = (int64_t)bz * A.Wz + lz;
        A.ring[slot * nlev + e] = A.uin[c * A.npt + (z * A.ny + y) * A.nx + x];
    }
}

// LDS of the plane tiles of a TY-row variant carrying NC components; variants
// above the 160 KiB a gfx950 workgroup may allocate are not instantiated
constexpr size_t kMaxLds = 160 * 1024;
constexpr size_t tile_lds(int TY, int NC) { return 2ull * NC * (TY + 2) * (TX + 2) * 8 + 6 * kZB; }
constexpr bool lds_fits(int TY, int NC) { return tile_lds(TY, NC) <= kMaxLds; }

int zchunk(int64_t nz, int64_t tiles_xy)
{
    // enough workgroups to fill 256 CUs several times over, long z runs otherwise
    int64_t zc = nz;
    while (zc > 16 && tiles_xy * ((nz + zc - 1) / zc) < 2048) zc = (zc + 1) / 2;
    return (int)zc;
}

}  // namespace

}  // namespace atk

using namespace atk;

at_status at3_check(const at_config *c)
{
    if (c->order != 2) return at_fail(AT_ERR_ARG, "3D stepper is order 2");
    if (c->nscalars < 0 || c->nscalars > AT_MAX_SCALARS)
        return at_fail(AT_ERR_ARG, "nscalars out of range");
    for (int a = 0; a < 3; ++a)
        if (c->n[a] / c->p[a] < 2) return at_fail(AT_ERR_SHAPE, "3D block narrower than 2");
    if (c->n[0] * c->n[1] * c->n[2] >= ((int64_t)1 << 31))
        return at_fail(AT_ERR_SHAPE, "3D grid too large (at most 2^31 - 1 points per component)");
    return AT_OK;
}

static int ncomp(const at_config *c) { return 3 + c->nscalars; }

// doubles of one block in a ring level: two faces per axis, NC components each
static int64_t block_stride(const at_config *c)
{
    const int64_t Wx = c->n[0] / c->p[0], Wy = c->n[1] / c->p[1], Wz = c->n[2] / c->p[2];
    return 2 * ncomp(c) * (Wy * Wz + Wx * Wz + Wx * Wy);
}

uint64_t at3_ring_level_doubles(const at_config *c)
{
    return (uint64_t)((int64_t)c->p[0] * c->p[1] * c->p[2] * block_stride(c));
}

// kernel variants the autotuner may choose from (tile rows, prefetch depth,
// register budget); every variant performs the same operations.  Variants
// 15 and 16 advance two steps per launch (k_step3d_f2 with 8 and 4 tile rows).
int at3_variants() { return 17; }
static int k3_rows(int var)
{
    static const int r[17] = {8, 8, 4, 4, 16, 16, 8, 16, 4, 4, 8, 16, 8, 8, 16, 8, 4};
    return r[var < 0 || var > 16 ? 0 : var];
}
static bool is_direct(int var) { return var >= 9 && var <= 11; }
static bool is_aligned(int var) { return (var >= 6 && var <= 8) || (var >= 12 && var <= 14); }
bool at3_is_fused(int var) { return var == 15 || var == 16; }

// LDS of the two-step kernel for TY rows and NC components (0: no build)
static size_t f2_lds_bytes(int ty, int nc)
{
#define F2L(T)                                                                   \
    switch (nc) {                                                                \
    case 3: return f2_lds<T, 3>();                                               \
    case 4: return f2_lds<T, 4>();                                               \
    case 5: return f2_lds<T, 5>();                                               \
    case 6: return f2_lds<T, 6>();                                               \
    case 7: return f2_lds<T, 7>();                                               \
    default: return 0;                                                           \
    }
    if (ty == 8) { F2L(8) }
    if (ty == 4) { F2L(4) }
#undef F2L
    return 0;
}

// aligned variants need block widths that are multiples of the tile; tiled
// variants need their LDS planes for NC components within a workgroup's LDS;
// the two-step variants need both, and blocks at least 2 wide in z
bool at3_variant_ok(const at_config *c, int var)
{
    if (var < 0 || var > 16) return false;
    const int nc = ncomp(c);
    const int64_t Wx = c->n[0] / c->p[0], Wy = c->n[1] / c->p[1], Wz = c->n[2] / c->p[2];
    if (at3_is_fused(var)) {
        // 32-bit offsets: NC fields and the ring (2L + 4 levels) below 2^31 doubles
        const uint64_t npt = (uint64_t)c->n[0] * c->n[1] * c->n[2];
        const uint64_t ring = (uint64_t)(2 * c->L + 4) * at3_ring_level_doubles(c);
        if ((uint64_t)nc * npt >= ((uint64_t)1 << 31) || ring >= ((uint64_t)1 << 31)) return false;
        const size_t lds = f2_lds_bytes(k3_rows(var), nc);
        return lds > 0 && lds <= kMaxLds && Wx % TX == 0 && Wy % k3_rows(var) == 0 && Wz >= 2;
    }
    if (!is_direct(var) && tile_lds(k3_rows(var), nc) > kMaxLds) return false;
    if (!is_aligned(var)) return true;
    return Wx % TX == 0 && Wy % k3_rows(var) == 0;
}

// steps per launch the configuration allows: 2 when a two-step variant has a
// build for its shape
int at3_max_fuse(const at_ctx *ctx)
{
    const at_config *c = at_ctx_cfg(ctx);
    return (at3_variant_ok(c, 15) || at3_variant_ok(c, 16)) ? 2 : 1;
}

// the one-step variant used for a single step when a two-step variant is
// selected (an odd step at the end of a run, at_step)
int at3_single_variant(const at_config *c, int var)
{
    if (!at3_is_fused(var)) return var;
    for (int v : {7, 6, 14, 12, 0})
        if (at3_variant_ok(c, v)) return v;
    return 0;
}

static void fill_step3d(at_ctx *ctx, const double *uin, double *uout, int64_t n0, int publish,
                        Step3D &A)
{
    const at_config *c = at_ctx_cfg(ctx);
    A.uin = uin;
    A.uout = uout;
    A.ring = at_ctx_ring(ctx);
    A.delays = at_ctx_delays(ctx);
    A.nx = c->n[0]; A.ny = c->n[1]; A.nz = c->n[2];
    A.npt = A.nx * A.ny * A.nz;
    A.Px = c->p[0]; A.Py = c->p[1]; A.Pz = c->p[2];
    A.Wx = (int32_t)(A.nx / A.Px); A.Wy = (int32_t)(A.ny / A.Py); A.Wz = (int32_t)(A.nz / A.Pz);
    A.F = 6LL * A.Px * A.Py * A.Pz;
    A.bstride = block_stride(c);
    A.level = (int64_t)A.Px * A.Py * A.Pz * A.bstride;
    A.psz[0] = (int64_t)A.Wy * A.Wz;
    A.psz[1] = (int64_t)A.Wx * A.Wz;
    A.psz[2] = (int64_t)A.Wx * A.Wy;
    const int64_t nc = ncomp(c);
    A.nc = (int32_t)nc;
    A.foff[0] = 0;
    A.foff[1] = nc * A.psz[0];
    A.foff[2] = 2 * nc * A.psz[0];
    A.foff[3] = 2 * nc * A.psz[0] + nc * A.psz[1];
    A.foff[4] = 2 * nc * (A.psz[0] + A.psz[1]);
    A.foff[5] = 2 * nc * (A.psz[0] + A.psz[1]) + nc * A.psz[2];
    A.n = n0;
    A.R = at_ctx_R(ctx);
    A.slot0 = (int32_t)(n0 % A.R);
    A.stale = c->halo_mode;
    A.publish = publish;
    for (int k = 0; k < 3 + AT_MAX_SCALARS; ++k)
        A.kappa[k] = k < 3 ? c->nu : (k - 3 < c->nscalars ? c->alpha[k - 3] : 0.0);
    A.dt = c->dt;
    A.ZC = 0;
    at_ctx_coefs(ctx, A.c1, A.c2);
}

// the k_ws3d build for NC components, or null
static const void *ws3d_kernel(int nc)
{
    switch (nc) {
    case 3: return (const void *)k_ws3d<3>;
    case 4: return (const void *)k_ws3d<4>;
    case 5: return (const void *)k_ws3d<5>;
    case 6: return (const void *)k_ws3d<6>;
    case 7: return (const void *)k_ws3d<7>;
    default: return nullptr;
    }
}

// blocks the weakly-synchronous 3D run can keep resident for this
// configuration, 0 when its block shape is not supported
int64_t at3_ws_capacity(const at_config *c)
{
    const int64_t Wx = c->n[0] / c->p[0], Wy = c->n[1] / c->p[1];
    if (Wx % TX != 0 || Wy % kWsTY != 0) return 0;
    const void *f = ws3d_kernel(ncomp(c));
    if (!f) return 0;
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, TX * kWsTY, 0) != hipSuccess)
        return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return (int64_t)per_cu * cus;
}

// the weakly-synchronous run: level n0 in u, scratch the second field buffer;
// on return the last level is in u (or in scratch: *in_scratch = 1)
at_status at3_launch_ws(at_ctx *ctx, double *u, double *scratch, int64_t n0, int64_t nsteps,
                        int32_t *cnt, int32_t *err, int8_t *delays, int32_t jitter, uint64_t seed,
                        int64_t spin_limit, int *in_scratch)
{
    Step3D A;
    fill_step3d(ctx, u, scratch, n0, 1, A);
    const void *f = ws3d_kernel(A.nc);
    if (!f) return at_fail(AT_ERR_ARG, "no weakly-synchronous 3D build for this component count");
    Ws3D W;
    W.cnt = cnt;
    W.err = err;
    W.delays = delays;
    W.n0 = n0;
    W.nsteps = nsteps;
    W.spin_limit = spin_limit;
    W.L = at_ctx_cfg(ctx)->L;
    W.jitter = jitter;
    W.seed = seed;
    void *args[] = {(void *)&A, (void *)&W};
    const int64_t nb = (int64_t)A.Px * A.Py * A.Pz;
    hipError_t e = hipLaunchCooperativeKernel(f, dim3((unsigned)nb), dim3(TX, kWsTY), args, 0,
                                              at_ctx_stream(ctx));
    if (e != hipSuccess) return at_fail(AT_ERR_HIP, hipGetErrorString(e));
    *in_scratch = (int)(nsteps & 1);
    return AT_OK;
}

at_status at3_publish(at_ctx *ctx, const double *u, int64_t n)
{
    Step3D A;
    fill_step3d(ctx, u, nullptr, n, 1, A);
    int64_t g = (A.level + 255) / 256;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k3_publish, dim3((unsigned)g), dim3(256), 0, at_ctx_stream(ctx), A);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return at_fail(AT_ERR_HIP, hipGetErrorString(e));
    return AT_OK;
}

// The variant table: (tile rows, prefetch depth, waves per SIMD) per kernel
// family; false when the variant has no build for NC components.
template <int NC>
static bool launch3(int var, dim3 grid, dim3 block, hipStream_t st, const Step3D &A)
{
#define K3_TILED(KERNEL, TY)                                                         \
    do {                                                                             \
        if constexpr (lds_fits(TY, NC)) {                                            \
            hipLaunchKernelGGL(KERNEL, grid, block, 0, st, A);                      \
            return true;                                                             \
        }                                                                            \
        return false;                                                                \
    } while (0)
    switch (var) {
    case 0: K3_TILED((k_step3d<8, 1, 4, NC>), 8);
    case 1: K3_TILED((k_step3d<8, 2, 4, NC>), 8);
    case 2: K3_TILED((k_step3d<4, 2, 4, NC>), 4);
    case 3: K3_TILED((k_step3d<4, 2, 3, NC>), 4);
    case 4: K3_TILED((k_step3d<16, 1, 2, NC>), 16);
    case 5: K3_TILED((k_step3d<16, 2, 2, NC>), 16);
    case 6: K3_TILED((k_step3d_aligned<8, 4, 1, NC>), 8);
    case 7: K3_TILED((k_step3d_aligned<16, 2, 1, NC>), 16);
    case 8: K3_TILED((k_step3d_aligned<4, 5, 1, NC>), 4);
    case 12: K3_TILED((k_step3d_aligned<8, 2, 2, NC>), 8);
    case 13: K3_TILED((k_step3d_aligned<8, 3, 2, NC>), 8);
    case 14: K3_TILED((k_step3d_aligned<16, 1, 2, NC>), 16);
    case 9: hipLaunchKernelGGL((k_step3d_direct<4, NC>), grid, block, 0, st, A); return true;
    case 10: hipLaunchKernelGGL((k_step3d_direct<8, NC>), grid, block, 0, st, A); return true;
    case 11: hipLaunchKernelGGL((k_step3d_direct<16, NC>), grid, block, 0, st, A); return true;
    default: return false;
    }
#undef K3_TILED
}

// two steps n0 -> n0 + 2 (k_step3d_f2)
template <int TY, int NC>
static bool launch_f2(dim3 grid, hipStream_t st, const Step3D &A)
{
    if constexpr (f2_lds<TY, NC>() <= kMaxLds) {
        hipLaunchKernelGGL((k_step3d_f2<TY, NC>), grid, dim3(kF2X, TY + 2), 0, st, A);
        return true;
    }
    return false;
}

static at_status at3_launch_f2(at_ctx *ctx, const double *uin, double *uout, int64_t n0)
{
    const at_config *c = at_ctx_cfg(ctx);
    const int var = at_ctx_variant(ctx);
    if (!at3_is_fused(var) || !at3_variant_ok(c, var))
        return at_fail(AT_ERR_ARG, "two steps per launch need a two-step 3D variant (15, 16) "
                                   "that fits this block shape");
    Step3D A;
    fill_step3d(ctx, uin, uout, n0, 1, A);
    const int TYv = k3_rows(var);
    const int64_t gx = A.nx / TX, gy = A.ny / TYv;
    A.ZC = zchunk(A.nz, gx * gy);
    // the chunk's planes Z0-1 .. Z1 span at most kZB2 z-block rows
    if (A.ZC > (kZB2 - 3) * A.Wz) A.ZC = (kZB2 - 3) * A.Wz;
    const int64_t gz = (A.nz + A.ZC - 1) / A.ZC;
    const dim3 grid((unsigned)gx, (unsigned)gy, (unsigned)gz);
    hipStream_t st = at_ctx_stream(ctx);
    bool ok = false;
#define F2N(T)                                                                   \
    switch (A.nc) {                                                              \
    case 3: ok = launch_f2<T, 3>(grid, st, A); break;                            \
    case 4: ok = launch_f2<T, 4>(grid, st, A); break;                            \
    case 5: ok = launch_f2<T, 5>(grid, st, A); break;                            \
    case 6: ok = launch_f2<T, 6>(grid, st, A); break;                            \
    case 7: ok = launch_f2<T, 7>(grid, st, A); break;                            \
    default: break;                                                              \
    }
    if (TYv == 8) { F2N(8) } else { F2N(4) }
#undef F2N
    if (!ok) return at_fail(AT_ERR_ARG, "no two-step 3D build for this component count");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return at_fail(AT_ERR_HIP, hipGetErrorString(e));
    return AT_OK;
}

at_status at3_launch(at_ctx *ctx, const double *uin, double *uout, int64_t n0, int s, int publish)
{
    if (s == 2) return at3_launch_f2(ctx, uin, uout, n0);
    if (s != 1) return at_fail(AT_ERR_ARG, "3D stepper advances one or two steps per launch");
    Step3D A;
    fill_step3d(ctx, uin, uout, n0, publish, A);
    const int var = at3_single_variant(at_ctx_cfg(ctx), at_ctx_variant(ctx));
    const int TYv = k3_rows(var);
    const int64_t gx = (A.nx + TX - 1) / TX, gy = (A.ny + TYv - 1) / TYv;
    A.ZC = zchunk(A.nz, gx * gy);
    if (is_aligned(var) && A.ZC > (kZB - 2) * A.Wz) A.ZC = (kZB - 2) * A.Wz;   // LDS delay table
    const int64_t gz = (A.nz + A.ZC - 1) / A.ZC;
    const dim3 grid((unsigned)gx, (unsigned)gy, (unsigned)gz), block(TX, TYv);
    hipStream_t st = at_ctx_stream(ctx);
    bool ok = false;
    switch (A.nc) {
    case 3: ok = launch3<3>(var, grid, block, st, A); break;
    case 4: ok = launch3<4>(var, grid, block, st, A); break;
    case 5: ok = launch3<5>(var, grid, block, st, A); break;
    case 6: ok = launch3<6>(var, grid, block, st, A); break;
    case 7: ok = launch3<7>(var, grid, block, st, A); break;
    default: break;
    }
    if (!ok) {
        char msg[96];
        snprintf(msg, sizeof msg, "3D kernel variant %d has no build for %d components", var,
                 (int)A.nc);
        return at_fail(AT_ERR_ARG, msg);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return at_fail(AT_ERR_HIP, hipGetErrorString(e));
    return AT_OK;
}
