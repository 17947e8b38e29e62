// 3D vector stepper of libat.so for gfx950.
//
// Method: u_i,t + u_j d_j u_i = nu d_j d_j u_i (paper section 3.1, Eq. (4)),
// i, j over x, y, z, on a periodic grid split into Px x Py x Pz blocks,
// second-order central differences and forward Euler (section 3.2).  A point
// on a block face reads its neighbour across the face through an AT halo:
// the neighbour block's face value extrapolated in time from levels n-k and
// n-k-1 (section 2, Eqs. (1)-(2): H = v0 + k*(v0 - v1)), with the delay k
// prescribed per directed face and per step.  With k = 0 the halo is the
// neighbour's current value.  Fixed evaluation order (contraction off):
//   D1_a = (r - l)*c1_a,  D2_a = ((r - 2u) + l)*c2_a       for a = x, y, z
//   lap = (D2_x + D2_y) + D2_z,  adv = (u_x*D1_x + u_y*D1_y) + u_z*D1_z
//   u' = u + dt*(nu*lap - adv)
//
// Layout: fields double[3][nz][ny][nx] (x fastest).  Ring level: per block,
// faces x-low, x-high, y-low, y-high, z-low, z-high, each [3][plane] with the
// plane indexed (z, y) for x-faces, (z, x) for y-faces, (y, x) for z-faces.
//
// Work decomposition (2.5D): a workgroup of 64 x 4 threads owns a 64 x 16
// x-y tile and marches through ZC planes in z.  Each thread keeps the z-1, z,
// z+1 values of its 4 rows (3 components) in registers; the current plane
// with one-point rims sits in LDS for the x and y neighbours.  Block faces
// inside the tile are handled per point (any block width >= 2).
#include "../../include/at.h"
#include "at_internal.h"

at_status at_fail(at_status st, const char *msg);
struct at_ctx;
const at_config *at_ctx_cfg(const at_ctx *c);
double *at_ctx_ring(const at_ctx *c);
const int8_t *at_ctx_delays(const at_ctx *c);
int at_ctx_R(const at_ctx *c);
hipStream_t at_ctx_stream(const at_ctx *c);
void at_ctx_coefs(const at_ctx *c, double *c1, double *c2);

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
    double nu, dt, c1[3], c2[3];
};

namespace {

constexpr int TX = 64;        // tile width in x (one wave64 per row)
constexpr int TYW = 4;        // waves per workgroup
constexpr int RY = 4;         // rows per thread
constexpr int TY = TYW * RY;  // tile height in y

__device__ __forceinline__ int64_t wrapi(int64_t i, int64_t n)
{
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

// AT halo across face (axis a, side s) of block (bx, by, bz) for component c
// at face-plane position pos; kk > 0.
__device__ __forceinline__ double halo3(const Step3D &A, int a, int s, int kk, int64_t bx,
                                        int64_t by, int64_t bz, int c, int64_t pos)
{
    int64_t nb[3] = {bx, by, bz};
    const int64_t Pa = a == 0 ? A.Px : (a == 1 ? A.Py : A.Pz);
    nb[a] = wrapi(nb[a] + (s ? 1 : -1), Pa);
    const int64_t b2 = (nb[2] * A.Py + nb[1]) * A.Px + nb[0];
    const int64_t off = b2 * A.bstride + A.foff[2 * a + (1 - s)] + c * A.psz[a] + pos;
    const double v0 = A.ring[((A.n - kk) % A.R) * A.level + off];
    if (A.stale) return v0;
    const double v1 = A.ring[((A.n - kk - 1) % A.R) * A.level + off];
    const double dk = (double)kk;
    return v0 + dk * (v0 - v1);
}

__global__ __launch_bounds__(TX * TYW) void k_step3d(Step3D A)
{
    __shared__ double pl[3][TY + 2][TX + 2];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int64_t X0 = (int64_t)blockIdx.x * TX, Y0 = (int64_t)blockIdx.y * TY;
    const int64_t Z0 = (int64_t)blockIdx.z * A.ZC;
    const int64_t Z1 = (Z0 + A.ZC < A.nz) ? Z0 + A.ZC : A.nz;
    const int wx = (int)((A.nx - X0 < TX) ? A.nx - X0 : TX);
    const int hy = (int)((A.ny - Y0 < TY) ? A.ny - Y0 : TY);
    const int64_t x = X0 + tx;
    const bool xin = tx < wx;
    const int64_t bx = x / A.Wx, lx = x - bx * A.Wx;
    const int64_t plane = A.nx * A.ny;

    double zm[RY][3], zc[RY][3], zp[RY][3];
    int64_t yr[RY], by[RY], ly[RY];
    bool rin[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int yy = ty * RY + r;
        rin[r] = xin && yy < hy;
        yr[r] = Y0 + yy;
        by[r] = yr[r] / A.Wy;
        ly[r] = yr[r] - by[r] * A.Wy;
    }
    {
        const int64_t zlo = wrapi(Z0 - 1, A.nz);
#pragma unroll
        for (int r = 0; r < RY; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                zm[r][c] = rin[r] ? A.uin[c * A.npt + zlo * plane + yr[r] * A.nx + x] : 0.0;
                zc[r][c] = rin[r] ? A.uin[c * A.npt + Z0 * plane + yr[r] * A.nx + x] : 0.0;
            }
    }
    const int8_t *krow = A.delays + A.n * A.F;
    const int64_t slot = A.n % A.R;

    for (int64_t z = Z0; z < Z1; ++z) {
        const int64_t zn = wrapi(z + 1, A.nz);
#pragma unroll
        for (int r = 0; r < RY; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                zp[r][c] = rin[r] ? A.uin[c * A.npt + zn * plane + yr[r] * A.nx + x] : 0.0;
        // current plane -> LDS, with one-point rims
#pragma unroll
        for (int r = 0; r < RY; ++r)
            if (rin[r])      // only owned cells: the rims are written below
#pragma unroll
                for (int c = 0; c < 3; ++c) pl[c][ty * RY + r + 1][tx + 1] = zc[r][c];
        const int64_t zoff = z * plane;
        if (tx < 2) {     // x rims of this thread's rows
            const int64_t xs = tx == 0 ? wrapi(X0 - 1, A.nx) : wrapi(X0 + wx, A.nx);
            const int col = tx == 0 ? 0 : wx + 1;
#pragma unroll
            for (int r = 0; r < RY; ++r)
                if (ty * RY + r < hy)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        pl[c][ty * RY + r + 1][col] = A.uin[c * A.npt + zoff + yr[r] * A.nx + xs];
        }
        if (ty < 2 && xin) {   // y rims
            const int64_t ys = ty == 0 ? wrapi(Y0 - 1, A.ny) : wrapi(Y0 + hy, A.ny);
            const int row = ty == 0 ? 0 : hy + 1;
#pragma unroll
            for (int c = 0; c < 3; ++c) pl[c][row][tx + 1] = A.uin[c * A.npt + zoff + ys * A.nx + x];
        }
        __syncthreads();
        const int64_t bz = z / A.Wz, lz = z - bz * A.Wz;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            if (!rin[r]) continue;
            const int row = ty * RY + r + 1;
            const int64_t b = (bz * A.Py + by[r]) * A.Px + bx;
            // delays of the faces this point touches (0 when it touches none)
            const int kxl = lx == 0 ? krow[6 * b + 0] : 0;
            const int kxh = lx == A.Wx - 1 ? krow[6 * b + 1] : 0;
            const int kyl = ly[r] == 0 ? krow[6 * b + 2] : 0;
            const int kyh = ly[r] == A.Wy - 1 ? krow[6 * b + 3] : 0;
            const int kzl = lz == 0 ? krow[6 * b + 4] : 0;
            const int kzh = lz == A.Wz - 1 ? krow[6 * b + 5] : 0;
            const double ux = zc[r][0], uy = zc[r][1], uz = zc[r][2];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double u = zc[r][c];
                double xl = pl[c][row][tx], xr = pl[c][row][tx + 2];
                double yl = pl[c][row - 1][tx + 1], yh = pl[c][row + 1][tx + 1];
                double zl = zm[r][c], zh = zp[r][c];
                if (kxl) xl = halo3(A, 0, 0, kxl, bx, by[r], bz, c, lz * A.Wy + ly[r]);
                if (kxh) xr = halo3(A, 0, 1, kxh, bx, by[r], bz, c, lz * A.Wy + ly[r]);
                if (kyl) yl = halo3(A, 1, 0, kyl, bx, by[r], bz, c, lz * A.Wx + lx);
                if (kyh) yh = halo3(A, 1, 1, kyh, bx, by[r], bz, c, lz * A.Wx + lx);
                if (kzl) zl = halo3(A, 2, 0, kzl, bx, by[r], bz, c, ly[r] * A.Wx + lx);
                if (kzh) zh = halo3(A, 2, 1, kzh, bx, by[r], bz, c, ly[r] * A.Wx + lx);
                const double D1x = (xr - xl) * A.c1[0], D2x = ((xr - 2.0 * u) + xl) * A.c2[0];
                const double D1y = (yh - yl) * A.c1[1], D2y = ((yh - 2.0 * u) + yl) * A.c2[1];
                const double D1z = (zh - zl) * A.c1[2], D2z = ((zh - 2.0 * u) + zl) * A.c2[2];
                const double lap = (D2x + D2y) + D2z;
                const double adv = (ux * D1x + uy * D1y) + uz * D1z;
                const double F = A.nu * lap - adv;
                A.uout[c * A.npt + zoff + yr[r] * A.nx + x] = u + A.dt * F;
            }
            // publish level n values of points on block faces
            if (A.publish) {
                const int64_t base = slot * A.level + b * A.bstride;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double u = zc[r][c];
                    if (lx == 0) A.ring[base + A.foff[0] + c * A.psz[0] + lz * A.Wy + ly[r]] = u;
                    if (lx == A.Wx - 1) A.ring[base + A.foff[1] + c * A.psz[0] + lz * A.Wy + ly[r]] = u;
                    if (ly[r] == 0) A.ring[base + A.foff[2] + c * A.psz[1] + lz * A.Wx + lx] = u;
                    if (ly[r] == A.Wy - 1) A.ring[base + A.foff[3] + c * A.psz[1] + lz * A.Wx + lx] = u;
                    if (lz == 0) A.ring[base + A.foff[4] + c * A.psz[2] + ly[r] * A.Wx + lx] = u;
                    if (lz == A.Wz - 1) A.ring[base + A.foff[5] + c * A.psz[2] + ly[r] * A.Wx + lx] = u;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RY; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) { zm[r][c] = zc[r][c]; zc[r][c] = zp[r][c]; }
    }
}

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
    for (int a = 0; a < 3; ++a)
        if (c->n[a] / c->p[a] < 2) return at_fail(AT_ERR_SHAPE, "3D block narrower than 2");
    if (c->n[0] * c->n[1] * c->n[2] > ((int64_t)1 << 36))
        return at_fail(AT_ERR_SHAPE, "3D grid too large");
    return AT_OK;
}

static int64_t block_stride(const at_config *c)
{
    const int64_t Wx = c->n[0] / c->p[0], Wy = c->n[1] / c->p[1], Wz = c->n[2] / c->p[2];
    return 6 * (Wy * Wz + Wx * Wz + Wx * Wy);
}

uint64_t at3_ring_level_doubles(const at_config *c)
{
    return (uint64_t)((int64_t)c->p[0] * c->p[1] * c->p[2] * block_stride(c));
}

int at3_max_fuse(const at_ctx *) { return 1; }

at_status at3_launch(at_ctx *ctx, const double *uin, double *uout, int64_t n0, int s, int publish)
{
    if (s != 1) return at_fail(AT_ERR_ARG, "3D stepper advances one step per launch");
    const at_config *c = at_ctx_cfg(ctx);
    Step3D A;
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
    A.foff[0] = 0;
    A.foff[1] = 3 * A.psz[0];
    A.foff[2] = 6 * A.psz[0];
    A.foff[3] = 6 * A.psz[0] + 3 * A.psz[1];
    A.foff[4] = 6 * A.psz[0] + 6 * A.psz[1];
    A.foff[5] = 6 * A.psz[0] + 6 * A.psz[1] + 3 * A.psz[2];
    A.n = n0;
    A.R = at_ctx_R(ctx);
    A.stale = c->halo_mode;
    A.publish = publish;
    A.nu = c->nu;
    A.dt = c->dt;
    at_ctx_coefs(ctx, A.c1, A.c2);
    const int64_t gx = (A.nx + TX - 1) / TX, gy = (A.ny + TY - 1) / TY;
    A.ZC = zchunk(A.nz, gx * gy);
    const int64_t gz = (A.nz + A.ZC - 1) / A.ZC;
    hipLaunchKernelGGL(k_step3d, dim3((unsigned)gx, (unsigned)gy, (unsigned)gz), dim3(TX, TYW),
                       0, at_ctx_stream(ctx), A);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return at_fail(AT_ERR_HIP, hipGetErrorString(e));
    return AT_OK;
}
