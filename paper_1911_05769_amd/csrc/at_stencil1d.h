// The 1D halo extrapolation and stencil update shared by the 1D kernels of
// libat.so (prescribed-delay steppers and the weakly-synchronous one), so
// that every launch form evaluates the same operations in the same order.
//
//   order 2: D1 = (r1 - l1)*c1,                 D2 = ((r1 - 2u) + l1)*c2
//   order 4: D1 = (8(r1 - l1) - (r2 - l2))*c1,  D2 = ((16(r1 + l1) - 30u) - (r2 + l2))*c2
//   F = nu*D2 - a*D1 (a = u, or c for linear advection),  u' = u + dt*F
//   halo, two levels:   H = v0 + k*(v0 - v1)                     (Eqs. (1)-(2))
//   halo, three levels: H = (v0 + k*d1) + w2*(d1 - (v1 - v2)), d1 = v0 - v1, w2 = 0.5*k*(k+1)
#pragma once

#include "at_internal.h"

namespace atk {

namespace {

template <bool FMA = false>
__device__ __forceinline__ double extrap(int kk, bool stale, double v0, double v1, double v2,
                                         int M)
{
    if (stale) return v0;
    const double dk = (double)kk;
    const double d1 = v0 - v1;
    if constexpr (FMA) {
        if (M == 2) return fma(dk, d1, v0);
        const double w2 = 0.5 * dk * (dk + 1.0);
        return fma(w2, d1 - (v1 - v2), fma(dk, d1, v0));
    }
    if (M == 2) return v0 + dk * d1;
    const double w2 = 0.5 * dk * (dk + 1.0);
    return (v0 + dk * d1) + w2 * (d1 - (v1 - v2));
}

// Exact order: the increment dt*F, with D1 = (8(r1-l1) - (r2-l2))*c1 and
// D2 = ((16(r1+l1) - 30u) - (r2+l2))*c2 (order 2: D1 = (r1-l1)*c1,
// D2 = ((r1 - 2u) + l1)*c2), each operation rounded on its own.  A product by
// 2, 8 or 16 is exact, so fusing it with the following add into one fma rounds
// once where the separate pair also rounds once: the same bits in one
// instruction instead of two.
template <int ORDER, bool LINEAR>
__device__ __forceinline__ double increment(const double *nb, double u, const Step1D &a)
{
    double D1, D2;
    if constexpr (ORDER == 2) {
        const double l1 = nb[0], r1 = nb[1];
        D1 = (r1 - l1) * a.c1;
        D2 = (fma(-2.0, u, r1) + l1) * a.c2;
    } else {
        const double l2 = nb[0], l1 = nb[1], r1 = nb[2], r2 = nb[3];
        D1 = fma(8.0, r1 - l1, -(r2 - l2)) * a.c1;
        D2 = (fma(16.0, r1 + l1, -(30.0 * u)) - (r2 + l2)) * a.c2;
    }
    const double adv = LINEAR ? a.cadv : u;
    const double F = a.nu * D2 - adv * D1;
    return a.dt * F;
}

// Contracted: u' = u + A2*T2 - (a*A1)*T1 with T1 = D1/c1, T2 = D2/c2, split
// into the part that reads the neighbours (T1, T2) and the part that reads the
// point itself, u' = fma(A2, T2, fma(-(a*A1), T1, u))
template <int ORDER>
__device__ __forceinline__ void contracted_terms(const double *nb, double u, double &T1,
                                                 double &T2)
{
    if constexpr (ORDER == 2) {
        T1 = nb[1] - nb[0];
        T2 = fma(-2.0, u, nb[1]) + nb[0];
    } else {
        T1 = fma(8.0, nb[2] - nb[1], -(nb[3] - nb[0]));
        T2 = fma(16.0, nb[2] + nb[1], fma(-30.0, u, -(nb[3] + nb[0])));
    }
}

template <bool LINEAR>
__device__ __forceinline__ double contracted_finish(double T1, double T2, double u,
                                                    const Step1D &a)
{
    const double adv = LINEAR ? a.cadv : u;
    return fma(a.A2, T2, fma(-(adv * a.A1), T1, u));
}

// u' of one point from its neighbours nb (points -H..-1, 1..H) and itself
template <int ORDER, bool LINEAR, bool FMA = false>
__device__ __forceinline__ double update(const double *nb, double u, const Step1D &a)
{
    if constexpr (FMA) {
        double T1, T2;
        contracted_terms<ORDER>(nb, u, T1, T2);
        return contracted_finish<LINEAR>(T1, T2, u, a);
    }
    return u + increment<ORDER, LINEAR>(nb, u, a);
}

// One step of a thread's window w[0 .. PPT+2H): points w[H .. H+PPT) with
// their neighbours' H values on each side.  The new value of point p is
// formed right after the stencil of point p+H, the last one that reads its
// old value, so each new value takes the register of its old one (no window
// copies) and only H+1 pending increments are live at a time.  Every point
// gets exactly the operations of update(), so the bits are the same.
template <int ORDER, bool LINEAR, bool FMA, int PPT>
__device__ __forceinline__ void step_window(double *w, const Step1D &a)
{
    constexpr int H = ORDER / 2;
    if constexpr (!FMA) {
        double g[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            double nb[2 * H];
#pragma unroll
            for (int q = 0; q < H; ++q) { nb[q] = w[j + q]; nb[H + q] = w[j + H + 1 + q]; }
            g[j] = increment<ORDER, LINEAR>(nb, w[H + j], a);
            if (j >= H) w[j] = w[j] + g[j - H];            // point j-H
        }
#pragma unroll
        for (int j = PPT - H; j < PPT; ++j) w[H + j] = w[H + j] + g[j];
    } else {
        double T1[PPT], T2[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            double nb[2 * H];
#pragma unroll
            for (int q = 0; q < H; ++q) { nb[q] = w[j + q]; nb[H + q] = w[j + H + 1 + q]; }
            contracted_terms<ORDER>(nb, w[H + j], T1[j], T2[j]);
            if (j >= H) w[j] = contracted_finish<LINEAR>(T1[j - H], T2[j - H], w[j], a);
        }
#pragma unroll
        for (int j = PPT - H; j < PPT; ++j)
            w[H + j] = contracted_finish<LINEAR>(T1[j], T2[j], w[H + j], a);
    }
}

}  // namespace

}  // namespace atk
