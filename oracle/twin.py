"""NumPy restatement of the oracle with full-grid history of every level.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Same method and readings
as at_oracle.c -- delays per directed face and step (section 2), halo values
extrapolated in time from the neighbour's levels n-k, n-k-1, ...
(section 2, Eqs. (1)-(2); quadratic Newton extrapolation for the 4th-order
reading), central differences and forward Euler (section 3.2) -- but written
array-wise, keeping every level ever computed, and generic in the dtype so
that a complex perturbation u0 + i*eps*d gives the exact directional
derivative of the discrete map (complex-step differentiation).  Meant for
small grids only.
"""
from __future__ import annotations

import numpy as np


def _coefs(order, dx):
    if order == 2:
        return 1.0 / (2.0 * dx), 1.0 / (dx * dx)
    return 1.0 / (12.0 * dx), 1.0 / (12.0 * (dx * dx))


def _extrap(kk, m, stale, v0, v1, v2):
    """kk: float array (>= 1 where used); v_j at level n-kk-j."""
    if stale:
        return v0
    d1 = v0 - v1
    if m == 2:
        return v0 + kk * d1
    w2 = 0.5 * kk * (kk + 1.0)
    return (v0 + kk * d1) + w2 * (d1 - (v1 - v2))


class _Neighbours1D:
    """For every point i and stencil offset d: the source point, and the face
    whose halo it is (or -1 when it lies in the point's own tile)."""

    def __init__(self, N, P, h):
        W = N // P
        i = np.arange(N)
        t = i // W
        self.src, self.face = {}, {}
        for d in list(range(-h, 0)) + list(range(1, h + 1)):
            j = i + d
            lo, hi = t * W, (t + 1) * W
            inside = (j >= lo) & (j < hi)
            side = np.where(j < lo, 0, 1)
            self.src[d] = np.mod(j, N)
            self.face[d] = np.where(inside, -1, 2 * t + side)


def run1d(u0, N, P, order, L, nu, dt, k, nsteps, length=2 * np.pi, stale=False,
          linear=False, adv_speed=0.0, nu_c=None, return_history=False):
    """Advance u0 by nsteps.  ``nu_c`` may carry a complex viscosity for
    complex-step derivatives with respect to nu."""
    h = order // 2
    m = 2 if order == 2 else 3
    dx = length / N
    c1, c2 = _coefs(order, dx)
    nb = _Neighbours1D(N, P, h)
    nuv = nu if nu_c is None else nu_c
    hist = [np.array(u0)]
    for n in range(nsteps):
        un = hist[n]
        vals = {}
        for d, src in nb.src.items():
            v = un[src].copy()
            face = nb.face[d]
            halo = face >= 0
            if np.any(halo):
                kk = k[n][face[halo]].astype(np.int64)
                s = src[halo]
                delayed = kk > 0
                if np.any(delayed):
                    kd = kk[delayed]
                    sd = s[delayed]
                    lv = n - kd
                    v0 = np.array([hist[a][b] for a, b in zip(lv, sd)])
                    v1 = np.array([hist[a - 1][b] if m >= 2 and not stale else 0.0
                                   for a, b in zip(lv, sd)])
                    v2 = np.array([hist[a - 2][b] if m >= 3 and not stale else 0.0
                                   for a, b in zip(lv, sd)])
                    hv = _extrap(kd.astype(np.float64), m, stale, v0, v1, v2)
                    tmp = v[halo]
                    tmp[delayed] = hv
                    v[halo] = tmp
            vals[d] = v
        u = un
        if order == 2:
            l1, r1 = vals[-1], vals[1]
            D1 = (r1 - l1) * c1
            D2 = ((r1 - 2.0 * u) + l1) * c2
        else:
            l2, l1, r1, r2 = vals[-2], vals[-1], vals[1], vals[2]
            D1 = (8.0 * (r1 - l1) - (r2 - l2)) * c1
            D2 = ((16.0 * (r1 + l1) - 30.0 * u) - (r2 + l2)) * c2
        a = adv_speed if linear else u
        F = nuv * D2 - a * D1
        hist.append(u + dt * F)
    return hist if return_history else hist[-1]


def run3d(u0, n, p, L, nu, dt, k, nsteps, length=2 * np.pi, stale=False, alpha=()):
    """3D vector Burgers, order 2, u0[3 + len(alpha)][z][y][x]; blocks
    b = (bz*Py+by)*Px+bx, faces f = 6b + 2a + s.  Components past the velocity
    are passive scalars with diffusivities alpha."""
    kappa = [nu, nu, nu] + list(alpha)
    nc = len(kappa)
    nx, ny, nz = n
    Px, Py, Pz = p
    W = (nx // Px, ny // Py, nz // Pz)
    dxs = [length / nx, length / ny, length / nz]
    cs = [_coefs(2, d) for d in dxs]
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    coords = [X, Y, Z]
    blk = [coords[a] // W[a] for a in range(3)]
    b = (blk[2] * Py + blk[1]) * Px + blk[0]
    sizes = [nx, ny, nz]
    hist = [np.array(u0)]
    for step in range(nsteps):
        un = hist[step]
        vel = [un[0], un[1], un[2]]
        D1 = [[None] * 3 for _ in range(nc)]
        D2 = [[None] * 3 for _ in range(nc)]
        for a in range(3):
            lo = blk[a] * W[a]
            hi = lo + W[a]
            for d in (-1, 1):
                j = coords[a] + d
                inside = (j >= lo) & (j < hi)
                side = np.where(j < lo, 0, 1)
                face = 6 * b + 2 * a + side
                sc = [c.copy() for c in coords]
                sc[a] = np.mod(j, sizes[a])
                kk = np.where(inside, 0, k[step][face]).astype(np.int64)
                for comp in range(nc):
                    v = un[comp][sc[2], sc[1], sc[0]]
                    delayed = kk > 0
                    if np.any(delayed):
                        zz, yy, xx = sc[2][delayed], sc[1][delayed], sc[0][delayed]
                        lv = step - kk[delayed]
                        v0 = np.array([hist[q][comp][e, f_, g_] for q, e, f_, g_ in zip(lv, zz, yy, xx)])
                        v1 = np.array([hist[q - 1][comp][e, f_, g_] if not stale else 0.0
                                       for q, e, f_, g_ in zip(lv, zz, yy, xx)])
                        v = v.copy()
                        v[delayed] = _extrap(kk[delayed].astype(np.float64), 2, stale, v0, v1, None)
                    if d == -1:
                        D1[comp][a] = v            # stash l1 temporarily
                    else:
                        l1 = D1[comp][a]
                        r1 = v
                        u = un[comp]
                        D1[comp][a] = (r1 - l1) * cs[a][0]
                        D2[comp][a] = ((r1 - 2.0 * u) + l1) * cs[a][1]
        out = np.empty_like(un)
        for comp in range(nc):
            lap = (D2[comp][0] + D2[comp][1]) + D2[comp][2]
            adv = (vel[0] * D1[comp][0] + vel[1] * D1[comp][1]) + vel[2] * D1[comp][2]
            out[comp] = un[comp] + dt * (kappa[comp] * lap - adv)
        hist.append(out)
    return hist[-1]
