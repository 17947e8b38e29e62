"""Seeded synthetic inputs for the AT Burgers stepper: initial fields, workload
parameters, finite-difference probe directions.

This module is the only piece shared by the GPU path and the CPU oracle. It
holds none of the method's arithmetic (no stencil, no halo extrapolation, no
delay generator): it only draws the initial data and fixes the workload
parameters, so that both sides receive identical bytes.

The paper's workload is Burgers' turbulence in a periodic cube with a
"multi-scale sinusoidal" initial condition (section 3.1, Eq. (4)); it names no
dataset. The fields below are seeded stand-ins of that kind:

* ``u0_sines``      sin x plus eight small seeded Fourier modes (1D);
* ``u0_powerlaw``   random-phase Fourier field with amplitude spectrum
                    kappa**-2 up to a cut-off wavenumber (1D);
* ``u0_solenoidal`` divergence-free random vector field with energy spectrum
                    kappa**(-5/3) up to a cut-off, normalised to max |u_i| = 1;
* ``phi0_spectral`` random-phase scalar fields with spectrum kappa**(-5/3),
                    normalised to max |phi| = 1 (the passive scalars of the
                    second line of Eq. (4); the paper gives neither their
                    number nor their diffusivities, so the workload fixes two
                    scalars at Schmidt numbers nu/alpha = 1 and 2).

The time step follows the rule dt = 0.2 * min(dx / max|u0|, dx^2 / (2 nu))
(advective and diffusive limits of forward Euler, section 3.2); it is
computed once, on the host, and is constant for the run.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

BASE_SEED = 20191112
TWO_PI = 2.0 * math.pi

# delay distributions understood by both the library and the oracle
DIST_UNIFORM = 0      # k ~ U{0..L} i.i.d.
DIST_HALF_ZERO = 1    # k = 0 with probability 1/2, else U{1..L}


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(int(seed))


def grid_1d(n: int, length: float = TWO_PI) -> np.ndarray:
    """x_i = i * dx, dx = length / n (periodic, section 3.1)."""
    return np.arange(n, dtype=np.float64) * (length / n)


def u0_sines(n: int, seed: int, nmodes: int = 8, amp: float = 0.01,
             kmin: int = 2, kmax: int = 32) -> np.ndarray:
    """sin(x) + amp * sum_j sin(kappa_j x + theta_j), kappa_j distinct in
    U{kmin..kmax}, theta_j ~ U[0, 2 pi)."""
    g = rng(seed)
    kap = g.choice(np.arange(kmin, kmax + 1), size=nmodes, replace=False)
    th = g.uniform(0.0, TWO_PI, size=nmodes)
    x = grid_1d(n)
    u = np.sin(x)
    for k, t in zip(kap, th):
        u = u + amp * np.sin(k * x + t)
    return np.ascontiguousarray(u, dtype=np.float64)


def u0_powerlaw(n: int, kmax: int, seed: int, slope: float = -2.0) -> np.ndarray:
    """sum_{kappa=1..kmax} kappa**slope * cos(kappa x + theta_kappa), random
    phases, unnormalised, evaluated by an inverse real FFT."""
    kmax = int(min(kmax, n // 2 - 1))
    g = rng(seed)
    th = g.uniform(0.0, TWO_PI, size=kmax)
    spec = np.zeros(n // 2 + 1, dtype=np.complex128)
    kap = np.arange(1, kmax + 1, dtype=np.float64)
    spec[1:kmax + 1] = (n / 2.0) * kap ** slope * np.exp(1j * th)
    return np.ascontiguousarray(np.fft.irfft(spec, n=n), dtype=np.float64)


def u0_solenoidal(n: int, kmax: int, seed: int) -> np.ndarray:
    """Divergence-free random field u[3][z][y][x] on an n^3 periodic grid.

    Complex Gaussian vectors on the shell 1 <= |kappa| <= kmax, projected
    orthogonal to kappa, per-mode amplitude |kappa|**(-11/6) (energy
    spectrum kappa**(-5/3)), made real by an inverse real FFT and scaled so
    that max_i max_x |u_i| = 1."""
    g = rng(seed)
    kfull = np.fft.fftfreq(n, d=1.0 / n)
    sel = np.nonzero(np.abs(kfull) <= kmax)[0]          # z and y indices kept
    selx = np.arange(0, min(kmax, n // 2) + 1)          # rfft (x) indices kept
    # spectrum axes are (z, y, x); physical wavevector (kx, ky, kz)
    KZ, KY, KX = np.meshgrid(kfull[sel], kfull[sel], selx.astype(np.float64),
                             indexing="ij")
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    kmag = np.sqrt(k2)
    shell = (kmag >= 1.0) & (kmag <= kmax)
    c = g.standard_normal((3,) + KX.shape) + 1j * g.standard_normal((3,) + KX.shape)
    kvec = np.stack([KX, KY, KZ])                       # pairs with c[0]=u_x, c[1]=u_y, c[2]=u_z
    kdotc = np.sum(kvec * c, axis=0)
    safe = np.where(k2 > 0, k2, 1.0)
    c = c - kvec * np.where(k2 > 0, kdotc / safe, 0.0)
    c = c * np.where(shell, np.sqrt(safe) ** (-11.0 / 6.0), 0.0)
    out = np.empty((3, n, n, n), dtype=np.float64)
    for comp in range(3):
        spec = np.zeros((n, n, n // 2 + 1), dtype=np.complex128)
        spec[np.ix_(sel, sel, selx)] = c[comp]
        out[comp] = np.fft.irfftn(spec, s=(n, n, n), axes=(0, 1, 2))
        del spec
    out /= np.max(np.abs(out))
    return np.ascontiguousarray(out)


def phi0_spectral(n: int, count: int, kmax: int, seed: int) -> np.ndarray:
    """count scalar fields phi[count][z][y][x] on an n^3 periodic grid: complex
    Gaussian coefficients on the shell 1 <= |kappa| <= kmax with amplitude
    |kappa|**(-11/6), made real by an inverse real FFT, each scaled to
    max |phi| = 1."""
    g = rng(seed)
    kfull = np.fft.fftfreq(n, d=1.0 / n)
    sel = np.nonzero(np.abs(kfull) <= kmax)[0]
    selx = np.arange(0, min(kmax, n // 2) + 1)
    KZ, KY, KX = np.meshgrid(kfull[sel], kfull[sel], selx.astype(np.float64),
                             indexing="ij")
    kmag = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    shell = (kmag >= 1.0) & (kmag <= kmax)
    amp = np.where(shell, np.where(kmag > 0, kmag, 1.0) ** (-11.0 / 6.0), 0.0)
    out = np.empty((count, n, n, n), dtype=np.float64)
    for s_ in range(count):
        c = (g.standard_normal(KX.shape) + 1j * g.standard_normal(KX.shape)) * amp
        spec = np.zeros((n, n, n // 2 + 1), dtype=np.complex128)
        spec[np.ix_(sel, sel, selx)] = c
        out[s_] = np.fft.irfftn(spec, s=(n, n, n), axes=(0, 1, 2))
        del spec
        out[s_] /= max(np.max(np.abs(out[s_])), 1e-300)
    return np.ascontiguousarray(out)


def u0_modes3d(n, nmodes: int, kmax: int, seed: int) -> np.ndarray:
    """Smooth vector field u[3][nz][ny][nx] on a periodic box of any shape:
    per component a sum of nmodes sines with integer wavevectors in
    [-kmax, kmax]^3 and random phases, scaled to max |u_i| = 1."""
    nx, ny, nz = n
    g = rng(seed)
    z = np.arange(nz) * (TWO_PI / nz)
    y = np.arange(ny) * (TWO_PI / ny)
    x = np.arange(nx) * (TWO_PI / nx)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    out = np.zeros((3, nz, ny, nx))
    for c in range(3):
        for _ in range(nmodes):
            k = g.integers(-kmax, kmax + 1, size=3)
            out[c] += g.uniform(0.2, 1.0) * np.sin(k[0] * X + k[1] * Y + k[2] * Z +
                                                   g.uniform(0.0, TWO_PI))
    out /= max(np.max(np.abs(out)), 1e-300)
    return np.ascontiguousarray(out)


def dt_rule(dx: float, max_abs_u: float, nu: float, cfl: float = 0.2) -> float:
    """dt = cfl * min(dx / max|u|, dx^2 / (2 nu))."""
    adv = dx / max_abs_u if max_abs_u > 0 else math.inf
    return cfl * min(adv, dx * dx / (2.0 * nu))


def fd_directions(n: int, count: int, seed: int) -> np.ndarray:
    """count seeded N(0,1) directions of length n (rows)."""
    return rng(seed).standard_normal((count, n))


@dataclasses.dataclass
class Workload:
    name: str
    dim: int
    n: tuple            # points per axis (x, y, z)
    p: tuple            # tiles per axis
    order: int
    L: int
    dist: int
    seed: int           # delay seed
    nu: float
    dt: float
    nsteps: int
    u0: np.ndarray
    length: float = TWO_PI
    extra: Optional[dict] = None

    @property
    def npoints(self) -> int:
        return int(np.prod(self.n))

    @property
    def nfaces(self) -> int:
        return (2 if self.dim == 1 else 6) * int(np.prod(self.p))


def wl_sines_1d(n=1024, p=8, L=2, nu=0.05, nsteps=1000, seed=BASE_SEED,
                dist=DIST_UNIFORM) -> Workload:
    """1D, sin x + 8 small seeded modes, order 2, k ~ U{0..L}."""
    u0 = u0_sines(n, seed)
    dx = TWO_PI / n
    dt = dt_rule(dx, float(np.max(np.abs(u0))), nu)
    return Workload("burgers1d_sines_n%d_p%d_o2_L%d" % (n, p, L), 1, (n, 1, 1), (p, 1, 1),
                    2, L, dist, seed, nu, dt, nsteps, u0)


def wl_powerlaw_1d(n=1 << 24, p=4096, order=4, L=4, nu=1e-3, nsteps=2000,
                   seed=BASE_SEED, dist=DIST_HALF_ZERO, kmax=None) -> Workload:
    """1D, kappa^-2 random-phase field up to n/16, order 4, k = 0 w.p. 1/2
    else U{1..L}."""
    kmax = n // 16 if kmax is None else kmax
    u0 = u0_powerlaw(n, kmax, seed)
    dx = TWO_PI / n
    dt = dt_rule(dx, float(np.max(np.abs(u0))), nu)
    return Workload("burgers1d_powerlaw_n%d_p%d_o%d_L%d" % (n, p, order, L), 1, (n, 1, 1),
                    (p, 1, 1), order, L, dist, seed, nu, dt, nsteps, u0)


def wl_solenoidal_3d(n=512, p=8, L=3, nu=5e-3, nsteps=200, seed=BASE_SEED,
                     dist=DIST_UNIFORM, kmax=32) -> Workload:
    """3D vector, solenoidal kappa^-5/3 field normalised to max|u_i| = 1,
    order 2, blocks of (n/p)^3, k ~ U{0..L}."""
    u0 = u0_solenoidal(n, min(kmax, n // 2 - 1), seed)
    dx = TWO_PI / n
    dt = dt_rule(dx, float(np.max(np.abs(u0))), nu)
    return Workload("burgers3d_solenoidal_n%d_p%d_o2_L%d" % (n, p, L), 3, (n, n, n),
                    (p, p, p), 2, L, dist, seed, nu, dt, nsteps, u0)


def wl_scalars_3d(n=512, p=8, L=3, nu=5e-3, schmidt=(1.0, 2.0), nsteps=200,
                  seed=BASE_SEED, dist=DIST_UNIFORM, kmax=32) -> Workload:
    """3D vector Burgers plus passive scalars (section 3.1, Eq. (4)): the
    solenoidal velocity of wl_solenoidal_3d and len(schmidt) kappa^-5/3
    scalar fields with diffusivities alpha_k = nu / Sc_k; u0 holds
    [3 + len(schmidt)][z][y][x] and extra["alpha"] the diffusivities."""
    km = min(kmax, n // 2 - 1)
    vel = u0_solenoidal(n, km, seed)
    phi = phi0_spectral(n, len(schmidt), km, seed + 1)
    u0 = np.ascontiguousarray(np.concatenate([vel, phi], axis=0))
    del vel, phi
    alpha = tuple(nu / sc for sc in schmidt)
    dx = TWO_PI / n
    dt = dt_rule(dx, 1.0, max((nu,) + alpha))
    return Workload("burgers3d_scalars%d_n%d_p%d_o2_L%d" % (len(schmidt), n, p, L), 3,
                    (n, n, n), (p, p, p), 2, L, dist, seed, nu, dt, nsteps, u0,
                    extra={"alpha": alpha})


def wl_adjoint_1d(n=1 << 20, p=1024, L=3, nu=2e-3, nu_target=3e-3, nsteps=4000,
                  ckpt=100, seed=BASE_SEED, kmax=None) -> Workload:
    """1D adjoint workload: order 2, k ~ U{0..L}; the target field is the same
    u0 advanced with nu_target and the same delays; dt uses max(nu, nu_target)
    so both runs share one step size."""
    kmax = n // 16 if kmax is None else kmax
    u0 = u0_powerlaw(n, kmax, seed)
    dx = TWO_PI / n
    dt = dt_rule(dx, float(np.max(np.abs(u0))), max(nu, nu_target))
    return Workload("burgers1d_adjoint_n%d_p%d_o2_L%d" % (n, p, L), 1, (n, 1, 1), (p, 1, 1),
                    2, L, DIST_UNIFORM, seed, nu, dt, nsteps, u0,
                    extra={"nu_target": nu_target, "ckpt": ckpt})


def batch_instances(count=256, seed=BASE_SEED, log2_lo=12.0, log2_hi=18.0,
                    tile=256, nsteps=500, order=4, kdiv=16):
    """Independent 1D instances of uneven size: N_j = tile*round(2^u/tile),
    u ~ U[log2_lo, log2_hi]; nu_j ~ U[1e-3, 1e-1]; L_j ~ U{1,2,4}; delays
    k = 0 w.p. 1/2 else U{1..L_j}; per-instance seed; P_j = N_j / tile."""
    g = rng(seed)
    out = []
    for j in range(count):
        u = g.uniform(log2_lo, log2_hi)
        n = int(tile * max(1, round(2.0 ** u / tile)))
        nu = float(g.uniform(1e-3, 1e-1))
        L = int(g.choice([1, 2, 4]))
        s = seed + j
        u0 = u0_powerlaw(n, n // kdiv, s)
        dx = TWO_PI / n
        dt = dt_rule(dx, float(np.max(np.abs(u0))), nu)
        out.append(Workload("inst%d" % j, 1, (n, 1, 1), (n // tile, 1, 1), order, L,
                            DIST_HALF_ZERO, s, nu, dt, nsteps, u0))
    return out
