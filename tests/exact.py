"""Closed-form solutions used to pin the oracle (test fixtures).

* Cole-Hopf: for phi_t = nu * Lap(phi) with phi > 0, u = -2 nu grad(log phi)
  solves the viscous Burgers equation u_t + (u . grad) u = nu Lap(u) (the
  paper's Eq. (4) without scalars), in 1D and, for potential flow, in 3D.
  phi = a0 + sum_j b_j exp(-nu |kappa_j|^2 t) cos(kappa_j . x + theta_j),
  a0 > sum |b_j|, is periodic on [0, 2 pi)^d.
* Linear advection-diffusion u_t + c u_x = nu u_xx (the paper's verification
  problem, section 3.2): u = sum_j A_j exp(-nu kappa_j^2 t) sin(kappa_j (x - c t) + theta_j).
* Passive scalar in a uniform velocity U (the second line of Eq. (4); U is an
  exact steady solution of the velocity equation):
  phi = sum_j A_j exp(-alpha |kappa_j|^2 t) sin(kappa_j . (x - U t) + theta_j).
"""
import numpy as np


class ColeHopf1D:
    def __init__(self, nu, modes=((1, 0.3, 0.4), (2, 0.2, 1.3), (3, 0.1, 2.1)), a0=1.2):
        self.nu, self.modes, self.a0 = nu, modes, a0

    def phi(self, x, t):
        p = self.a0 + 0 * x
        for k, b, th in self.modes:
            p = p + b * np.exp(-self.nu * k * k * t) * np.cos(k * x + th)
        return p

    def phi_x(self, x, t):
        p = 0 * x
        for k, b, th in self.modes:
            p = p - b * k * np.exp(-self.nu * k * k * t) * np.sin(k * x + th)
        return p

    def phi_xx(self, x, t):
        p = 0 * x
        for k, b, th in self.modes:
            p = p - b * k * k * np.exp(-self.nu * k * k * t) * np.cos(k * x + th)
        return p

    def u(self, x, t):
        return -2.0 * self.nu * self.phi_x(x, t) / self.phi(x, t)


class ColeHopf3D:
    def __init__(self, nu, modes=(((1, 0, 0), 0.25, 0.3), ((0, 1, 0), 0.2, 1.1),
                                  ((0, 0, 1), 0.15, 2.0), ((1, 1, 0), 0.1, 0.7),
                                  ((0, 1, -1), 0.1, 1.9)), a0=1.3):
        self.nu, self.modes, self.a0 = nu, modes, a0

    def u(self, n, t, length=2 * np.pi):
        x = np.arange(n) * (length / n)
        Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
        phi = self.a0 + 0 * X
        grad = [0 * X, 0 * X, 0 * X]
        for kv, b, th in self.modes:
            kk = kv[0] ** 2 + kv[1] ** 2 + kv[2] ** 2
            arg = kv[0] * X + kv[1] * Y + kv[2] * Z + th
            e = b * np.exp(-self.nu * kk * t)
            phi = phi + e * np.cos(arg)
            for a in range(3):
                grad[a] = grad[a] - e * kv[a] * np.sin(arg)
        return np.stack([-2.0 * self.nu * g / phi for g in grad])


class AdvDiff1D:
    def __init__(self, nu, c, modes=((1, 1.0, 0.2), (2, 0.5, 1.0), (3, 0.25, 2.5))):
        self.nu, self.c, self.modes = nu, c, modes

    def u(self, x, t):
        out = 0 * x
        for k, A, th in self.modes:
            out = out + A * np.exp(-self.nu * k * k * t) * np.sin(k * (x - self.c * t) + th)
        return out


class ScalarUniform3D:
    def __init__(self, alpha, U, modes=(((1, 0, 0), 0.5, 0.3), ((0, 2, 0), 0.3, 1.1),
                                        ((0, 0, 1), 0.4, 2.0), ((1, -1, 1), 0.2, 0.7))):
        self.alpha, self.U, self.modes = alpha, U, modes

    def phi(self, n, t, length=2 * np.pi):
        x = np.arange(n) * (length / n)
        Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
        out = 0 * X
        for kv, A, th in self.modes:
            kk = kv[0] ** 2 + kv[1] ** 2 + kv[2] ** 2
            arg = (kv[0] * (X - self.U[0] * t) + kv[1] * (Y - self.U[1] * t) +
                   kv[2] * (Z - self.U[2] * t) + th)
            out = out + A * np.exp(-self.alpha * kk * t) * np.sin(arg)
        return out
