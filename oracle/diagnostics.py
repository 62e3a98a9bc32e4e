"""Global diagnostics in FP64 (Sec. 5.2).

* Conserved totals: sum_x U_v(x) dV for the five conserved variables.
* Volume-averaged kinetic energy  K = 1/(2 rho0 V) int rho u_i u_i dV.
* Volume-averaged enstrophy  eps = 1/(2 rho0 V) int rho w_i w_i dV, with the
  vorticity w = curl u from the CD4 derivative of the current global field
  (the synchronous view: no delayed data enters a diagnostic).

Integrals are trapezoidal sums on the periodic grid; rho0 = 1.
"""
import numpy as np

from . import flow


def totals(U, h):
    dV = h[0] * h[1] * h[2]
    return np.array([U[v].sum() * dV for v in range(5)])


def kinetic_energy(U, rho0=1.0):
    rho = U[0]
    ke = (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / rho
    return float(ke.sum() / (2.0 * rho0 * ke.size))


def vorticity(U, h, ndim):
    rho = U[0]
    vel = [U[1] / rho, U[2] / rho, U[3] / rho]
    H = 2
    pads = [(0, 0) if ndim == 2 else (H, H), (H, H), (H, H)]
    own = tuple(slice(H, -H) if p != (0, 0) else slice(None) for p in pads)

    def D(f, d):
        if d == 2 and ndim == 2:
            return np.zeros_like(f)
        return flow.cd4(np.pad(f, pads, mode="wrap"), d, h[d])[own]

    wx = D(vel[2], 1) - D(vel[1], 2)
    wy = D(vel[0], 2) - D(vel[2], 0)
    wz = D(vel[1], 0) - D(vel[0], 1)
    return wx, wy, wz


def enstrophy(U, h, ndim, rho0=1.0):
    wx, wy, wz = vorticity(U, h, ndim)
    e = U[0] * (wx * wx + wy * wy + wz * wz)
    return float(e.sum() / (2.0 * rho0 * e.size))


def all_diagnostics(U, h, ndim):
    """[mass, x-mom, y-mom, z-mom, energy totals, K, eps] (7 doubles)."""
    return np.concatenate([totals(U, h), [kinetic_energy(U), enstrophy(U, h, ndim)]])
