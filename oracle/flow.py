"""Compressible Euler / Navier-Stokes right-hand side on a Cartesian block.

Equations (Sec. 2, Eq. 1; App. A) on a uniform periodic Cartesian grid, where
the metric terms are constants and the contravariant velocities reduce to
u, v, w:
    dU/dt = -sum_d D_d F_d(U) + (1/Re) sum_d D_d Fv_d(U, grad u, grad T)
with U = (rho, rho u, rho v, rho w, rho E_t) and, for direction d,
    F_d  = (rho u_d, rho u u_d + p delta_{1d}, rho v u_d + p delta_{2d},
            rho w u_d + p delta_{3d}, (rho E_t + p) u_d),
    Fv_d = (0, tau_{d1}, tau_{d2}, tau_{d3}, u_j tau_{dj} + kappa dT/dx_d).
Equation of state from App. A: E_t = T/(gamma (gamma-1) M^2) + |u|^2/2, so
    p = (gamma-1) (rho E_t - rho |u|^2 / 2),   T = gamma M^2 p / rho.

Readings where App. A is garbled or silent (all used consistently):
* a single 1/Re multiplies the whole viscous flux (App. A's heat-flux term
  carries a second Re that would double-count it);
* tau_ij = mu (du_i/dx_j + du_j/dx_i) - (2/3) mu delta_ij div u (Stokes);
* kappa = mu / ((gamma-1) M^2 Pr), Pr = 0.71, mu = 1 (constant);
* viscous terms are built as repeated first derivatives (gradients first,
  then the divergence of the viscous flux), as in the paper's form.

Derivatives: the explicit member of Eq. (2) (alpha = 0),
    phi'_i = b (phi_{i+2} - phi_{i-2}) / (4 h) + a (phi_{i+1} - phi_{i-1}) / (2 h),
with the parameters of App. B: CD4 a = 4/3, b = -1/3 (order 4, the default)
and CD2 a = 1, b = 0 (order 2, Table 1 cases 1-3).

Arrays are (z, y, x) per variable, conserved state is (5, z, y, x).  The
"extended" arrays used below carry an apron of depth H around the owned
points (H = 2 for Euler, 4 for Navier-Stokes) and NaN wherever the method
supplies no value, so any use of a point outside the stencil footprint shows
up as NaN in the result.
"""
import numpy as np

CD4_A = 4.0 / 3.0
CD4_B = -1.0 / 3.0
CD2_A = 1.0

EULER, NS = "euler", "ns"


class Gas:
    def __init__(self, gamma=1.4, mach=0.1, re=1600.0, pr=0.71, mu=1.0):
        self.gamma = float(gamma)
        self.mach = float(mach)
        self.re = float(re)
        self.pr = float(pr)
        self.mu = float(mu)

    @property
    def kappa(self):
        g, m = self.gamma, self.mach
        return self.mu / ((g - 1.0) * m * m * self.pr)


def halo_depth(physics):
    return 2 if physics == EULER else 4


def cd4(f, d, h):
    """CD4 derivative of a (z, y, x) array along direction d (0=x, 1=y, 2=z).

    Returns an array of the same shape; the two points at each end of the
    axis, which lack a full stencil, are NaN.
    """
    ax = 2 - d
    n = f.shape[ax]
    out = np.full(f.shape, np.nan)
    if n < 5:
        return out

    def sl(a, b):
        idx = [slice(None)] * 3
        idx[ax] = slice(a, b)
        return tuple(idx)

    fp1 = f[sl(3, n - 1)]
    fm1 = f[sl(1, n - 3)]
    fp2 = f[sl(4, n)]
    fm2 = f[sl(0, n - 4)]
    out[sl(2, n - 2)] = (CD4_B * (fp2 - fm2) / (4.0 * h)
                         + CD4_A * (fp1 - fm1) / (2.0 * h))
    return out


def cd2(f, d, h):
    """CD2 derivative along direction d; the end point on each side is NaN."""
    ax = 2 - d
    n = f.shape[ax]
    out = np.full(f.shape, np.nan)
    if n < 3:
        return out

    def sl(a, b):
        idx = [slice(None)] * 3
        idx[ax] = slice(a, b)
        return tuple(idx)

    out[sl(1, n - 1)] = CD2_A * (f[sl(2, n)] - f[sl(0, n - 2)]) / (2.0 * h)
    return out


def derivative(order):
    """The central difference of the given order (2 or 4)."""
    if order == 4:
        return cd4
    if order == 2:
        return cd2
    raise ValueError("order must be 2 or 4")


def primitives(E, gas):
    rho, mx, my, mz, et = E
    u = mx / rho
    v = my / rho
    w = mz / rho
    p = (gas.gamma - 1.0) * (et - 0.5 * (mx * u + my * v + mz * w))
    return rho, u, v, w, p


def inviscid_fluxes(E, gas):
    """[F_x, F_y, F_z], each a (5, z, y, x) array."""
    _, mx, my, mz, et = E
    _, u, v, w, p = primitives(E, gas)
    out = []
    for mass_flux, vel, pidx in ((mx, u, 1), (my, v, 2), (mz, w, 3)):
        F = np.stack([mass_flux, mx * vel, my * vel, mz * vel, (et + p) * vel])
        F[pidx] = F[pidx] + p
        out.append(F)
    return out


def rhs_extended(E, H, ndim, h, physics, gas, order=4):
    """RHS at the owned points of an extended block.

    E: (5, ez, ey, ex) with an apron of H on both sides of every active
    direction (z has no apron when ndim == 2).  Returns (5, bz, by, bx).
    order: 4 (CD4) or 2 (CD2); the apron depth H is that of CD4 either way,
    CD2 simply reaches less of it.
    """
    cd = derivative(order)
    dims = [0, 1] if ndim == 2 else [0, 1, 2]
    own = [slice(None)] * 3            # (z, y, x) slices of the owned region
    for d in dims:
        own[2 - d] = slice(H, E.shape[3 - d] - H)
    own = tuple(own)

    R = np.zeros((5,) + E[0][own].shape)
    Fs = inviscid_fluxes(E, gas)
    for d in dims:
        for v in range(5):
            R[v] -= cd(Fs[d][v], d, h[d])[own]

    if physics == NS:
        _, u, vv, w, p = primitives(E, gas)
        rho = E[0]
        T = gas.gamma * gas.mach ** 2 * p / rho
        vel = [u, vv, w]
        zero = np.zeros_like(u)
        # gradients du_i/dx_j (i = velocity component, j = direction) and dT/dx_j
        g = [[cd(vel[i], j, h[j]) if j in dims else zero for j in range(3)]
             for i in range(3)]
        gT = [cd(T, j, h[j]) if j in dims else zero for j in range(3)]
        div = g[0][0] + g[1][1] + g[2][2]
        mu = gas.mu
        tau = [[mu * (g[i][j] + g[j][i]) - (2.0 / 3.0) * mu * div * (i == j)
                for j in range(3)] for i in range(3)]
        for d in dims:
            Fv = [zero,
                  tau[d][0], tau[d][1], tau[d][2],
                  u * tau[d][0] + vv * tau[d][1] + w * tau[d][2]
                  + gas.kappa * gT[d]]
            for v in range(1, 5):
                R[v] += cd(Fv[v], d, h[d])[own] / gas.re
    return R


def pad_periodic(U, H, ndim):
    """Periodic padding of a global (5, nz, ny, nx) field by H (the
    synchronous, single-block view)."""
    pads = [(0, 0), (0, 0) if ndim == 2 else (H, H), (H, H), (H, H)]
    return np.pad(U, pads, mode="wrap")


def rhs_global(U, h, ndim, physics, gas, order=4):
    """RHS of the whole periodic field as one block (synchronous view)."""
    H = halo_depth(physics)
    return rhs_extended(pad_periodic(U, H, ndim), H, ndim, h, physics, gas, order)
