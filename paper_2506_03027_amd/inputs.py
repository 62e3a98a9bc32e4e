"""Seeded, synthetic inputs shared by the tests, the benchmark and the oracle.

This module only *generates* inputs: analytic initial fields, seeded smooth
random fields and the time step from a CFL number.  It holds none of the
method's arithmetic (no fluxes, no stencils, no asynchrony-tolerant weights,
no time integration) and imports neither the HIP binding nor the oracle.

Analytic cases
--------------
* Isentropic vortex (the paper's first test case, Sec. 5.1).  The workloads
  use the standard translating isentropic vortex on a periodic box:
  rho_inf = p_inf = T_inf = 1, p = rho T, strength beta, centre (5, 5) of
  [0, 10]^2, freestream 0.5*sqrt(gamma) (Mach 0.5) along the diagonal --
  (1, 1)/sqrt(2) in 2D and (1, 1, 1)/sqrt(3) in 3D with the vortex axis along
  z.  With r the minimum-image distance to the translated centre,
      du = -(beta/2pi) (y-yc) exp((1-r^2)/2),   dv = (beta/2pi) (x-xc) exp((1-r^2)/2),
      T  = 1 - (gamma-1) beta^2 exp(1-r^2) / (8 gamma pi^2),   rho = T^(1/(gamma-1)).
  It is an exact Euler solution on the infinite plane; on the periodic box the
  tail of the perturbation (about 2.4e-5 in velocity at r = 5) sets a floor
  on the error against the translated initial field.
* The paper's own vortex (Sec. 5.1, its Gaussian vortex after Visbal) on
  [-8, 8]^2, Mach 0.1 freestream U_inf = 1 along x, strength
  beta / (U_inf R) = 0.02:  u = U_inf - beta (y-yc)/R^2 exp(-W^2/2),
  v = beta (x-xc)/R^2 exp(-W^2/2),  p_inf - p = rho beta^2/(2 R^2) exp(-W^2),
  W^2 = r^2 / R^2.  The paper leaves R and the density open; R = 1 and a
  uniform rho = 1 are used, with p_inf = 1/(gamma M^2) (so that the sound
  speed is U_inf / M).  With uniform density this field is an exact
  solution of the Euler equations that translates with U_inf: the pressure
  balances the centripetal acceleration and is constant along the
  streamlines of the moving frame.  Grid index 0 sits at x = -8.
* Taylor-Green vortex (Sec. 5.2, Eq. 16) with rho0 = U0 = L0 = 1 on
  [0, 2pi]^3.  The printed v has the sign that makes the field divergent; the
  divergence-free form v = -U0 cos x sin y cos z is used.  The initial
  temperature is uniform, T0 = 1, so rho = gamma M0^2 p.
"""
import math

import numpy as np


def grid_axes(n, length):
    """x_i = i * len / N, i = 0..N-1 (periodic, no duplicated endpoint)."""
    return [np.arange(n[d]) * (length[d] / n[d]) for d in range(3)]


def spacing(n, length):
    return tuple(length[d] / n[d] for d in range(3))


def to_conserved(rho, u, v, w, p, gamma):
    et = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, et]).astype(np.float64)


def vortex_freestream(ndim, gamma, mach=0.5):
    speed = mach * math.sqrt(gamma)
    if ndim == 2:
        return (speed / math.sqrt(2.0), speed / math.sqrt(2.0), 0.0)
    s = speed / math.sqrt(3.0)
    return (s, s, s)


def vortex_state(n, length, ndim, t=0.0, gamma=1.4, beta=5.0,
                 center=(5.0, 5.0), mach=0.5):
    """Conserved isentropic-vortex field (5, nz, ny, nx) at time t."""
    xs, ys, zs = grid_axes(n, length)
    uinf = vortex_freestream(ndim, gamma, mach)
    xc = center[0] + uinf[0] * t
    yc = center[1] + uinf[1] * t
    Lx, Ly = length[0], length[1]
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    dx = (X - xc + 0.5 * Lx) % Lx - 0.5 * Lx
    dy = (Y - yc + 0.5 * Ly) % Ly - 0.5 * Ly
    r2 = dx * dx + dy * dy
    f = np.exp(0.5 * (1.0 - r2))
    u = uinf[0] - beta / (2 * math.pi) * dy * f
    v = uinf[1] + beta / (2 * math.pi) * dx * f
    w = np.full_like(u, uinf[2])
    T = 1.0 - (gamma - 1.0) * beta ** 2 * np.exp(1.0 - r2) / (8.0 * gamma * math.pi ** 2)
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T
    return to_conserved(rho, u, v, w, p, gamma)


VISBAL_BOX = (16.0, 16.0, 1.0)


def visbal_vortex_state(n, t=0.0, gamma=1.4, mach=0.1, strength=0.02, radius=1.0):
    """Conserved field (5, 1, ny, nx) of the paper's Gaussian vortex on
    [-8, 8]^2 (grid index 0 at -8), centred at the origin at t = 0 and
    carried by U_inf = 1 along x (periodic images by minimum distance)."""
    xs, ys, _ = grid_axes((n[0], n[1], 1), VISBAL_BOX)
    Y, X = np.meshgrid(ys - 8.0, xs - 8.0, indexing="ij")
    uinf = 1.0
    beta = strength * uinf * radius
    dx = (X - uinf * t + 8.0) % 16.0 - 8.0
    dy = (Y + 8.0) % 16.0 - 8.0
    om2 = (dx * dx + dy * dy) / radius ** 2
    g = np.exp(-0.5 * om2)
    rho = np.ones_like(X)
    u = uinf - beta * dy / radius ** 2 * g
    v = beta * dx / radius ** 2 * g
    w = np.zeros_like(X)
    p = 1.0 / (gamma * mach ** 2) - rho * beta ** 2 / (2.0 * radius ** 2) * g * g
    return to_conserved(rho[None], u[None], v[None], w[None], p[None], gamma)


def tgv_state(n, mach=0.1, gamma=1.4):
    """Conserved Taylor-Green field on [0, 2pi]^3 (5, nz, ny, nx)."""
    length = (2 * math.pi,) * 3
    xs, ys, zs = grid_axes(n, length)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    u = np.sin(X) * np.cos(Y) * np.cos(Z)
    v = -np.cos(X) * np.sin(Y) * np.cos(Z)
    w = np.zeros_like(u)
    p = 1.0 / (gamma * mach ** 2) + (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0) / 16.0
    rho = gamma * mach ** 2 * p
    return to_conserved(rho, u, v, w, p, gamma)


def smooth_random_state(n, length, seed, amp=0.05, modes=3, gamma=1.4, ndim=3,
                        mach=0.3):
    """A seeded smooth periodic field: uniform state plus a few random
    Fourier modes in every primitive variable."""
    rng = np.random.default_rng(seed)
    xs, ys, zs = grid_axes(n, length)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    prims = []
    base = [1.0, mach * math.sqrt(gamma), -0.5 * mach * math.sqrt(gamma),
            0.25 * mach * math.sqrt(gamma) if ndim == 3 else 0.0, 1.0]
    for var in range(5):
        f = np.full(X.shape, base[var])
        if var == 3 and ndim == 2:
            prims.append(f)
            continue
        for _ in range(modes):
            kx, ky = rng.integers(1, 3, size=2)
            kz = rng.integers(1, 3) if ndim == 3 else 0
            ph = rng.uniform(0, 2 * math.pi)
            a = amp * rng.uniform(0.5, 1.0)
            f = f + a * np.sin(2 * math.pi * (kx * X / length[0] + ky * Y / length[1]
                                                + kz * Z / length[2]) + ph)
        prims.append(f)
    rho, u, v, w, p = prims
    return to_conserved(rho, u, v, w, p, gamma)


def separable_spec(n, length, seed, amp=0.05, modes=2, gamma=1.4, mach=0.3):
    """Parameters of a seeded smooth periodic 3-D field whose primitive
    variables are the uniform state of smooth_random_state plus products of
    1-D sine waves: per variable a list of (amplitude, sx, sy, sz), the 1-D
    factors sampled on the grid.  Cheap at any size, and its value at one
    point is cheap too (separable_at), which the full-size sampled checks
    need."""
    rng = np.random.default_rng(seed)
    xs, ys, zs = grid_axes(n, length)
    base = [1.0, mach * math.sqrt(gamma), -0.5 * mach * math.sqrt(gamma), 0.25 * mach * math.sqrt(gamma), 1.0]
    terms = []
    for _ in range(5):
        tv = []
        for _ in range(modes):
            k = rng.integers(1, 4, size=3)
            ph = rng.uniform(0, 2 * math.pi, size=3)
            a = float(amp * rng.uniform(0.5, 1.0))
            tv.append((a, np.sin(2 * math.pi * k[0] * xs / length[0] + ph[0]),
                       np.sin(2 * math.pi * k[1] * ys / length[1] + ph[1]),
                       np.sin(2 * math.pi * k[2] * zs / length[2] + ph[2])))
        terms.append(tv)
    return {"base": base, "terms": terms, "gamma": gamma}


def _separable_conserved(spec, prim):
    rho, u, v, w, p = (prim(var) for var in range(5))
    inv_gm1 = 1.0 / (spec["gamma"] - 1.0)   # a product, not a division, on every backend
    et = p * inv_gm1 + 0.5 * rho * (u * u + v * v + w * w)
    return [rho, rho * u, rho * v, rho * w, et]


def separable_at(spec, x, y, z):
    """Conserved variables of separable_spec at grid point (x, y, z), in the
    same operation order as separable_field, so both give the same bits."""
    def prim(var):
        f = spec["base"][var]
        for a, sx, sy, sz in spec["terms"][var]:
            f = f + a * (float(sz[z]) * (float(sy[y]) * float(sx[x])))
        return f
    return _separable_conserved(spec, prim)


def separable_field(spec, conv):
    """The five conserved fields of separable_spec on the whole grid, each a
    (nz, ny, nx) array of the type conv() turns a 1-D numpy vector into
    (numpy itself, or a device tensor): only broadcasting arithmetic."""
    def prim(var):
        f = spec["base"][var]
        for a, sx, sy, sz in spec["terms"][var]:
            f = f + a * (conv(sz)[:, None, None] * (conv(sy)[None, :, None] * conv(sx)[None, None, :]))
        return f
    return _separable_conserved(spec, prim)


def cfl_dt(U, n, length, ndim, gamma, cfl):
    """dt = CFL / max_x sum_d (|u_d| + c) / h_d, from the given field."""
    h = spacing(n, length)
    rho = U[0]
    vel = [U[1] / rho, U[2] / rho, U[3] / rho]
    p = (gamma - 1.0) * (U[4] - 0.5 * rho * (vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2))
    c = np.sqrt(gamma * p / rho)
    s = np.zeros_like(rho)
    for d in range(ndim):
        s = s + (np.abs(vel[d]) + c) / h[d]
    return float(cfl / s.max())


# The workloads of the benchmark and parity tests, named by what they are.
WORKLOADS = {
    "vortex2d_64": dict(n=(64, 64, 1), length=(10.0, 10.0, 1.0), ndim=2,
                        nblk=(1, 1, 1), physics="euler", rk="rk4", mode="sa",
                        L=1, cfl=0.5, steps=200, precision="f64"),
    "vortex3d_128": dict(n=(128, 128, 128), length=(10.0, 10.0, 10.0), ndim=3,
                         nblk=(4, 4, 4), physics="euler", rk="rk4", mode="at",
                         algo="saa", L=4, cfl=0.02, precision="f32"),
    # the 128^3 vortex refined once with the same 4 x 4 x 4 blocks (64^3 each):
    # one 5-variable level (335 MB) no longer fits the 256 MB last-level cache
    "vortex3d_256": dict(n=(256, 256, 256), length=(10.0, 10.0, 10.0), ndim=3,
                         nblk=(4, 4, 4), physics="euler", rk="rk4", mode="at",
                         algo="saa", L=4, cfl=0.02, precision="f32"),
    # the second-order method of Table 1 cases 1-3 on the same grid and blocks
    "vortex3d_128_lserk2": dict(n=(128, 128, 128), length=(10.0, 10.0, 10.0), ndim=3,
                                nblk=(4, 4, 4), physics="euler", rk="lserk2", mode="at",
                                algo="saa", L=4, cfl=0.02, precision="f32"),
    # the vortex grid in 8 x 8 x 8 blocks of 16^3 (free-running steps: one
    # resident workgroup per block)
    "vortex3d_128_b16": dict(n=(128, 128, 128), length=(10.0, 10.0, 10.0), ndim=3,
                             nblk=(8, 8, 8), physics="euler", rk="rk4", mode="at",
                             algo="saa", L=4, cfl=0.02, precision="f32"),
    "tgv_256": dict(n=(256, 256, 256), length=(2 * math.pi,) * 3, ndim=3,
                    nblk=(16, 16, 8), physics="ns", rk="rk4", mode="at",
                    algo="saa", L=4, re=1600.0, mach=0.1, cfl=0.02,
                    steps=2000, precision="f32"),
    # the Taylor-Green blocks of tgv_256 (16 x 16 x 32) on a 128^3 grid:
    # 256 blocks, few enough for one resident workgroup each
    "tgv_128": dict(n=(128, 128, 128), length=(2 * math.pi,) * 3, ndim=3,
                    nblk=(8, 8, 4), physics="ns", rk="rk4", mode="at",
                    algo="saa", L=4, re=1600.0, mach=0.1, cfl=0.02,
                    precision="f32"),
    "tgv_512": dict(n=(512, 512, 512), length=(2 * math.pi,) * 3, ndim=3,
                    nblk=(16, 16, 16), physics="ns", rk="rk4", mode="at",
                    algo="saa", L=5, re=1600.0, mach=0.1, cfl=0.01,
                    precision="f32"),
}


def block_split(n, bmax=32):
    """Blocks of bmax points along an axis, the remainder as a last, smaller
    block (uneven at the remainder)."""
    q, r = divmod(n, bmax)
    return [bmax] * q + ([r] if r else [])


def batch_instances(seed=7, count=48, cubes=40):
    """A seeded batch of independent 3-D instances of uneven sizes: `cubes`
    cubes with sides drawn from {32, 48, ..., 160} and the rest boxes of
    other aspect ratios; alternately the isentropic vortex (Euler, [0,10]^3)
    and the Taylor-Green vortex (Navier-Stokes, Re 1600, Mach 0.1,
    [0,2pi]^3); SAA delays with L drawn from {1, 2, 4}; blocks of at most
    32^3 points, uneven at the remainders."""
    rng = np.random.default_rng(seed)
    aspect = [(192, 64, 48), (160, 96, 32), (128, 48, 80), (64, 160, 48),
              (96, 32, 144), (176, 80, 32), (48, 112, 96), (144, 64, 64)]
    out = []
    for i in range(count):
        if i < cubes:
            s = int(rng.choice(np.arange(32, 161, 16)))
            n = (s, s, s)
        else:
            n = aspect[(i - cubes) % len(aspect)]
        ns = i % 2 == 1
        split = tuple(block_split(n[d]) for d in range(3))
        out.append(dict(n=n, length=(2 * math.pi,) * 3 if ns else (10.0, 10.0, 10.0), ndim=3,
                        nblk=tuple(len(s) for s in split), split=split,
                        physics="ns" if ns else "euler", rk="rk4", mode="at", algo="saa",
                        L=int(rng.choice([1, 2, 4])), seed=1000 + i, re=1600.0, mach=0.1,
                        cfl=0.02, precision="f32"))
    return out
