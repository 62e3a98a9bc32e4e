"""Brute-force, one-point-at-a-time evaluation of the right-hand side.

An independent second statement of Eq. (1) / App. A and of the halo rule of
Sec. 3, written with scalar loops so that it can be checked against
``flow.rhs_extended`` and ``solver.Oracle`` on tiny inputs, and used to
check single sampled outputs of large runs.

The CD4 derivative (Eq. 2 with a = 4/3, b = -1/3, alpha = 0) is written here
in its expanded form  (phi_{i-2} - 8 phi_{i-1} + 8 phi_{i+1} - phi_{i+2}) / (12 h),
and CD2 (a = 1, b = 0) as  (phi_{i+1} - phi_{i-1}) / (2 h).
"""
import math

CD4_W = ((-2, 1.0 / 12.0), (-1, -8.0 / 12.0), (1, 8.0 / 12.0), (2, -1.0 / 12.0))
CD2_W = ((-1, -0.5), (1, 0.5))


def weights(order):
    return {4: CD4_W, 2: CD2_W}[order]

UNIT = ((1, 0, 0), (0, 1, 0), (0, 0, 1))


def _prim(get, x, y, z, gas):
    rho = get(0, x, y, z)
    u = get(1, x, y, z) / rho
    v = get(2, x, y, z) / rho
    w = get(3, x, y, z) / rho
    ke = 0.5 * rho * (u * u + v * v + w * w)
    p = (gas.gamma - 1.0) * (get(4, x, y, z) - ke)
    T = gas.gamma * gas.mach * gas.mach * p / rho
    return rho, (u, v, w), p, T


def _inviscid(get, d, x, y, z, gas):
    rho, vel, p, _ = _prim(get, x, y, z, gas)
    ud = vel[d]
    et = get(4, x, y, z)
    f = [rho * ud]
    for i in range(3):
        f.append(rho * vel[i] * ud + (p if i == d else 0.0))
    f.append((et + p) * ud)
    return f


def _gradients(get, x, y, z, h, dims, gas, order=4):
    """(du_i/dx_j, dT/dx_j) at one point."""
    gu = [[0.0] * 3 for _ in range(3)]
    gT = [0.0] * 3
    for j in dims:
        for o, c in weights(order):
            e = UNIT[j]
            _, vel, _, T = _prim(get, x + o * e[0], y + o * e[1], z + o * e[2], gas)
            for i in range(3):
                gu[i][j] += c * vel[i] / h[j]
            gT[j] += c * T / h[j]
    return gu, gT


def _viscous(get, d, x, y, z, h, dims, gas, order=4):
    gu, gT = _gradients(get, x, y, z, h, dims, gas, order)
    _, vel, _, _ = _prim(get, x, y, z, gas)
    divu = gu[0][0] + gu[1][1] + gu[2][2]
    tau = [[gas.mu * (gu[i][j] + gu[j][i]) - (2.0 / 3.0) * gas.mu * divu * (1.0 if i == j else 0.0)
            for j in range(3)] for i in range(3)]
    kappa = gas.mu / ((gas.gamma - 1.0) * gas.mach * gas.mach * gas.pr)
    energy = sum(vel[j] * tau[d][j] for j in range(3)) + kappa * gT[d]
    return [0.0, tau[d][0], tau[d][1], tau[d][2], energy]


def rhs_point(get, h, ndim, physics, gas, order=4):
    """RHS (5 values) at local point (0, 0, 0); get(v, x, y, z) returns the
    conserved variable v at the local offset (x, y, z).  order: 4 (CD4) or 2."""
    dims = [0, 1] if ndim == 2 else [0, 1, 2]
    R = [0.0] * 5
    for d in dims:
        e = UNIT[d]
        for o, c in weights(order):
            F = _inviscid(get, d, o * e[0], o * e[1], o * e[2], gas)
            for v in range(5):
                R[v] -= c * F[v] / h[d]
    if physics == "ns":
        for d in dims:
            e = UNIT[d]
            for o, c in weights(order):
                Fv = _viscous(get, d, o * e[0], o * e[1], o * e[2], h, dims, gas, order)
                for v in range(5):
                    R[v] += c * Fv[v] / h[d] / gas.re
    return R


def slot_of(offsets):
    """Neighbour slot index of a halo point, from its per-axis sign
    (-1 below the block, 0 inside, +1 above)."""
    sx, sy, sz = offsets
    faces = {(-1, 0, 0): 0, (1, 0, 0): 1, (0, -1, 0): 2, (0, 1, 0): 3,
             (0, 0, -1): 4, (0, 0, 1): 5}
    if (sx, sy, sz) in faces:
        return faces[(sx, sy, sz)]
    if sz == 0:
        return 6 + (0 if sx < 0 else 1) + (0 if sy < 0 else 2)
    if sy == 0:
        return 10 + (0 if sx < 0 else 1) + (0 if sz < 0 else 2)
    if sx == 0:
        return 14 + (0 if sy < 0 else 1) + (0 if sz < 0 else 2)
    raise ValueError("corner points carry no halo value")


def block_accessor(Y, history, n, origin, size, point, k=None, W=None, e=0,
                   C=5, mode="sa"):
    """get(v, x, y, z) for block-local stencil access around ``point``.

    Inside the block the stage field Y is used.  Outside: SA uses Y (periodic),
    AS the level n-k, AT sum_l W[e][k][l] U^{n-k-l}; k = k[slot].
    """
    nz, ny, nx = Y.shape[1:]

    def get(v, x, y, z):
        loc = (point[0] + x, point[1] + y, point[2] + z)
        sign = []
        for d in range(3):
            if loc[d] < 0:
                sign.append(-1)
            elif loc[d] >= size[d]:
                sign.append(1)
            else:
                sign.append(0)
        gx = (origin[0] + loc[0]) % nx
        gy = (origin[1] + loc[1]) % ny
        gz = (origin[2] + loc[2]) % nz
        if sign == [0, 0, 0] or mode == "sa" or k is None:
            return float(Y[v, gz, gy, gx])
        kk = int(k[slot_of(tuple(sign))])
        if mode == "as":
            return float(history[n - kk][v, gz, gy, gx])
        tot = 0.0
        for l in range(C):
            tot += W[e][kk][l] * float(history[n - kk - l][v, gz, gy, gx])
        return tot

    return get


def modified_wavenumber(kappa, h, order=4):
    """Exact response of the central difference: D sin(kappa x) =
    kstar cos(kappa x), kstar = (8 sin(kappa h) - sin(2 kappa h)) / (6 h) for
    CD4 and sin(kappa h) / h for CD2."""
    if order == 2:
        return math.sin(kappa * h) / h
    return (8.0 * math.sin(kappa * h) - math.sin(2.0 * kappa * h)) / (6.0 * h)
