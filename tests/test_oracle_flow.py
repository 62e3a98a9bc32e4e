"""Pins of the oracle's flux/stencil code against closed forms, exact
invariants and an independent brute-force implementation (no GPU)."""
import math

import numpy as np
import pytest

from oracle import diagnostics, flow, pointwise
from oracle import solver
from paper_2506_03027_amd import inputs


def kstar(kappa, h):
    return pointwise.modified_wavenumber(kappa, h)


# ------------------------------------------------------------------- CD4
def test_cd4_modified_wavenumber_exact():
    n, L = 32, 2 * math.pi
    h = L / n
    x = np.arange(n) * h
    for kap in (1, 2, 5):
        f = np.sin(kap * x)[None, None, :] * np.ones((1, 1, 1))
        fp = np.pad(f, ((0, 0), (0, 0), (2, 2)), mode="wrap")
        d = flow.cd4(fp, 0, h)[:, :, 2:-2]
        assert np.allclose(d[0, 0], kstar(kap, h) * np.cos(kap * x), atol=1e-13)


def test_cd4_fourth_order():
    errs = []
    for n in (32, 64, 128):
        h = 1.0 / n
        x = np.arange(n) * h
        f = np.exp(np.sin(2 * math.pi * x))
        fp = np.pad(f[None, None, :], ((0, 0), (0, 0), (2, 2)), mode="wrap")
        d = flow.cd4(fp, 0, h)[0, 0, 2:-2]
        exact = 2 * math.pi * np.cos(2 * math.pi * x) * f
        errs.append(np.abs(d - exact).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) > 3.8


def test_cd2_modified_wavenumber_exact():
    # CD2 (App. B: a = 1, b = 0) maps sin(kx) to (sin(kh)/h) cos(kx) exactly
    n, L = 32, 2 * math.pi
    h = L / n
    x = np.arange(n) * h
    for kap in (1, 3, 7):
        f = np.sin(kap * x)[None, None, :]
        fp = np.pad(f, ((0, 0), (0, 0), (2, 2)), mode="wrap")
        d = flow.cd2(fp, 0, h)[:, :, 2:-2]
        assert np.allclose(d[0, 0], math.sin(kap * h) / h * np.cos(kap * x), atol=1e-13)


def test_cd2_second_order_and_exact_for_quadratics():
    errs = []
    for n in (32, 64, 128):
        h = 1.0 / n
        x = np.arange(n) * h
        f = np.exp(np.sin(2 * math.pi * x))
        fp = np.pad(f[None, None, :], ((0, 0), (0, 0), (1, 1)), mode="wrap")
        d = flow.cd2(fp, 0, h)[0, 0, 1:-1]
        exact = 2 * math.pi * np.cos(2 * math.pi * x) * f
        errs.append(np.abs(d - exact).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert 1.9 < min(orders) and max(orders) < 2.1, orders
    # a quadratic along y (no wrap needed inside the array): exact derivative
    y = np.linspace(-1.0, 2.0, 9)
    h = y[1] - y[0]
    q = (3.0 * y * y - 2.0 * y + 0.5)[None, :, None] * np.ones((2, 1, 3))
    d = flow.cd2(q, 1, h)[:, 1:-1, :]
    assert np.allclose(d, (6.0 * y - 2.0)[None, 1:-1, None], atol=1e-12)
    assert np.isnan(flow.cd2(q, 1, h)[:, 0, :]).all()


# ------------------------------------------------------- NS closed forms
def _rhs(U, n, length, physics, gas, ndim=3):
    h = inputs.spacing(n, length)
    return flow.rhs_global(U, h, ndim, physics, gas)


def _grid(n, length):
    xs, ys, zs = inputs.grid_axes(n, length)
    return np.meshgrid(zs, ys, xs, indexing="ij")


GAS = flow.Gas(gamma=1.4, mach=0.1, re=100.0, pr=0.71)
N3 = (16, 16, 16)
L3 = (2 * math.pi,) * 3


def test_ns_shear_wave_closed_form():
    # rho = 1, u = eps sin y, p const: inviscid part vanishes; viscous part
    # is the CD4-of-CD4 response of the shear stress tau_xy = mu du/dy.
    Z, Y, X = _grid(N3, L3)
    eps, p0 = 1e-2, 1.0 / (GAS.gamma * GAS.mach ** 2)
    u = eps * np.sin(Y)
    z0 = np.zeros_like(u)
    U = inputs.to_conserved(np.ones_like(u), u, z0, z0, np.full_like(u, p0), GAS.gamma)
    R = _rhs(U, N3, L3, flow.NS, GAS)
    h = L3[1] / N3[1]
    k1, k2 = kstar(1, h), kstar(2, h)
    exp_mx = -eps * k1 * k1 * np.sin(Y) / GAS.re
    exp_e = (eps ** 2 * k1 / 2) * k2 * np.cos(2 * Y) / GAS.re
    assert np.abs(R[1] - exp_mx).max() < 1e-12
    assert np.abs(R[4] - exp_e).max() < 1e-12
    for v in (0, 2, 3):
        assert np.abs(R[v]).max() < 1e-11


def test_ns_heat_conduction_closed_form():
    # rho = 1, u = 0, T = 1 + eps sin z: pressure gradient and heat flux only.
    Z, Y, X = _grid(N3, L3)
    eps = 1e-2
    g, M = GAS.gamma, GAS.mach
    T = 1 + eps * np.sin(Z)
    p = T / (g * M * M)
    z0 = np.zeros_like(T)
    U = inputs.to_conserved(np.ones_like(T), z0, z0, z0, p, g)
    R = _rhs(U, N3, L3, flow.NS, GAS)
    h = L3[2] / N3[2]
    k1 = kstar(1, h)
    kappa = 1.0 / ((g - 1) * M * M * GAS.pr)
    assert np.abs(R[3] - (-eps * k1 * np.cos(Z) / (g * M * M))).max() < 1e-9
    assert np.abs(R[4] - (-kappa * eps * k1 * k1 * np.sin(Z) / GAS.re)).max() < 1e-9
    for v in (0, 1, 2):
        assert np.abs(R[v]).max() < 1e-10


def test_ns_compression_wave_closed_form():
    # u = eps sin x: pins tau_xx = (4/3) mu du/dx (the Stokes -2/3 div term)
    # and the u tau energy flux, with the exact inviscid response.
    Z, Y, X = _grid(N3, L3)
    eps, g = 1e-2, GAS.gamma
    p0 = 1.0 / (g * GAS.mach ** 2)
    u = eps * np.sin(X)
    z0 = np.zeros_like(u)
    U = inputs.to_conserved(np.ones_like(u), u, z0, z0, np.full_like(u, p0), g)
    R = _rhs(U, N3, L3, flow.NS, GAS)
    h = L3[0] / N3[0]
    k1, k2, k3 = kstar(1, h), kstar(2, h), kstar(3, h)
    re = GAS.re
    exp_rho = -eps * k1 * np.cos(X)
    exp_mx = -(eps ** 2 / 2) * k2 * np.sin(2 * X) - (4.0 / 3.0) * eps * k1 * k1 * np.sin(X) / re
    inv_e = (g * p0 / (g - 1)) * eps * k1 * np.cos(X) \
        + 0.5 * eps ** 3 * (3 * k1 * np.cos(X) - k3 * np.cos(3 * X)) / 4
    exp_e = -inv_e + (2.0 / 3.0) * eps ** 2 * k1 * k2 * np.cos(2 * X) / re
    assert np.abs(R[0] - exp_rho).max() < 1e-12
    assert np.abs(R[1] - exp_mx).max() < 1e-11
    assert np.abs(R[4] - exp_e).max() < 1e-9
    assert np.abs(R[2]).max() < 1e-11 and np.abs(R[3]).max() < 1e-11


def test_rhs_rotation_covariance():
    # Cyclic relabelling x->y->z->x of coordinates and velocity components
    # must relabel the RHS the same way (catches direction-specific slips).
    n = (12, 12, 12)
    U = inputs.smooth_random_state(n, L3, seed=5, amp=0.05)
    # new field at (x,y,z) = old at (z,x,y): array axes (z,y,x)
    def rot(A):
        # new field B(x', y', z') = A(x=y', y=z', z=x'); arrays are [z, y, x],
        # so B[z', y', x'] = A[x', z', y'].  Velocity: u'_x = u_z, u'_y = u_x, u'_z = u_y.
        return np.transpose(A, (1, 2, 0))
    Ur = np.stack([rot(U[0]), rot(U[3]), rot(U[1]), rot(U[2]), rot(U[4])])
    for phys in (flow.EULER, flow.NS):
        R = _rhs(U, n, L3, phys, GAS)
        Rr = _rhs(Ur, n, L3, phys, GAS)
        expect = np.stack([rot(R[0]), rot(R[3]), rot(R[1]), rot(R[2]), rot(R[4])])
        assert np.abs(Rr - expect).max() < 1e-10 * np.abs(R).max()


# ------------------------------------------------------ brute force pins
@pytest.mark.parametrize("order", [4, 2])
@pytest.mark.parametrize("physics", [flow.EULER, flow.NS])
def test_vectorized_rhs_matches_pointwise_sync(physics, order):
    n = (10, 10, 10) if physics == flow.EULER else (12, 12, 12)
    U = inputs.smooth_random_state(n, L3, seed=7)
    h = inputs.spacing(n, L3)
    R = flow.rhs_global(U, h, 3, physics, GAS, order)
    rng = np.random.default_rng(0)
    pts = rng.integers(0, n[0], size=(25, 3))
    for x, y, z in pts:
        get = pointwise.block_accessor(U, None, 0, (x, y, z), n, (0, 0, 0))
        r = pointwise.rhs_point(get, h, 3, physics, GAS, order)
        assert np.allclose(r, R[:, z, y, x], rtol=1e-11, atol=1e-11 * np.abs(R).max())


def test_vortex_rhs_is_translation_to_fourth_order():
    # The isentropic vortex translates rigidly: dU/dt = -u_inf . grad U.
    errs = []
    for N in (64, 128, 256):
        n, length = (N, N, 1), (10.0, 10.0, 1.0)
        U = inputs.vortex_state(n, length, 2)
        h = inputs.spacing(n, length)
        R = flow.rhs_global(U, h, 2, flow.EULER, GAS)
        dt = 1e-6
        Up = inputs.vortex_state(n, length, 2, t=dt)
        Um = inputs.vortex_state(n, length, 2, t=-dt)
        dUdt = (Up - Um) / (2 * dt)
        # away from the periodic seam, where the truncated tail jumps
        xs = np.arange(N) * h[0]
        m = np.abs(xs - 5.0) < 4.0
        mask = m[None, :, None] & m[None, None, :]
        errs.append(np.abs(R - dUdt)[:, mask].max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) > 3.7, (errs, orders)


def test_visbal_vortex_is_a_translating_solution():
    # The paper's Gaussian vortex (Sec. 5.1) with uniform density: the Euler
    # RHS equals -U_inf dU/dx (the field moves rigidly), to fourth order.
    errs = []
    for N in (64, 128, 256):
        n = (N, N, 1)
        U = inputs.visbal_vortex_state(n)
        h = inputs.spacing(n, inputs.VISBAL_BOX)
        R = flow.rhs_global(U, h, 2, flow.EULER, GAS)
        dt = 1e-6
        dUdt = (inputs.visbal_vortex_state(n, t=dt) - inputs.visbal_vortex_state(n, t=-dt)) / (2 * dt)
        errs.append(np.abs(R - dUdt).max() / np.abs(dUdt).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) > 3.7 and errs[-1] < 1e-3, (errs, orders)
    # uniform density, divergence-free velocity, pressure from the balance
    U = inputs.visbal_vortex_state((64, 64, 1))
    assert np.all(U[0] == 1.0)
    assert abs(U[1].mean() - 1.0) < 1e-12


# ---------------------------------------------------------- TGV + diag
def test_tgv_initial_invariants():
    n = (16, 16, 16)
    g, M = 1.4, 0.1
    U = inputs.tgv_state(n, mach=M, gamma=g)
    h = inputs.spacing(n, L3)
    V = (2 * math.pi) ** 3
    tot = diagnostics.totals(U, h)
    # mass = V, momentum = 0, energy = V (1/(g (g-1) M^2) + 1/8): the
    # trapezoidal sum is exact for these trigonometric products.
    assert abs(tot[0] - V) < 1e-12 * V
    assert np.abs(tot[1:4]).max() < 1e-12 * V
    assert abs(tot[4] - V * (1 / (g * (g - 1) * M * M) + 1 / 8)) < 1e-12 * tot[4]
    assert abs(diagnostics.kinetic_energy(U) - 0.125) < 1e-14
    # divergence-free initial velocity (CD4 on a single Fourier mode)
    rho = U[0]
    div = sum(flow.cd4(np.pad(U[1 + d] / rho, 2, mode="wrap"), d, h[d])[2:-2, 2:-2, 2:-2]
              for d in range(3))
    assert np.abs(div).max() < 1e-12


def test_tgv_enstrophy_closed_form():
    # eps(0) = 3/8 - 5 g M^2 / 128 for the exact vorticity; CD4 scales every
    # vorticity component by the modified wavenumber k*(1).
    for N in (16, 32):
        n = (N, N, N)
        g, M = 1.4, 0.1
        U = inputs.tgv_state(n, mach=M, gamma=g)
        h = inputs.spacing(n, L3)
        ks = kstar(1, h[0])
        expect = ks ** 2 * (3 / 8 - 5 * g * M * M / 128)
        assert abs(diagnostics.enstrophy(U, h, 3) - expect) < 1e-13


# ----------------------------------------------------------- 2D == 3D
def test_2d_matches_z_invariant_3d():
    n2, n3 = (16, 16, 1), (16, 16, 6)
    length = (10.0, 10.0, 3.0)
    U2 = inputs.vortex_state(n2, length, 2)
    U3 = np.repeat(U2, 6, axis=1)
    for phys in (flow.EULER, flow.NS):
        R2 = flow.rhs_global(U2, inputs.spacing(n2, length), 2, phys, GAS)
        R3 = flow.rhs_global(U3, inputs.spacing(n3, length), 3, phys, GAS)
        assert np.abs(R3 - R2).max() < 1e-12 * max(1.0, np.abs(R2).max())
