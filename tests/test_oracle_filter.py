"""Pins of the oracle's tenth-order Pade filter (Sec. 2; Sec. 5.2: alpha_f =
0.499) and of its block-local, delay-tolerant application."""
from fractions import Fraction as Fr
from math import comb

import numpy as np
import pytest

from oracle import filter as filt
from paper_2506_03027_amd import inputs
from oracle import flow
from oracle import solver as sv

ALPHAS = [Fr(0), Fr(3, 10), 0.499, Fr(1, 2)]


def test_coefficients_at_zero_are_the_binomial_filter():
    # alpha = 0: the explicit filter of maximal order has T(w) = 1 - sin^10(w/2)
    # = 1 - ((1 - cos w)/2)^5; expanding the power of (1 - cos w) gives
    # a_0 = 1 - C(10,5)/2^10 and a_m = -2 (-1)^m C(10,5-m)/2^10.
    a = filt.coefficients(Fr(0))
    assert a[0] == 1 - Fr(comb(10, 5), 1024)
    for m in range(1, 6):
        assert a[m] == Fr(-2 * (-1) ** m * comb(10, 5 - m), 1024)


def test_coefficients_at_one_half_are_the_identity():
    # alpha = 1/2: numerator 1 + cos w equals the denominator, T = 1
    assert filt.coefficients(Fr(1, 2)) == [1, 1, 0, 0, 0, 0]


def test_coefficients_are_affine_in_alpha():
    # the conditions are linear with right-hand sides affine in alpha, so
    # the two pinned ends fix every alpha
    a0, ah = filt.coefficients(Fr(0)), filt.coefficients(Fr(1, 2))
    for al in (Fr(499, 1000), Fr(-49, 100), Fr(0.499)):
        a = filt.coefficients(al)
        assert a == [x + 2 * al * (y - x) for x, y in zip(a0, ah)]


@pytest.mark.parametrize("alpha", [Fr(0), Fr(3, 10), Fr(499, 1000)])
def test_transfer_function_kills_odd_even_and_is_tenth_order(alpha):
    a = filt.coefficients(alpha)
    # T(pi) = 0 and T(0) = 1 exactly
    assert sum(x * (-1) ** m for m, x in enumerate(a)) == 0
    assert sum(a) == 1 + 2 * alpha
    # with the two pinned ends, N(w) = (1 - 2 alpha) (1 - sin^10(w/2))
    # + 2 alpha (1 + cos w), hence 1 - T(w) = (1 - 2 alpha) sin^10(w/2) /
    # (1 + 2 alpha cos w): tenth order, and monotone damping
    w = np.linspace(0.5, np.pi, 40)
    al = float(alpha)
    want = (1 - 2 * al) * np.sin(w / 2) ** 10 / (1 + 2 * al * np.cos(w))
    got = 1.0 - filt.transfer(w, alpha)
    assert np.all(np.abs(got - want) < 1e-9 * want + 1e-13)
    if al < 0.4:
        # 1 - T(w) ~ c w^10: halving w divides it by 2^10
        e = 1.0 - filt.transfer(np.array([0.2, 0.1]), alpha)
        assert abs(e[0] / e[1] / 1024.0 - 1.0) < 0.02


@pytest.mark.parametrize("alpha", [0.0, 0.3, 0.499])
def test_periodic_filter_multiplies_fourier_modes_by_T(alpha):
    n = 64
    x = np.arange(n)
    for kappa in (1, 5, 17, 31, 32):
        w = 2 * np.pi * kappa / n
        f = np.cos(w * x + 0.3)
        g = filt.filter_periodic_lines(f, alpha)
        assert np.max(np.abs(g - filt.transfer(w, alpha) * f)) < 1e-12 / max(1e-3, 1 - 2 * alpha)


@pytest.mark.parametrize("alpha", [0.0, 0.3, 0.499])
def test_block_filter_exact_on_degree_nine(alpha):
    rng = np.random.default_rng(3)
    n = 12
    t = np.linspace(-1.0, 1.0, n + 2 * filt.HALO)
    c = rng.standard_normal(10)
    f = np.polyval(c, t)
    g = filt.filter_block_lines(f, alpha)
    assert np.max(np.abs(g - f[filt.HALO:-filt.HALO])) < 1e-11
    # degree ten is not reproduced: the order is exactly ten
    f10 = np.polyval(np.concatenate([[50.0], c]), t)
    g10 = filt.filter_block_lines(f10, alpha)
    assert np.max(np.abs(g10 - f10[filt.HALO:-filt.HALO])) > 1e-9


@pytest.mark.parametrize("alpha", [0.3, 0.499])
def test_block_filter_equals_periodic_far_from_faces(alpha):
    rng = np.random.default_rng(4)
    n = 1200
    f = rng.standard_normal(n)
    per = filt.filter_periodic_lines(f, alpha)
    lo, m = 50, 1100               # block [lo, lo+m) of the periodic line
    ext = f[lo - filt.HALO:lo + m + filt.HALO]
    blk = filt.filter_block_lines(ext, alpha)
    al = alpha
    r = abs((-1 + np.sqrt(1 - 4 * al * al)) / (2 * al))
    mid = slice(m // 2 - 20, m // 2 + 20)
    assert np.max(np.abs(blk[mid] - per[lo:lo + m][mid])) < 50 * r ** (m // 2 - 20) + 1e-12
    # and they differ next to the faces (the closure is a real change)
    assert abs(blk[0] - per[lo]) > 1e-6


def test_block_filter_removes_odd_even_inside():
    n = 400
    f = (-1.0) ** np.arange(n + 2 * filt.HALO)
    g = filt.filter_block_lines(f, 0.3)
    assert np.max(np.abs(g[40:-40])) < 1e-12


def test_next_level_weights_exact_in_time():
    # the C levels of a time polynomial of degree C-1 extrapolate to n+1 exactly
    C = 5
    for k in range(5):
        w = filt.next_level_weights(k, C)
        assert sum(w) == 1
        for deg in range(C):
            p = lambda t: (t + Fr(1, 3)) ** deg
            assert sum(w[l] * p(-(k + l)) for l in range(C)) == p(1)


def _oracle(nblk, mode="sa", alpha=0.499, n=(20, 20, 20), ndim=3, L=1, algo="caa"):
    cfg = sv.Config(n, (2 * np.pi,) * 3, ndim=ndim, nblk=nblk, physics=flow.NS, rk="rk4", mode=mode,
                    algo=algo, L=L, dt=1e-3, filter_alpha=alpha)
    return sv.Oracle(cfg)


def test_three_passes_act_one_axis_each():
    # f(x) g(y) h(z): each pass filters one factor with the 1-D block filter
    # of the periodic line split like the blocks
    n = (20, 20, 20)
    o = _oracle((2, 2, 2), n=n)
    rng = np.random.default_rng(5)
    fs = [rng.standard_normal(n[d]) for d in range(3)]
    U = np.einsum("z,y,x->zyx", fs[2], fs[1], fs[0])[None].repeat(5, axis=0)
    V = o.filter_state(U)

    def line(f):
        out = np.empty_like(f)
        for b0 in (0, 10):
            idx = (np.arange(b0 - filt.HALO, b0 + 10 + filt.HALO)) % 20
            out[b0:b0 + 10] = filt.filter_block_lines(f[idx], 0.499)
        return out
    want = np.einsum("z,y,x->zyx", line(fs[2]), line(fs[1]), line(fs[0]))
    assert np.max(np.abs(V[0] - want)) < 1e-12 * np.max(np.abs(want))


def test_identity_filter_leaves_steps_unchanged():
    # alpha = 1/2 is the identity: filtered and unfiltered steps agree
    n = (16, 16, 16)
    U0 = inputs.tgv_state(n, mach=0.1)
    res = []
    for a in (0.5, None):
        cfg = sv.Config(n, (2 * np.pi,) * 3, ndim=3, nblk=(2, 2, 2), physics=flow.NS, rk="rk4", mode="at",
                        algo="saa", L=3, seed=2, dt=2e-3, filter_alpha=a)
        o = sv.Oracle(cfg)
        o.set_state(U0)
        o.step(8)
        res.append(o.U)
    assert np.max(np.abs(res[0] - res[1])) < 1e-13 * np.max(np.abs(res[1]))


def test_at_filter_halo_is_the_next_level_of_a_time_polynomial():
    # history levels U^m = A + m B + m^2 Q + m^4 R (degree 4 <= C-1): the AT
    # halo at level n+1 is exact, so one AT pass over V = U^{n+1} equals the
    # synchronous pass over V (whose halo is V itself), for each axis
    n = (20, 20, 20)
    o = _oracle((2, 2, 2), mode="at", L=4, algo="saa")
    rng = np.random.default_rng(6)
    A, B, Q, R = (rng.standard_normal((5,) + n[::-1]) for _ in range(4))
    lev = lambda m: A + m * B + m * m * Q + m ** 4 * R * 1e-3
    step = 9
    for m in range(step - 8, step + 1):
        o.history[m] = lev(m)
    o.n = step
    k = o.delays(step)
    assert k is not None and k.max() > 0
    V = lev(step + 1)
    for d in range(3):
        got = o._filter_pass(V, d, k)
        want = o._filter_pass(V, d, None)
        assert np.max(np.abs(got - want)) < 1e-9 * np.max(np.abs(want))
    # a history one level behind (levels U^{m-1} stored as U^m) is visibly
    # different: the test sees the level the halo is extrapolated to
    for m in range(step - 8, step + 1):
        o.history[m] = lev(m - 1)
    for d in range(3):
        bad = o._filter_pass(V, d, k)
        assert np.max(np.abs(bad - o._filter_pass(V, d, None))) > 1e-6 * np.max(np.abs(V))
