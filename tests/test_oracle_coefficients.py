"""Pins of the oracle's coefficient machinery against what the paper prints
and against exact mathematics (no GPU)."""
import random
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import at, rk
from conftest import read_golden


# --------------------------------------------------------------- RK schemes
def test_lserk4_table4_matches_fixture():
    rows = read_golden("lserk4_table4.txt")
    for m, (_, a, b) in enumerate(rows):
        assert rk.LSERK4_A[m] == Fr(a)
        assert rk.LSERK4_B[m] == Fr(b)


def test_lserk4_is_fourth_order_to_printed_digits():
    # App. B Table 4 is printed to 8 digits: all eight order conditions of a
    # fourth-order method hold to the rounding of those digits.
    res = [abs(float(r)) for r in rk.order_condition_residuals(rk.LSERK4)]
    assert max(res) < 5e-8
    assert max(res) > 1e-12        # not exact: the printed digits are rounded


def test_rk4_order_conditions_exact():
    assert all(r == 0 for r in rk.order_condition_residuals(rk.RK4))


def test_lserk2_is_explicit_midpoint():
    a, b, c = rk.butcher(rk.LSERK2)
    assert a == [[0, 0], [Fr(1, 2), 0]]
    assert b == [0, 1]


def test_stage_polynomials_match_exponential():
    for sch, order in ((rk.RK4, 4), (rk.LSERK4, 4), (rk.LSERK2, 2)):
        _, step = rk.stage_polynomials(sch)
        for j in range(order + 1):
            fact = 1
            for i in range(2, j + 1):
                fact *= i
            tol = 0 if sch != rk.LSERK4 else Fr(1, 10 ** 7)
            assert abs(step[j] - Fr(1, fact)) <= tol


def test_nu_first_and_last_coefficients():
    # Sec. 3.1, below Eq. (9): nu_0^e = 1, nu_e^e = prod_{j<=e} B_j,
    # nu_1^e = sum of the Butcher row (the stage abscissa).
    nus = rk.nu(rk.LSERK4)
    _, _, c = rk.butcher(rk.LSERK4)
    prod = Fr(1)
    for e in range(5):
        assert nus[e][0] == 1
        if e >= 1:
            prod *= rk.LSERK4_B[e - 1]
            assert nus[e][e] == prod
            assert nus[e][1] == c[e]
    assert [list(map(Fr, r))[:e + 1] for e, r in enumerate(rk.nu(rk.RK4))] == [
        [1], [1, Fr(1, 2)], [1, Fr(1, 2), Fr(1, 4)], [1, 1, Fr(1, 2), Fr(1, 4)]]


def _ode_error(sch, nsteps, T=2.0, w=6.0):
    # y' = -y + w cos(w t), y(0) = 1; exact solution in closed form.
    A = w / (1 + w * w)

    def exact(t):
        return A * (np.cos(w * t) + w * np.sin(w * t)) + (1 - A) * np.exp(-t)

    a, b, c = rk.butcher(sch)
    a = [[float(x) for x in r] for r in a]
    b = [float(x) for x in b]
    c = [float(x) for x in c]
    dt, y, t = T / nsteps, 1.0, 0.0
    for _ in range(nsteps):
        ks = []
        for i in range(len(b)):
            yi = y + dt * sum(a[i][j] * ks[j] for j in range(i))
            ks.append(-yi + w * np.cos(w * (t + c[i] * dt)))
        y += dt * sum(bi * ki for bi, ki in zip(b, ks))
        t += dt
    return abs(y - exact(T))


def test_rk4_observed_temporal_order_on_ode():
    errs = [_ode_error(rk.RK4, n) for n in (10, 20, 40, 80)]
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert min(orders) > 3.9, orders


def test_lserk4_temporal_order_until_coefficient_floor():
    # Fourth order until the error meets the floor set by the 8 printed
    # digits of Table 4 (first order condition off by ~5e-8 per unit time).
    errs = [_ode_error(rk.LSERK4, n) for n in (10, 20, 40, 80)]
    assert errs[0] / errs[1] > 2 ** 3.8
    assert max(errs[1:]) < 1e-6


# ----------------------------------------------------------- AT boundary
def _poly_rows(rows, k, ncoef):
    out = []
    for r in rows:
        num, den = int(r[1]), int(r[2])
        coefs = [int(x) for x in r[3:3 + ncoef]]
        val = sum(c * Fr(k) ** (ncoef - 1 - i) for i, c in enumerate(coefs))
        out.append(Fr(num, den) * val)
    return out


@pytest.mark.parametrize("k", range(0, 9))
def test_at4_extrapolation_eq15(k):
    printed = _poly_rows(read_golden("at4_extrapolation_eq15.txt"), k, 5)
    derived = at.boundary_coefficients(k, at.AT4_C)
    assert derived == at.lagrange_extrapolation(k, at.AT4_C)
    # rows 0, 2, 3, 4 exactly as printed
    for l in (0, 2, 3, 4):
        assert derived[l] == printed[l]
    # row 1 is printed with 25 k^2; the consistent value has 26 k^2
    assert derived[1] == printed[1] - Fr(k * k, 6)
    assert sum(derived) == 1
    assert sum(printed) == 1 + Fr(k * k, 6)


@pytest.mark.parametrize("k", range(0, 9))
def test_at2_extrapolation_eq14(k):
    printed = _poly_rows(read_golden("at2_extrapolation_eq14.txt"), k, 3)
    assert at.boundary_coefficients(k, at.AT2_C) == printed
    assert at.lagrange_extrapolation(k, at.AT2_C) == printed


def test_at4_boundary_k1_values():
    assert at.boundary_coefficients(1, 5) == [5, -10, 10, -5, 1]


@pytest.mark.parametrize("k", range(0, 6))
def test_extrapolation_exact_for_polynomials(k):
    # Degree <= C-1 polynomials in time are extrapolated exactly; degree C is not.
    w = at.lagrange_extrapolation(k, 5)
    for deg in range(5):
        val = sum(wl * Fr(-(k + l)) ** deg for l, wl in enumerate(w))
        assert val == (1 if deg == 0 else 0)
    val5 = sum(wl * Fr(-(k + l)) ** 5 for l, wl in enumerate(w))
    assert (val5 != 0) == (k > 0)     # k = 0 reads the node itself


# --------------------------------------------------------- buffer updates
@pytest.mark.parametrize("k", range(0, 7))
def test_lserk2_at2_buffer_derivative_appC(k):
    printed = _poly_rows(read_golden("lserk2_at2_buffer_appC.txt"), k, 2)
    assert at.buffer_derivative(k, at.AT2_C, [1]) == printed


def _table5(e, l, k, nuv):
    rows = [r for r in read_golden("lserk4_at4_buffer_table5.txt")
            if int(r[0]) == e and int(r[1]) == l]
    assert len(rows) == 1
    r = [int(x) for x in rows[0]]
    num, den = r[2], r[3]
    coef = r[4:]
    nus = [Fr(1)] + list(nuv) + [Fr(0)] * (3 - len(nuv))
    val = Fr(0)
    for p in range(4):                      # k^3, k^2, k^1, k^0
        c = sum(coef[4 * p + j] * nus[j] for j in range(4))
        val += c * Fr(k) ** (3 - p)
    return Fr(num, den) * val


@pytest.mark.parametrize("e", range(4))
def test_lserk4_at4_table5_for_any_nu(e):
    # Table 5 holds for arbitrary nu (the constraints are linear in nu):
    # check the scheme's own nu and random rationals.
    rnd = random.Random(e)
    nu_sets = [rk.nu(rk.LSERK4)[e][1:e + 1]]
    for _ in range(3):
        nu_sets.append([Fr(rnd.randint(-50, 50), rnd.randint(1, 40)) for _ in range(e)])
    for nuv in nu_sets:
        for k in range(0, 6):
            derived = at.buffer_derivative(k, at.AT4_C, [1] + list(nuv))
            for l in range(5):
                assert derived[l] == _table5(e, l, k, nuv), (e, k, l)


# -------------------------------------------------------- stage halo W
@pytest.mark.parametrize("sch", [rk.RK4, rk.LSERK4, rk.LSERK2])
def test_halo_weights_literal_equals_closed_form(sch):
    C = at.AT2_C if sch == rk.LSERK2 else at.AT4_C
    for k in range(0, 6):
        assert at.halo_weights_literal(sch, k, C) == at.halo_weights_closed(sch, k, C)


@pytest.mark.parametrize("sch", [rk.RK4, rk.LSERK4])
def test_halo_weights_identities(sch):
    for k in range(0, 6):
        W = at.halo_weights_closed(sch, k, 5)
        for w in W:
            assert sum(w) == 1
        assert W[0] == at.lagrange_extrapolation(k, 5)
    assert at.halo_weights_closed(sch, 0, 5)[0] == [1, 0, 0, 0, 0]


@pytest.mark.parametrize("sch", [rk.RK4, rk.LSERK4])
def test_halo_weights_reproduce_stage_polynomial(sch):
    # On data that is a polynomial of degree <= C-1 in time, the stage-e halo
    # value equals sum_j nu_j^e p^{(j)}(t_n): the stage value the RK scheme
    # would produce if the buffer were advanced with the exact derivatives.
    rnd = random.Random(3)
    nus = rk.nu(sch)
    for k in range(0, 5):
        W = at.halo_weights_closed(sch, k, 5)
        coeffs = [Fr(rnd.randint(-9, 9), rnd.randint(1, 5)) for _ in range(5)]

        def p(t, j=0):
            tot = Fr(0)
            for i, c in enumerate(coeffs):
                if i >= j:
                    f = 1
                    for r in range(i - j + 1, i + 1):
                        f *= r
                    tot += c * f * Fr(t) ** (i - j)
            return tot
        samples = [p(-(k + l)) for l in range(5)]
        for e, w in enumerate(W):
            lhs = sum(wl * s for wl, s in zip(w, samples))
            rhs = sum(nj * p(0, j) for j, nj in enumerate(nus[e]) if j < 5)
            assert lhs == rhs


def test_halo_weight_norms():
    # ||W||_1 is the factor by which rounding noise in the delayed levels is
    # amplified; record the values for RK4 (these set the FP32 floor).
    n0 = [float(sum(abs(x) for x in w)) for w in at.halo_weights_closed(rk.RK4, 0, 5)]
    n3 = [float(sum(abs(x) for x in w)) for w in at.halo_weights_closed(rk.RK4, 3, 5)]
    assert np.allclose(n0, [1, 19 / 3, 13, 33])
    assert np.allclose(n3, [351, 1513 / 3, 553, 775])
