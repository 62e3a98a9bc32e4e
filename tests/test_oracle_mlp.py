"""Pins of the FP64 learned-halo reference (no GPU)."""
import numpy as np
import pytest

from bounds import bf16_forward_bound
from oracle import mlp


def test_layout_size():
    assert mlp.NPARAM == 9360


def test_gradient_matches_central_differences():
    th = mlp.init(3)
    rng = np.random.default_rng(0)
    X = rng.standard_normal((7, 64))
    Y = rng.standard_normal((7, 8))
    _, g = mlp.loss_and_grad(th, X, Y)
    eps = 1e-6
    for i in list(range(0, 9360, 331)) + [9344, 9359]:
        e = np.zeros_like(th)
        e[i] = eps
        num = (mlp.loss_and_grad(th + e, X, Y)[0] - mlp.loss_and_grad(th - e, X, Y)[0]) / (2 * eps)
        assert abs(num - g[i]) < 1e-7 + 1e-6 * abs(num), i


def test_unused_outputs_carry_no_gradient():
    th = mlp.init(1)
    X = np.random.default_rng(1).standard_normal((4, 64))
    _, g = mlp.loss_and_grad(th, X, np.zeros((4, 8)))
    p = mlp.unpack(g)
    assert np.all(p["W3"][5:] == 0) and np.all(p["b3"][5:] == 0)


def test_bf16_rounding():
    # round to nearest, ties to even, on the 8-bit significand
    assert mlp.bf16(1.0) == 1.0
    assert mlp.bf16(1.0 + 2 ** -8) == 1.0                 # tie -> even (down)
    assert mlp.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6   # tie -> even (up)
    assert mlp.bf16(1.0 + 2 ** -8 + 2 ** -12) == 1.0 + 2 ** -7
    assert mlp.bf16(-3.14159) == -3.140625
    x = np.random.default_rng(2).standard_normal(1000)
    assert np.all(np.abs(mlp.bf16(x) - x) <= 2 ** -8 * np.abs(x))     # half an ulp


def test_correction_fallback_rule():
    d, ok = mlp.correct(np.array([0.3, 0.4, 0, 0, 0, 9, 9]), np.ones(5) * 2, tau=0.6)
    assert ok and np.allclose(d, [0.6, 0.8, 0, 0, 0])
    d, ok = mlp.correct(np.array([0.3, 0.4, 0, 0, 0]), np.ones(5), tau=0.49)
    assert not ok and np.all(d == 0)


def test_features_of_constant_history_are_zero_but_delay():
    lv = [np.ones((5, 3)) * 2.5 for _ in range(4)]
    f = mlp.face_features(lv, 2, 4, 0, np.ones(5))
    assert np.all(f[:60] == 0) and f[60] == pytest.approx(2 / 3) and np.all(f[61:] == 0)


def test_bf16_emulation_within_derived_bound_of_plain_forward():
    # The learned-halo oracle of the corrected solver evaluates the network on
    # BF16-rounded operands (the GPU's arithmetic); pin that path to the plain
    # FP64 forward pass by the rounding bound of bounds.bf16_forward_bound.
    th = mlp.init(4)
    th[64 * 64:64 * 64 + 64] = 0.05
    X = np.random.default_rng(3).standard_normal((500, 64))
    plain, _ = mlp.forward(th, X)
    emul, _ = mlp.forward(th, X, round_bf16=True)
    bound = bf16_forward_bound(th, X)
    err = np.abs(emul - plain)
    assert np.all(err <= bound)
    # the worst case is far from typical: errors sit well inside the bound,
    # and the bound stays below the size of the outputs it bounds
    assert np.median(err / bound) < 0.05
    assert bound.max() < np.abs(plain).max()
