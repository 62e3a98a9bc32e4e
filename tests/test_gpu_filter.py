"""GPU parity of the tenth-order Pade filter (Sec. 2; alpha_f = 0.499 as in
Sec. 5.2) against the FP64 oracle (oracle/filter.py).

* One application to a state with grid-scale content (synchronous halos):
  3-D with uneven blocks, 2-D, FP64 and FP32.
* Filtered Taylor-Green steps, SA, AT and AS, RK4 and LSERK4, through the
  synchronous start and into delayed steps with delays up to 4 (L = 5): the
  filter halos then come from the delayed levels (AT: extrapolated to the
  new level).  FP64 <= 1e-12 relative max, FP32 <= 1e-5 relative L2.
* Graph-captured filtered steps give the same bits as eager ones.

FP32 tolerance of one application: the kernel works in FP64 on FP32 inputs
and rounds each pass's output once; the filter damps every mode (|T| <= 1),
so three passes leave a few ulp, bounded here by 4e-7 relative to the
largest value (about 7 ulp).
"""
import math

import numpy as np
import pytest

from gpu_helpers import announce, need_gpu, pair, rel_l2, rel_max, set_both, to_np
from test_gpu_parity import f32
from paper_2506_03027_amd import inputs

pytestmark = pytest.mark.gpu

L3 = (2 * math.pi,) * 3


def rough_state(n, seed, ndim=3):
    """Smooth field plus grid-scale noise, so the filter has work to do."""
    U = inputs.smooth_random_state(n, L3, seed=seed, ndim=ndim)
    rng = np.random.default_rng(seed + 100)
    return U + 1e-3 * rng.standard_normal(U.shape) * np.abs(U).mean(axis=(1, 2, 3), keepdims=True)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("alpha", [0.499, 0.3])
@pytest.mark.parametrize("case", ["3d_uneven", "3d_blocks32", "2d"])
def test_filter_state_matches_oracle(case, alpha, precision):
    # uneven blocks take the general kernel; blocks of one side 8, 16 or 32
    # along an axis the register-only one (32^3 blocks here, 16 in 2-D x)
    need_gpu()
    announce("filter state", case, alpha, precision)
    if case == "3d_uneven":
        n = (32, 32, 24)
        spec = dict(n=n, length=L3, nblk=(2, 2, 2), split=([13, 19], [16, 16], [10, 14]))
    elif case == "3d_blocks32":
        n = (64, 64, 32)
        spec = dict(n=n, length=L3, nblk=(2, 2, 1))
    else:
        n = (32, 24, 1)
        spec = dict(n=n, length=L3, ndim=2, nblk=(2, 2, 1))
    spec.update(physics="ns", filter_alpha=alpha)
    o, g = pair(spec, precision)
    U = rough_state(n, 5, ndim=spec.get("ndim", 3))
    if precision == "f32":
        U = f32(U)
    set_both(o, g, U)
    g.filter_state()
    got = to_np(g.get_state())
    want = o.filter_state(U)
    assert np.abs(want - U).max() > 1e-6 * np.abs(U).max()   # the filter changed the field
    err = rel_max(got, want)
    assert err < (1e-12 if precision == "f64" else 4e-7), err
    g.close()


def tgv_case(mode, rk, n=(32, 32, 32)):
    """Taylor-Green field with a little grid-scale noise (1e-4 of each
    variable's mean magnitude), which the filter removes."""
    U0 = inputs.tgv_state(n, mach=0.1)
    dt = inputs.cfl_dt(U0, n, L3, 3, 1.4, 0.1)
    rng = np.random.default_rng(21)
    U0 = U0 + 1e-4 * rng.standard_normal(U0.shape) * np.abs(U0).mean(axis=(1, 2, 3), keepdims=True)
    spec = dict(n=n, length=L3, nblk=(2, 2, 2), physics="ns", re=1600.0, mach=0.1, rk=rk, mode=mode,
                algo="saa", L=5 if mode != "sa" else 1, seed=13, filter_alpha=0.499)
    return U0, dt, spec


@pytest.mark.parametrize("mode, rk, precision", [
    ("sa", "rk4", "f64"), ("at", "rk4", "f64"), ("as", "rk4", "f64"), ("at", "lserk4", "f64"),
    ("at", "lserk2", "f64"), ("sa", "rk4", "f32"), ("at", "rk4", "f32"),
])
def test_filtered_steps_match_oracle(mode, rk, precision):
    need_gpu()
    announce("filtered steps", mode, rk, precision)
    U0, dt, spec = tgv_case(mode, rk)
    o, g = pair(spec, precision, dt=dt)
    U = f32(U0) if precision == "f32" else U0
    set_both(o, g, U)
    steps = 11                      # C synchronous (5, or 3 for LSERK2), then delayed steps
    g.set_graphs(False)
    g.step(steps)
    o.step(steps)
    got = to_np(g.get_state())
    if mode != "sa":
        C = 3 if rk == "lserk2" else 5
        k = np.stack([o.delays(m) for m in range(C, steps)])
        assert k.max() == 4
    assert np.abs(o.U - U).max() > 0
    if precision == "f64":
        err = rel_max(got, o.U)
        assert err < 1e-12, err
    else:
        err = rel_l2(got, o.U)
        assert err < 1e-5, err
    g.close()


def test_filtered_graph_steps_equal_eager():
    need_gpu()
    announce("filtered graph vs eager")
    U0, dt, spec = tgv_case("at", "rk4", n=(40, 32, 24))
    res = []
    for graphs in (False, True):
        _, g = pair(spec, "f32", dt=dt)
        import torch
        g.set_state(torch.from_numpy(f32(U0)))
        g.set_graphs(graphs)
        g.step(12)
        res.append(to_np(g.get_state()))
        g.close()
    assert np.array_equal(res[0], res[1])


@pytest.mark.parametrize("precision, n, mode", [
    ("f32", (64, 64, 64), "at"),    # blocks of 32^3
    ("f32", (32, 32, 32), "as"),    # 16^3
    ("f32", (16, 16, 16), "at"),    # 8^3
    ("f64", (32, 32, 32), "at"),    # 16^3 in double precision
])
def test_fused_filter_equals_per_axis_passes(precision, n, mode):
    """Steps with delayed halos filter each block in one launch (three passes
    on an LDS copy, then the ring write); the per-axis passes and the ring
    fill must give the same bits, eager and graph-captured, over several
    delayed steps (so the ring layers it wrote are read back too)."""
    torch = need_gpu()
    announce("fused filter vs per-axis passes", precision, n, mode)
    U0, dt, spec = tgv_case(mode, "rk4", n=n)
    U = f32(U0) if precision == "f32" else U0
    res = {}
    for fused in (False, True):
        for graphs in (False, True):
            _, g = pair(spec, precision, dt=dt)
            g.set_filter_fusion(fused)
            g.set_graphs(graphs)
            g.set_state(torch.from_numpy(U))
            g.step(9)                # 5 synchronous steps, then 4 with delays up to 4
            res[(fused, graphs)] = to_np(g.get_state())
            g.close()
    ref = res[(False, False)]
    assert np.isfinite(ref).all()
    for key, got in res.items():
        assert np.array_equal(got, ref), key
