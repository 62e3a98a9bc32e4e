"""GPU parity of the Navier-Stokes path (viscous terms, depth-4 faces and
2x2 edge halos) against the FP64 oracle, through the C ABI."""
import math

import numpy as np
import pytest

from gpu_helpers import announce, need_gpu, pair, rel_l2, rel_max, set_both, to_np
from test_gpu_parity import BOX, f32, rhs_tol, smooth_history
from paper_2506_03027_amd import inputs

pytestmark = pytest.mark.gpu

NSKW = dict(physics="ns", re=100.0, mach=0.3)
L3 = (2 * math.pi,) * 3


def ns_tol(U, h, precision, re, wnorm=1.0):
    # the viscous flux adds gradient-sized terms / Re: use the inviscid
    # bound on a scale that covers them (x 1 + 1/(Re h)).
    return rhs_tol(U, h, precision, wnorm) * (1.0 + 1.0 / (re * min(h)))


@pytest.mark.parametrize("rk", ["rk4", "lserk2"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("split", [None, ([10, 8, 6], [12, 8], [9, 7])])
def test_ns_rhs_synchronous(precision, split, rk):
    need_gpu()
    announce("ns rhs sync", precision, split)
    n = (24, 20, 16)
    nblk = (3, 2, 2) if split else (2, 2, 2)
    o, g = pair(dict(n=n, length=BOX, nblk=nblk, split=split, rk=rk, **NSKW), precision)
    U = inputs.smooth_random_state(n, BOX, seed=8)
    if precision == "f32":
        U = f32(U)
    set_both(o, g, U)
    R = to_np(g.rhs())
    ref = o.rhs(U)
    tol = ns_tol(U, o.cfg.h, precision, 100.0)
    assert np.abs(R - ref).max() < tol, (np.abs(R - ref).max(), tol)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("mode, algo, nstep, rk", [("at", "saa", 13, "rk4"), ("at", "caa", 16, "rk4"),
                                                   ("as", "saa", 13, "rk4"), ("at", "saa", 13, "lserk2")])
def test_ns_rhs_delayed_halos(precision, mode, algo, nstep, rk):
    need_gpu()
    announce("ns rhs delayed", precision, mode, algo, rk)
    n = (32, 24, 20)
    split = ([12, 12, 8], [14, 10], [10, 10])
    o, g = pair(dict(n=n, length=BOX, nblk=(3, 2, 2), split=split, mode=mode, algo=algo, L=4,
                     seed=23, rk=rk, **NSKW), precision)
    D = g.ring_depth
    hist = smooth_history(n, list(range(nstep - D + 1, nstep + 1)))
    for m, U in sorted(hist.items()):
        set_both(o, g, f32(U) if precision == "f32" else U, step=m)
    k = o.delays()
    assert k is not None and k[:, :18].max() == 3
    R = to_np(g.rhs())
    ref = o.rhs(o.U, 0, k)
    wn = max(np.abs(o.W[0, kk]).sum() for kk in range(4))
    tol = ns_tol(o.U, o.cfg.h, precision, 100.0, wn)
    assert np.abs(R - ref).max() < tol, (np.abs(R - ref).max(), tol)


@pytest.mark.parametrize("rk", ["rk4", "lserk4", "lserk2"])
@pytest.mark.parametrize("mode, algo, L", [("sa", "caa", 1), ("at", "caa", 4), ("at", "saa", 3),
                                           ("as", "saa", 2)])
def test_ns_steps_fp64_match_oracle(rk, mode, algo, L):
    need_gpu()
    announce("ns steps f64", rk, mode, algo, L)
    n = (20, 16, 16)
    U0 = inputs.smooth_random_state(n, L3, seed=12, amp=0.05)
    dt = inputs.cfl_dt(U0, n, L3, 3, 1.4, 0.05)
    o, g = pair(dict(n=n, length=L3, nblk=(2, 2, 2), rk=rk, mode=mode, algo=algo, L=L, seed=4,
                     **NSKW), "f64", dt=dt)
    set_both(o, g, U0)
    nsteps = 9
    g.step(nsteps)
    o.step(nsteps)
    err = rel_max(to_np(g.get_state()), o.U)
    assert err < 1e-12, err


def test_ns_2d_steps_fp64():
    need_gpu()
    announce("ns 2d")
    n = (24, 20, 1)
    box = (6.0, 5.0, 1.0)
    U0 = inputs.smooth_random_state(n, box, seed=3, ndim=2)
    dt = inputs.cfl_dt(U0, n, box, 2, 1.4, 0.05)
    o, g = pair(dict(n=n, length=box, ndim=2, nblk=(3, 2, 1), mode="at", algo="saa", L=3, seed=2,
                     **NSKW), "f64", dt=dt)
    set_both(o, g, U0)
    g.step(8)
    o.step(8)
    assert rel_max(to_np(g.get_state()), o.U) < 1e-12


@pytest.mark.parametrize("mode, algo, L", [("sa", "caa", 1), ("at", "saa", 4)])
def test_tgv_fp32_against_fp64_oracle(mode, algo, L):
    need_gpu()
    announce("tgv f32", mode, algo, L)
    n = (32, 32, 32)
    U0 = inputs.tgv_state(n, mach=0.1)
    dt = inputs.cfl_dt(U0, n, L3, 3, 1.4, 0.02)
    o, g = pair(dict(n=n, length=L3, nblk=(2, 2, 4), mode=mode, algo=algo, L=L, seed=6,
                     physics="ns", re=1600.0, mach=0.1), "f32", dt=dt)
    set_both(o, g, U0)
    g.step(12)
    o.step(12)
    err = rel_l2(to_np(g.get_state()), o.U)
    print("tgv fp32 rel L2", mode, err)
    assert err < 1e-5, err
    d, ok = g.reduce()
    assert ok


def test_ns_sa_decomposition_bitwise():
    need_gpu()
    announce("ns bitwise")
    n = (32, 32, 16)
    U0 = inputs.smooth_random_state(n, L3, seed=1)
    dt = inputs.cfl_dt(U0, n, L3, 3, 1.4, 0.1)
    import torch
    outs = []
    for nblk in ((1, 1, 1), (2, 4, 2), (2, 4, 2)):
        _, g = pair(dict(n=n, length=L3, nblk=nblk, **NSKW), "f32", dt=dt)
        g.set_state(torch.from_numpy(U0))
        g.step(4)
        outs.append(to_np(g.get_state()))
        g.close()
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[1], outs[2])
