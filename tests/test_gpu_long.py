"""GPU parity at the largest delay of the 512^3 Taylor-Green workload and over
a long run.

* SAA with L = 5 (delays 0..4, Alg. 3): k = 4 is the largest delay and the one
  whose AT weights have the largest norm (||W||_1 up to about 1.5e3 for the
  last RK4 stage).  Delays of 4 are injected on face and edge slots.  Every
  stage's right-hand side (Eqs. 8-15 give each stage its own halo weights) is
  checked element by element against the FP64 oracle, and whole RK steps in
  FP64 (<= 1e-12) and FP32 (<= 1e-5 relative L2).  Navier-Stokes blocks of
  32^3, as in the 512^3 workload.
* The 3-D isentropic vortex to T = 1 in FP32 (4 x 4 x 4 blocks, SAA L = 4)
  against the stored FP64 oracle state (tests/golden/make_vortex3d_t1.py):
  relative L2 <= 1e-5.
"""
import math
import os
import sys

import numpy as np
import pytest

from gpu_helpers import announce, need_gpu, pair, rel_l2, rel_max, set_both, to_np
from test_gpu_parity import f32, rhs_tol
from paper_2506_03027_amd import inputs

pytestmark = pytest.mark.gpu

L3 = (2 * math.pi,) * 3
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
OMEGA = 0.3


def tgv_history(n, steps):
    """U^m = TGV + sin(w s) G1 + (1 - cos(w s)) G2 (s = m - last): smooth in
    time but not a polynomial, so every AT weight matters."""
    base = inputs.tgv_state(n, mach=0.1)
    g1 = 0.02 * (inputs.smooth_random_state(n, L3, seed=41) - 1.0)
    g2 = 0.02 * (inputs.smooth_random_state(n, L3, seed=42) - 1.0)
    last = steps[-1]
    return {m: base + math.sin(OMEGA * (m - last)) * g1 + (1.0 - math.cos(OMEGA * (m - last))) * g2
            for m in steps}


def k4_schedule(nb, seed):
    """Delays 0..4 with every slot of block 0 and the faces and edges of
    alternate blocks at the bound 4."""
    rng = np.random.default_rng(seed)
    k = rng.integers(0, 5, size=(nb, 18))
    k[0, :] = 4
    k[1::2, 0:6] = 4
    k[2::2, 6:18] = 4
    return k


def ns_rhs_tol(U, h, precision, wnorm):
    return rhs_tol(U, h, precision, wnorm) * (1.0 + 1.0 / (1600.0 * min(h)))


@pytest.mark.parametrize("rk", ["rk4", "lserk4"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_rhs_every_stage_at_delay_bound_l5(precision, rk):
    need_gpu()
    announce("rhs every stage L=5", precision, rk)
    n = (64, 64, 32)
    o, g = pair(dict(n=n, length=L3, nblk=(2, 2, 1), physics="ns", re=1600.0, mach=0.1, mode="at",
                     algo="saa", L=5, seed=7, rk=rk), precision)
    nstep = 20
    D = g.ring_depth
    hist = tgv_history(n, list(range(nstep - D + 1, nstep + 1)))
    for m, U in sorted(hist.items()):
        set_both(o, g, f32(U) if precision == "f32" else U, step=m)
    k = k4_schedule(g.nblocks, 3)
    g.set_delays(nstep, k[None].astype(np.int8))
    o.set_delays(nstep, k)
    kk = o.delays()
    assert kk.max() == 4 and (kk[:, :18] == 4).sum() >= 18
    for e in range(o.s):
        R = to_np(g.rhs(stage=e))
        ref = o.rhs(o.U, e, kk)
        wn = max(np.abs(o.W[e, j]).sum() for j in range(5))
        tol = ns_rhs_tol(o.U, o.cfg.h, precision, wn)
        err = float(np.abs(R - ref).max())
        print("stage", e, "||W||_1", wn, "max err", err, "tol", tol, flush=True)
        assert err < tol, (e, err, tol)
    g.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_steps_at_delay_bound_l5(precision):
    need_gpu()
    announce("steps L=5", precision)
    n = (64, 32, 32)
    U0 = inputs.tgv_state(n, mach=0.1) + 0.02 * (inputs.smooth_random_state(n, L3, seed=43) - 1.0)
    if precision == "f32":
        U0 = f32(U0)
    dt = inputs.cfl_dt(U0, n, L3, 3, 1.4, 0.05)
    o, g = pair(dict(n=n, length=L3, nblk=(2, 1, 1), physics="ns", re=1600.0, mach=0.1, mode="at",
                     algo="saa", L=5, seed=9, rk="rk4"), precision, dt=dt)
    set_both(o, g, U0)
    nsteps = 12
    # steps 8.. may use k = 4 (guard k <= n - C + 1): inject it there
    first = 8
    ks = np.stack([k4_schedule(g.nblocks, 10 + j) for j in range(nsteps - first)])
    g.set_delays(first, ks.astype(np.int8))
    for j in range(nsteps - first):
        o.set_delays(first + j, ks[j])
    g.step(nsteps)
    o.step(nsteps)
    G = to_np(g.get_state())
    if precision == "f64":
        err = rel_max(G, o.U)
        print("f64 rel max", err)
        assert err < 1e-12, err
    else:
        err = rel_l2(G, o.U)
        print("f32 rel L2", err)
        assert err < 1e-5, err
    g.close()


def test_vortex_fp32_at_t1_against_stored_oracle():
    torch = need_gpu()
    announce("vortex T=1 f32")
    sys.path.insert(0, GOLDEN)
    import make_vortex3d_t1 as mk
    ref = np.load(mk.OUT)
    c = mk.CASE
    dt, steps = mk.time_step()
    _, g = pair(dict(n=c["n"], length=c["length"], nblk=c["nblk"], physics=c["physics"], rk=c["rk"],
                     mode=c["mode"], algo=c["algo"], L=c["L"], seed=c["seed"]), "f32", dt=dt)
    g.set_state(torch.from_numpy(mk.initial_state()))
    g.step(steps)
    G = to_np(g.get_state())
    err = rel_l2(G, ref)
    print("T=1 steps", steps, "FP32 rel L2 vs FP64 oracle", err, "rel Linf", rel_max(G, ref))
    assert np.isfinite(G).all()
    assert err <= 1e-5, err
    g.close()
