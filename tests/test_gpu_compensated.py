"""Compensated classical RK4 steps (atns_set_compensation): the last stage
adds U^n to the step's increments with Knuth's TwoSum and carries the
rounding error to the next step.

* The 3-D vortex to T = 1 in FP32 (4 x 4 x 4 blocks, SAA L = 4, 886 steps)
  against the stored FP64 oracle state: the compensated run must be closer
  than the plain FP32 run, which sits at 6.8e-6.
* FP64 steps with compensation still match the oracle to 1e-12.
* Graph-captured compensated steps equal eager ones bit for bit, and the
  carried error is cleared when a state is set.
"""
import math
import os
import sys

import numpy as np
import pytest

from gpu_helpers import announce, need_gpu, pair, rel_l2, rel_max, set_both, to_np
from paper_2506_03027_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
L3 = (2 * math.pi,) * 3


def test_compensated_vortex_fp32_at_t1_against_stored_oracle():
    torch = need_gpu()
    announce("compensated vortex T=1 f32")
    sys.path.insert(0, GOLDEN)
    import make_vortex3d_t1 as mk
    ref = np.load(mk.OUT)
    c = mk.CASE
    dt, steps = mk.time_step()
    errs = {}
    for comp in (False, True):
        _, g = pair(dict(n=c["n"], length=c["length"], nblk=c["nblk"], physics=c["physics"], rk=c["rk"],
                         mode=c["mode"], algo=c["algo"], L=c["L"], seed=c["seed"]), "f32", dt=dt)
        g.set_compensation(comp)
        g.set_state(torch.from_numpy(mk.initial_state()))
        g.step(steps)
        G = to_np(g.get_state())
        errs[comp] = rel_l2(G, ref)
        assert np.isfinite(G).all()
        g.close()
    print("T=1 FP32 rel L2 vs FP64 oracle: plain %.3e, compensated %.3e" % (errs[False], errs[True]))
    assert errs[True] <= 1e-5
    assert errs[True] < 0.5 * errs[False]


@pytest.mark.parametrize("physics", ["euler", "ns"])
def test_compensated_fp64_steps_match_oracle(physics):
    torch = need_gpu()
    announce("compensated f64 steps", physics)
    n = (32, 24, 20)
    box = L3 if physics == "ns" else (10.0, 10.0, 10.0)
    U0 = inputs.smooth_random_state(n, box, seed=8)
    dt = inputs.cfl_dt(U0, n, box, 3, 1.4, 0.05)
    o, g = pair(dict(n=n, length=box, nblk=(2, 2, 2), physics=physics, mode="at", algo="saa", L=4, seed=5),
                "f64", dt=dt)
    g.set_compensation(True)
    set_both(o, g, U0)
    g.step(12)
    o.step(12)
    err = rel_max(to_np(g.get_state()), o.U)
    assert err < 1e-12, err
    g.close()


@pytest.mark.parametrize("physics", ["euler", "ns"])
def test_compensated_graph_steps_equal_eager_and_reset(physics):
    torch = need_gpu()
    announce("compensated graph vs eager", physics)
    n = (48, 32, 32)
    box = L3 if physics == "ns" else (10.0, 10.0, 10.0)
    U0 = inputs.smooth_random_state(n, box, seed=9).astype(np.float32).astype(np.float64)
    dt = inputs.cfl_dt(U0, n, box, 3, 1.4, 0.05)
    res = []
    for graphs in (False, True):
        _, g = pair(dict(n=n, length=box, nblk=(2, 2, 2), physics=physics, mode="at", algo="saa", L=4, seed=5),
                    "f32", dt=dt)
        g.set_compensation(True)
        g.set_graphs(graphs)
        for _ in range(2):           # the second pass must not see the first one's carried error
            g.set_state(torch.from_numpy(U0))
            g.step(12)
            res.append(to_np(g.get_state()))
        g.close()
    assert np.array_equal(res[0], res[1])
    assert np.array_equal(res[0], res[2])
    assert np.array_equal(res[2], res[3])
