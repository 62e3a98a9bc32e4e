"""Writes vortex3d_32_saa_l4_t1.npy: the FP64 oracle's state at T = 1 of the
3-D isentropic vortex on [0, 10]^3 with 32^3 points in 4 x 4 x 4 blocks (the
block layout of the 128^3 vortex workload on the smallest grid that keeps
it), SAA delays with L = 4 (k in 0..3, Alg. 3), AT4 halos (Eqs. 7-15), CD4,
classical RK4, dt from CFL 0.02 rounded down so that a whole number of steps
ends exactly at T = 1.  The initial field is rounded to FP32 first, so a
single-precision run starts from the same values.

Only the oracle computes the stored field; the GPU test that reads it
(tests/test_gpu_long.py) compares the FP32 library against it.

    python tests/golden/make_vortex3d_t1.py        (about six minutes on one core)
"""
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2506_03027_amd import inputs  # noqa: E402  (input generator only)

OUT = os.path.join(HERE, "vortex3d_32_saa_l4_t1.npy")
CASE = dict(n=(32, 32, 32), length=(10.0, 10.0, 10.0), nblk=(4, 4, 4), physics="euler", rk="rk4",
            mode="at", algo="saa", L=4, seed=11, cfl=0.02, T=1.0)


def initial_state():
    U0 = inputs.vortex_state(CASE["n"], CASE["length"], 3)
    return U0.astype(np.float32).astype(np.float64)


def time_step():
    """(dt, steps): the CFL step rounded down to T / steps."""
    dt_cfl = inputs.cfl_dt(initial_state(), CASE["n"], CASE["length"], 3, 1.4, CASE["cfl"])
    steps = int(math.ceil(CASE["T"] / dt_cfl))
    return CASE["T"] / steps, steps


def main():
    from oracle import solver
    dt, steps = time_step()
    c = CASE
    o = solver.Oracle(solver.Config(c["n"], c["length"], 3, c["nblk"], c["physics"], rk=c["rk"], mode=c["mode"],
                                    algo=c["algo"], L=c["L"], seed=c["seed"], dt=dt))
    o.set_state(initial_state())
    o.step(steps)
    assert np.isfinite(o.U).all()
    np.save(OUT, o.U)
    print("wrote", OUT, "steps", steps, "dt", dt)


if __name__ == "__main__":
    main()
