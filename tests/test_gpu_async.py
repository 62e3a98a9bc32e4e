"""Free-running asynchronous steps (atns_step_async), Euler and 3-D
Navier-Stokes: one persistent workgroup per block, delays that arise from the run itself (the
synchronization-avoiding rule of Alg. 3 without a schedule).  Parity: the
realized delays are logged, and replaying them through the scheduled path
(atns_set_delays) and through the oracle reproduces the run."""
import numpy as np
import pytest

from gpu_helpers import announce, need_gpu, pair, rel_max, set_both, to_np
from paper_2506_03027_amd import atns, inputs

pytestmark = pytest.mark.gpu

BOX = (10.0, 10.0, 10.0)


def _start(o, g, n, dt, warm):
    """Same vortex start and `warm` scheduled steps on oracle and GPU."""
    U0 = inputs.vortex_state(n, BOX, 3)
    set_both(o, g, U0)
    g.step(warm)
    o.step(warm)


@pytest.mark.parametrize("physics, rk, mode, L", [("euler", "rk4", "at", 3), ("euler", "lserk2", "as", 2),
                                                  ("euler", "lserk2", "at", 4), ("ns", "rk4", "at", 3),
                                                  ("ns", "lserk2", "at", 2)])
def test_free_running_steps_replay_exactly(physics, rk, mode, L):
    torch = need_gpu()
    announce("free-running", physics, rk, mode, L)
    n = (32, 24, 16) if physics == "euler" else (24, 16, 16)
    U0 = inputs.vortex_state(n, BOX, 3)
    dt = inputs.cfl_dt(U0, n, BOX, 3, 1.4, 0.05)
    spec = dict(n=n, length=BOX, nblk=(2, 2, 2), physics=physics, rk=rk, mode=mode, algo="saa", L=L, seed=3,
                re=200.0, mach=0.3)
    o, g = pair(spec, "f64", dt=dt)
    C = 3 if rk == "lserk2" else 5
    warm = C + L
    _start(o, g, n, dt, warm)
    nsteps = 12
    log = g.step_async(nsteps)
    assert g.step_number() == warm + nsteps
    used = log >= 0
    assert log.shape == (nsteps, 8, 18)
    assert used.any() and np.all(log[used] <= L - 1)
    # slots the physics does not use (Euler: the 12 edges) stay -1
    if physics == "euler":
        assert np.all(log[:, :, 6:] == -1) and np.all(log[:, :, :6] >= 0)
    else:
        assert np.all(log >= 0)
    A = to_np(g.get_state())
    # replay on the scheduled path
    _, r = pair(spec, "f64", dt=dt)
    r.set_state(torch.from_numpy(U0))
    r.step(warm)
    r.set_delays(warm, log)
    r.step(nsteps)
    B = to_np(r.get_state())
    print("realized delay histogram", np.bincount(log[used].ravel(), minlength=L),
          "async vs replay max |diff|", np.abs(A - B).max())
    assert rel_max(A, B) < 1e-13
    # replay in the oracle
    for j in range(nsteps):
        o.set_delays(warm + j, log[j].astype(np.int64).clip(0))
    o.step(nsteps)
    assert rel_max(A, o.U) < 1e-12, rel_max(A, o.U)
    g.close()
    r.close()


def test_free_running_fp32_many_blocks():
    # 4x4x4 blocks of 16^3, FP32: the run stays finite, its delays stay
    # bounded, and its replay on the scheduled FP32 path agrees.
    torch = need_gpu()
    announce("free-running fp32 64 blocks")
    n = (64, 64, 64)
    U0 = inputs.vortex_state(n, BOX, 3)
    dt = inputs.cfl_dt(U0, n, BOX, 3, 1.4, 0.02)
    kw = dict(n=n, length=BOX, ndim=3, nblk=(4, 4, 4), mode=atns.AT, algo=atns.SAA, L=4, seed=1,
              precision=atns.F32)
    runs = []
    for replay in (False, True):
        g = atns.Solver(**kw)
        g.set_dt(dt)
        g.set_state(torch.from_numpy(U0))
        g.step(8)
        if replay:
            g.set_delays(8, log)
            g.step(40)
        else:
            log = g.step_async(40)
        runs.append(to_np(g.get_state()))
        g.close()
    used = log >= 0
    print("realized delay histogram", np.bincount(log[used].ravel(), minlength=4))
    assert np.isfinite(runs[0]).all() and np.all(log[used] <= 3)
    assert rel_max(runs[0], runs[1]) < 1e-6


def test_free_running_rejects_unsupported_contexts():
    torch = need_gpu()
    announce("free-running errors")
    n = (32, 32, 32)
    base = dict(n=n, length=BOX, ndim=3, nblk=(2, 2, 2), mode=atns.AT, algo=atns.SAA, L=2, seed=1)
    U0 = inputs.vortex_state(n, BOX, 3)
    base2d = dict(base, n=(32, 32, 1), ndim=2, nblk=(2, 2, 1), length=(10.0, 10.0, 1.0))
    for kw in (dict(base2d, physics=atns.NS), dict(base, mode=atns.SA), dict(base, rk=atns.LSERK4)):
        g = atns.Solver(**kw)
        g.set_dt(1e-3)
        g.set_state(torch.from_numpy(U0 if kw["ndim"] == 3 else inputs.vortex_state(kw["n"], kw["length"], 2)))
        g.step(8)
        with pytest.raises(atns.AtnsError):
            g.step_async(2)
        g.close()
    # history too short
    g = atns.Solver(**base)
    g.set_dt(1e-3)
    g.set_state(torch.from_numpy(U0))
    with pytest.raises(atns.AtnsError):
        g.step_async(2)
    g.close()
    # more blocks than resident workgroups: 16^3 blocks of 2^3 points
    g = atns.Solver(**dict(base, n=(32, 32, 32), nblk=(16, 16, 16)))
    g.set_dt(1e-3)
    g.set_state(torch.from_numpy(U0))
    g.step(8)
    with pytest.raises(atns.AtnsError):
        g.step_async(2)
    g.close()
