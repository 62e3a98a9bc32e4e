"""Observed order of accuracy under grid refinement on the GPU (Table 1 and
Sec. 5.1: the AT stencils keep the order of the synchronous scheme under
delays; standard stencils reading delayed values drop to first order), for
the fourth-order method (RK4, CD4, AT4) and the second-order one of cases 1-3
(LSERK2, CD2, AT2).

The 3-D isentropic vortex on [0,10]^3 in 4x4x4 blocks, SAA delays with L = 4,
classical RK4 and CD4, at 64^3, 128^3 and 256^3 with dt proportional to the
grid spacing, to a fixed final time.  The order comes from self-convergence,
e_N = |U_N - U_2N| / |U_2N| over the points the two grids share, all five
conserved variables: the exact infinite-plane vortex is not a solution on the
periodic box (the velocity tail reaching the box edge floors the error
against it near 1e-7 at 256^3), while every grid here solves the same
periodic problem.  FP64 state, so that rounding stays far below the
truncation error."""
import math

import numpy as np
import pytest

from gpu_helpers import announce, need_gpu
from paper_2506_03027_amd import atns, inputs

pytestmark = pytest.mark.gpu

BOX = (10.0, 10.0, 10.0)
GRIDS = (64, 128, 256)
T_END = 0.25
CFL = 0.015        # stable for SAA with L = 4 on every grid


def final_state(mode, N, dt, steps, rk=atns.RK4):
    """Final FP64 state of one run, copied to the host."""
    n = (N, N, N)
    g = atns.Solver(n=n, length=BOX, ndim=3, nblk=(4, 4, 4), rk=rk, mode=mode, algo=atns.SAA, L=4, seed=3,
                    precision=atns.F64)
    g.set_dt(dt)
    g.init_case(atns.CASE_VORTEX)
    g.step(steps)
    U = g.get_state()
    g.close()
    return U.double().cpu().numpy()


@pytest.mark.parametrize("rk, mode, lo, hi", [
    (atns.RK4, atns.SA, 3.5, 4.6), (atns.RK4, atns.AT, 3.3, 4.8), (atns.RK4, atns.AS, 0.6, 1.6),
    (atns.LSERK2, atns.SA, 1.7, 2.4), (atns.LSERK2, atns.AT, 1.7, 2.4)])
def test_refinement_order(rk, mode, lo, hi):
    need_gpu()
    U = inputs.vortex_state((GRIDS[0],) * 3, BOX, 3)
    dt0 = inputs.cfl_dt(U, (GRIDS[0],) * 3, BOX, 3, 1.4, CFL)
    steps0 = int(math.ceil(T_END / dt0))
    dt0 = T_END / steps0
    errs, prev = [], None
    for i, N in enumerate(GRIDS):
        announce("order", rk, mode, N)
        U = final_state(mode, N, dt0 / 2 ** i, steps0 * 2 ** i, rk)
        if prev is not None:
            fine = U[:, ::2, ::2, ::2]
            errs.append(float(np.linalg.norm(prev - fine) / np.linalg.norm(fine)))
        prev = U
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    print("rk", rk, "mode", mode, "errors", errs, "orders", orders)
    assert lo < orders[-1] < hi, (errs, orders)


@pytest.mark.parametrize("mode, lo, hi", [(atns.AS, 0.6, 1.6), (atns.AT, 1.7, 4.5)])
def test_second_order_method_delay_error(mode, lo, hi):
    # Table 1 cases 2 and 3.  At these grids and this small step the CD2
    # truncation error (~1e-4) hides the first-order error of stale halos
    # (AS) in the self-convergence of the whole solution, so the error the
    # delays add is measured directly: |U_mode - U_SA| on the same grid.  It
    # falls at first order for AS and at (at least) second order for AT2.
    need_gpu()
    U = inputs.vortex_state((GRIDS[0],) * 3, BOX, 3)
    dt0 = inputs.cfl_dt(U, (GRIDS[0],) * 3, BOX, 3, 1.4, CFL)
    steps0 = int(math.ceil(T_END / dt0))
    dt0 = T_END / steps0
    errs = []
    for i, N in enumerate(GRIDS):
        announce("delay error", mode, N)
        Ua = final_state(mode, N, dt0 / 2 ** i, steps0 * 2 ** i, atns.LSERK2)
        Us = final_state(atns.SA, N, dt0 / 2 ** i, steps0 * 2 ** i, atns.LSERK2)
        errs.append(float(np.linalg.norm(Ua - Us) / np.linalg.norm(Us)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    print("lserk2 mode", mode, "delay errors", errs, "orders", orders)
    assert lo < orders[-1] < hi, (errs, orders)


def _u_2d(N, T, mode, P, L):
    """u-velocity after time T of the second-order method on the 2-D vortex
    (FP64), CAA with delay bound L on P blocks along x."""
    torch = need_gpu()
    n, length = (N, N, 1), (10.0, 10.0, 1.0)
    U0 = inputs.vortex_state(n, length, 2)
    dt = inputs.cfl_dt(U0, n, length, 2, 1.4, 0.05)
    steps = int(math.ceil(T / dt))
    g = atns.Solver(n=n, length=length, ndim=2, nblk=(P, 1, 1), rk=atns.LSERK2, mode=mode, algo=atns.CAA,
                    L=L, seed=1, precision=atns.F64)
    g.set_dt(T / steps)
    g.set_state(torch.from_numpy(U0))
    g.step(steps)
    U = g.get_state().double().cpu().numpy()
    g.close()
    return U[1] / U[0]


def test_delay_error_scaling_in_L_and_P():
    # Sec. 5.1 error scaling for Table 1 case 3 (CAA-AT, LSERK2-CD2-AT2): the
    # error the delays add (RMS u-velocity difference to the synchronous run)
    # is a cubic polynomial in L (C = 3 delayed levels) and grows linearly
    # with the number of blocks P (cut along x).
    need_gpu()
    N, T = 256, 1.0
    ref = _u_2d(N, T, atns.SA, 1, 1)

    def err(P, L):
        announce("delay error scaling", P, L)
        d = _u_2d(N, T, atns.AT, P, L) - ref
        return float(np.sqrt(np.mean(d * d)))

    Ls = np.arange(1, 9)
    EL = np.array([err(16, int(L)) for L in Ls])
    rel = {}
    for deg in (2, 3):
        c = np.polyfit(Ls, EL, deg)
        rel[deg] = float(np.max(np.abs(np.polyval(c, Ls) - EL) / EL))
    Ps = np.array([4, 8, 16, 32])
    EP = np.array([err(int(P), 4) for P in Ps])
    c = np.polyfit(Ps, EP, 1)
    r2 = 1.0 - np.sum((np.polyval(c, Ps) - EP) ** 2) / np.sum((EP - EP.mean()) ** 2)
    print("E(L), P = 16:", EL.tolist(), "relative residual quadratic / cubic fit:", rel)
    print("E(P), L = 4:", EP.tolist(), "linear fit", c.tolist(), "R^2", r2)
    assert np.all(np.diff(EL) > 0), EL
    assert rel[3] < 0.05 and rel[2] > 5 * rel[3], rel
    assert c[0] > 0 and r2 > 0.99, (EP, r2)
