"""Pins of the oracle's asynchronous solver (no GPU): decomposition,
orders of accuracy of Table 1, conservation, delay schedules and the halo
rule, checked against brute force."""
import math

import numpy as np
import pytest

from oracle import at as atmod, delays as dl, diagnostics, flow, pointwise, rk, solver
from conftest import read_golden
from paper_2506_03027_amd import inputs


def vortex_run(N, mode, nblk=(2, 2, 1), algo="caa", L=4, T=0.5, rkname="rk4",
               seed=1, split=None, halo="closed", dt_scale=1.0, order=4, C=5):
    n, length = (N, N, 1), (10.0, 10.0, 1.0)
    U0 = inputs.vortex_state(n, length, 2)
    # dt proportional to h, fixed by the N = 32 value at CFL ~ 0.3
    dt32 = 0.3 * (10.0 / 32) / (0.5 * math.sqrt(1.4) * math.sqrt(2) + math.sqrt(1.4)) / 2
    nsteps = int(round(T / (dt_scale * dt32 * 32 / N)))
    cfg = solver.Config(n, length, ndim=2, nblk=nblk, physics="euler", rk=rkname,
                        mode=mode, algo=algo, L=L, seed=seed, dt=T / nsteps, split=split,
                        order=order, C=C)
    o = solver.Oracle(cfg)
    o.halo = halo
    o.set_state(U0)
    o.step(nsteps)
    return o, inputs.vortex_state(n, length, 2, t=T)


def rms(a):
    return float(np.sqrt(np.mean(a * a)))


# ---------------------------------------------------------- decomposition
@pytest.mark.parametrize("physics", ["euler", "ns"])
def test_sa_decomposed_equals_single_block_bitwise(physics):
    n, length = (16, 16, 16), (2 * math.pi,) * 3
    U0 = inputs.smooth_random_state(n, length, seed=3)
    out = []
    for nblk, split in (((1, 1, 1), None), ((2, 2, 2), None),
                        ((3, 2, 2), [[4, 7, 5], [9, 7], [8, 8]])):
        cfg = solver.Config(n, length, 3, nblk, physics, rk="rk4", mode="sa",
                            re=100.0, dt=1e-3, split=split)
        o = solver.Oracle(cfg)
        o.set_state(U0)
        o.step(2)
        out.append(o.U)
    assert np.array_equal(out[0], out[1])
    assert np.array_equal(out[0], out[2])


# -------------------------------------------------- Table 1 orders (4-6)
def _orders(mode, Ns=(32, 64, 128), **kw):
    errs = []
    for N in Ns:
        o, ex = vortex_run(N, mode, **kw)
        errs.append(rms(o.U[0] - ex[0]))
    return errs, [math.log2(errs[i] / errs[i + 1]) for i in range(2)]


@pytest.mark.slow
@pytest.mark.parametrize("rkname", ["rk4", "lserk4"])
def test_table1_orders_sa_at_as(rkname):
    # Table 1 cases 4, 6 and 5: SA and AT keep fourth order, AS drops to first.
    # Random (SAA) delays need a smaller step for stability (Sec. 3.1 notes the
    # stricter CFL condition under delays): L = 3 at a quarter of the step.
    _, o_sa = _orders("sa", rkname=rkname)
    _, o_at = _orders("at", rkname=rkname, algo="caa", L=4)
    _, o_saa = _orders("at", rkname=rkname, algo="saa", L=3, seed=7, dt_scale=0.25)
    _, o_as = _orders("as", rkname=rkname, algo="caa", L=4)
    assert o_sa[-1] > 3.7 and o_at[-1] > 3.7 and o_saa[-1] > 3.7, (o_sa, o_at, o_saa)
    assert 0.7 < o_as[-1] < 1.3, o_as


@pytest.mark.slow
def test_table1_orders_second_order_method():
    # Table 1 cases 1, 3 and 2: LSERK2 with CD2 in the interior and AT2 (three
    # delayed levels) at block boundaries keeps second order under CAA and
    # SAA delays; standard CD2 on stale data (AS) drops to first order.  The
    # expected orders are those of the golden table.
    expect = {(r[1], r[2]): int(r[-1]) for r in read_golden("table1_orders.txt")}
    kw = dict(rkname="lserk2", order=2, C=3, dt_scale=0.5)
    _, o_sa = _orders("sa", **kw)
    _, o_at = _orders("at", algo="caa", L=4, **kw)
    _, o_saa = _orders("at", algo="saa", L=3, seed=7, **kw)
    _, o_as = _orders("as", algo="caa", L=4, **kw)
    print("orders SA", o_sa, "CAA-AT", o_at, "SAA-AT", o_saa, "AS", o_as)
    assert expect[("SA", "lserk2")] == 2 and expect[("AT", "lserk2")] == 2 and expect[("AS", "lserk2")] == 1
    assert 1.8 < o_sa[-1] < 2.3 and 1.8 < o_at[-1] < 2.3 and 1.8 < o_saa[-1] < 2.3, (o_sa, o_at, o_saa)
    assert 0.7 < o_as[-1] < 1.3, o_as


_U_CACHE = {}


def _u_2d(N, T, mode, P, L):
    """u-velocity after time T of the second-order method (Table 1 cases
    1-3: LSERK2, CD2, AT2) on the 2-D vortex, CAA with delay bound L on P
    blocks along x."""
    key = (N, T, mode, P, L)
    if key not in _U_CACHE:
        n, length = (N, N, 1), (10.0, 10.0, 1.0)
        U0 = inputs.vortex_state(n, length, 2)
        dt = inputs.cfl_dt(U0, n, length, 2, 1.4, 0.05)
        steps = int(math.ceil(T / dt))
        cfg = solver.Config(n, length, ndim=2, nblk=(P, 1, 1), physics="euler", rk="lserk2", mode=mode,
                            algo="caa", L=L, seed=1, dt=T / steps, order=2, C=atmod.AT2_C)
        o = solver.Oracle(cfg)
        o.set_state(U0)
        o.step(steps)
        _U_CACHE[key] = o.U[1] / o.U[0]
    return _U_CACHE[key]


def _delay_error_2d(N, T, P, L):
    """RMS u-velocity difference between CAA-AT and the synchronous run."""
    d = _u_2d(N, T, "at", P, L) - _u_2d(N, T, "sa", 1, 1)
    return float(np.sqrt(np.mean(d * d)))


@pytest.mark.slow
def test_delay_error_cubic_in_L_and_linear_in_P():
    # Sec. 5.1 error scaling: the error that delays add grows with the
    # moments of the delay up to order C (a cubic polynomial in L for AT2,
    # C = 3) and with the share of points next to block boundaries (linear
    # in the number of blocks P when they are cut along one axis).
    Ls = np.arange(1, 9)
    EL = np.array([_delay_error_2d(64, 0.5, 8, int(L)) for L in Ls])
    assert np.all(np.diff(EL) > 0), EL
    rel = {}
    for deg in (2, 3):
        c = np.polyfit(Ls, EL, deg)
        rel[deg] = float(np.max(np.abs(np.polyval(c, Ls) - EL) / EL))
    print("E(L)", EL, "max relative residual of the quadratic / cubic fit", rel)
    assert rel[3] < 0.05 and rel[2] > 5 * rel[3], rel
    Ps = np.array([4, 8, 16])
    EP = np.array([_delay_error_2d(64, 0.5, int(P), 4) for P in Ps])
    c = np.polyfit(Ps, EP, 1)
    r2 = 1.0 - np.sum((np.polyval(c, Ps) - EP) ** 2) / np.sum((EP - EP.mean()) ** 2)
    print("E(P)", EP, "linear fit", c, "R^2", r2)
    assert c[0] > 0 and r2 > 0.99, (EP, r2)


def test_at_with_zero_delay_converges_to_sa():
    # AT with every delay 0 differs from SA only through the temporal
    # extrapolation of later stages, an O(h^4) effect.
    diffs = []
    for N in (32, 64):
        o_sa, _ = vortex_run(N, "sa")
        n, length = (N, N, 1), (10.0, 10.0, 1.0)
        cfg = o_sa.cfg
        cfg2 = solver.Config(n, length, 2, (2, 2, 1), "euler", rk="rk4", mode="at",
                             algo="saa", L=4, dt=cfg.dt)
        o = solver.Oracle(cfg2)
        o.set_state(inputs.vortex_state(n, length, 2))
        nsteps = o_sa.n
        for s in range(nsteps):
            o.set_delays(s, np.zeros((4, dl.NSLOTS), dtype=np.int64))
        o.step(nsteps)
        diffs.append(rms(o.U[0] - o_sa.U[0]))
    assert diffs[1] > 0
    assert math.log2(diffs[0] / diffs[1]) > 3.5


# ------------------------------------------------------------ conservation
@pytest.mark.parametrize("physics", ["euler", "ns"])
def test_sa_conserves_totals(physics):
    n, length = (16, 16, 16), (2 * math.pi,) * 3
    U0 = inputs.smooth_random_state(n, length, seed=11)
    h = inputs.spacing(n, length)
    cfg = solver.Config(n, length, 3, (2, 2, 2), physics, mode="sa", re=200.0, dt=2e-3)
    o = solver.Oracle(cfg)
    o.set_state(U0)
    t0 = diagnostics.totals(U0, h)
    o.step(20)
    t1 = diagnostics.totals(o.U, h)
    scale = np.abs(t0).max()
    assert np.abs(t1 - t0).max() < 1e-13 * scale


def test_at_conservation_drift_is_small_and_nonzero():
    o, _ = vortex_run(32, "at", algo="saa", L=3, seed=3, T=0.3, dt_scale=0.25)
    h = o.cfg.h
    t0 = diagnostics.totals(inputs.vortex_state(o.cfg.n, o.cfg.length, 2), h)
    t1 = diagnostics.totals(o.U, h)
    rel = np.abs(t1 - t0)[[0, 4]] / np.abs(t0)[[0, 4]]
    assert rel.max() > 1e-14 and rel.max() < 1e-5


# ------------------------------------------------------------- halo rules
def test_literal_buffer_recursion_equals_closed_form():
    for rkname in ("rk4", "lserk4"):
        a, _ = vortex_run(32, "at", algo="saa", L=3, seed=5, T=0.2, rkname=rkname,
                          dt_scale=0.25)
        b, _ = vortex_run(32, "at", algo="saa", L=3, seed=5, T=0.2, rkname=rkname,
                          halo="literal", dt_scale=0.25)
        assert np.abs(a.U - b.U).max() < 1e-11 * np.abs(a.U).max()


@pytest.mark.parametrize("physics", ["euler", "ns"])
@pytest.mark.parametrize("mode,rkname", [("at", "rk4"), ("as", "rk4"), ("at", "lserk2")])
def test_stage_rhs_matches_pointwise_halo_rule(physics, mode, rkname):
    # Brute force: classify every stencil point of every owned point into
    # owned / halo slot and evaluate the halo value from the full-field history.
    # lserk2 runs the second-order method: CD2 and AT2 (three levels).
    order, C = (2, atmod.AT2_C) if rkname == "lserk2" else (4, atmod.AT4_C)
    n, length = (12, 12, 8), (6.0, 6.0, 4.0)
    cfg = solver.Config(n, length, 3, (3, 2, 2), physics, rk=rkname, mode=mode, algo="saa",
                        L=4, seed=9, re=50.0, mach=0.3, dt=1e-3,
                        split=[[4, 4, 4], [5, 7], [4, 4]], order=order, C=C)
    o = solver.Oracle(cfg)
    nstep = 8
    hist = {}
    for m in range(nstep - 7, nstep + 1):
        hist[m] = inputs.smooth_random_state(n, length, seed=100 + m, amp=0.03)
        o.set_state(hist[m], step=m)
    k = o.delays()
    assert k is not None and k.max() > 0
    Y = inputs.smooth_random_state(n, length, seed=1)
    W = o.W if mode == "at" else None
    rng = np.random.default_rng(2)
    for e in ((0, 1) if rkname == "lserk2" else (0, 2)):
        R = o.rhs(Y, e, k)
        for b in range(len(o.blocks)):
            size = o.blocks.sizes[b]
            org = o.blocks.origins[b]
            cand = [(0, 0, 0), (size[0] - 1, size[1] - 1, size[2] - 1),
                    (1, size[1] - 2, 0), (size[0] - 2, 0, size[2] - 1)]
            cand += [tuple(rng.integers(0, s) for s in size) for _ in range(2)]
            for p in cand:
                get = pointwise.block_accessor(Y, hist, nstep, org, size, p, k=k[b],
                                               W=W, e=e, C=cfg.C, mode=mode)
                r = pointwise.rhs_point(get, cfg.h, 3, physics, cfg.gas, order)
                g = [(org[d] + p[d]) % n[d] for d in range(3)]
                ref = R[:, g[2], g[1], g[0]]
                assert np.allclose(r, ref, rtol=1e-9, atol=1e-9 * np.abs(R).max()), (e, b, p)


# ------------------------------------------------------------------ delays
def test_caa_delay_pattern():
    C, L = 5, 4
    assert dl.delays("caa", 3, 2, L, C, 0) is None
    seq = [int(dl.delays("caa", n, 2, L, C, 0)[0, 0]) for n in range(5, 15)]
    assert seq == [0, 1, 2, 3, 0, 1, 2, 3, 0, 1]


def test_saa_delays_uniform_and_bounded():
    C, L = 5, 4
    ks = np.concatenate([dl.delays("saa", n, 64, L, C, 42).ravel() for n in range(20, 60)])
    assert ks.min() == 0 and ks.max() == L - 1
    counts = np.bincount(ks, minlength=L)
    expected = len(ks) / L
    chi2 = ((counts - expected) ** 2 / expected).sum()
    assert chi2 < 16.3        # 3 dof, p = 0.001


def test_saa_first_async_step_limited_by_history():
    C, L = 5, 4
    k = dl.delays("saa", C, 64, L, C, 42)          # only levels 0..C exist
    assert k.max() <= 1


def test_guard_resets_large_and_unavailable_delays():
    C, L = 5, 4
    over = np.array([[0, 3, 4, 7, -1, 2]])
    k = dl.delays("saa", 6, 1, L, C, 0, override=over)   # n - C + 1 = 2
    assert k.tolist() == [[0, 0, 0, 0, 0, 2]]


def test_splitmix64_matches_published_outputs():
    """The SAA delay draw is SplitMix64's i-th output for the seed; pinned to
    the generator's published outputs from state 0."""
    from conftest import read_golden
    for i, hx in read_golden("splitmix64_state0.txt"):
        assert dl.splitmix64_draw(0, int(i)) == int(hx, 16)


def test_splitmix64_is_deterministic_and_seed_dependent():
    a = [dl.splitmix64_draw(1, i) for i in range(4)]
    assert a == [dl.splitmix64_draw(1, i) for i in range(4)]
    assert a != [dl.splitmix64_draw(2, i) for i in range(4)]
    assert all(0 <= x < 2 ** 64 for x in a)
    assert len(set(a)) == 4


# ----------------------------------------------------------- NS + delays
def test_tgv_ns_at_runs_close_to_sa():
    n = (16, 16, 16)
    length = (2 * math.pi,) * 3
    U0 = inputs.tgv_state(n)
    dt = inputs.cfl_dt(U0, n, length, 3, 1.4, 0.05)
    res = {}
    for mode in ("sa", "at"):
        cfg = solver.Config(n, length, 3, (2, 2, 2), "ns", mode=mode, algo="saa", L=4,
                            seed=3, re=1600.0, mach=0.1, dt=dt)
        o = solver.Oracle(cfg)
        o.set_state(U0)
        o.step(12)
        res[mode] = o.U
    rel = np.linalg.norm(res["at"] - res["sa"]) / np.linalg.norm(res["sa"])
    assert 0 < rel < 1e-6
