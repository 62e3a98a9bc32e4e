"""Full-size checks at the benchmark workloads' own sizes and launch
configuration (grid, blocks, delays, FP32, the tile shape the autotuner picks,
graph-captured steps):

* the right-hand side with AT halos from a delayed history, on sampled points
  (block corners, edges, faces and interior), against the one-point-at-a-time
  FP64 oracle evaluated from the same FP32 levels;
* graph-captured steps with the tuned tile shape against eager steps with a
  different shape, bit for bit (a property that holds at any size).

The history is U^m = B + sin(w s) G1 + (1 - cos(w s)) G2 with s = m - n: smooth
in time but not a polynomial, so the AT weights are exercised.  B, G1 and G2
are separable fields (inputs.separable_spec), built on the device by
broadcasting and evaluated on the host point by point with the same operations.
"""
import functools
import math

import numpy as np
import pytest

from gpu_helpers import EPS32, announce, need_gpu, pair, to_np
from oracle import pointwise
from paper_2506_03027_amd import inputs

pytestmark = pytest.mark.gpu

OMEGA = 0.3


def _spec(w):
    return dict(n=w["n"], length=w["length"], nblk=w["nblk"], physics=w["physics"], rk=w["rk"],
                mode=w["mode"], algo=w["algo"], L=w["L"], seed=w.get("seed", 1),
                re=w.get("re", 1600.0), mach=w.get("mach", 0.1))


class History:
    """Levels U^m of the full grid: on the device (whole fields) and on the
    host (single points, memoized)."""

    def __init__(self, torch, w, nstep):
        n, box = w["n"], w["length"]
        self.nstep = nstep
        self.specs = [inputs.separable_spec(n, box, seed=s, amp=0.05) for s in (31, 32, 33)]
        self.shape = (n[2], n[1], n[0])
        dev = lambda v: torch.from_numpy(np.ascontiguousarray(v)).to("cuda")
        B, Q1, Q2 = (inputs.separable_field(sp, dev) for sp in self.specs)
        self.dB = torch.stack(B)
        self.dG1 = 0.02 * (torch.stack(Q1) - 1.0)
        self.dG2 = 0.02 * (torch.stack(Q2) - 1.0)

    def coef(self, m):
        s = m - self.nstep
        return math.sin(OMEGA * s), 1.0 - math.cos(OMEGA * s)

    def device_level(self, m):
        c, d = self.coef(m)
        return (self.dB + c * self.dG1 + d * self.dG2).float()

    @functools.lru_cache(maxsize=None)
    def _point(self, x, y, z):
        return (inputs.separable_at(self.specs[0], x, y, z), inputs.separable_at(self.specs[1], x, y, z),
                inputs.separable_at(self.specs[2], x, y, z))

    def value(self, m, v, z, y, x):
        b, q1, q2 = self._point(x, y, z)
        c, d = self.coef(m)
        val = b[v] + c * (0.02 * (q1[v] - 1.0)) + d * (0.02 * (q2[v] - 1.0))
        return float(np.float32(val))

    def level(self, m):
        hist = self

        class Level:
            shape = (5,) + hist.shape

            def __getitem__(self, idx):
                v, z, y, x = idx
                return hist.value(m, int(v), int(z), int(y), int(x))

        return Level()


def _flux_scale(torch, U, gamma=1.4):
    """Largest magnitude among the inviscid flux components of U (device)."""
    rho = U[0].double()
    vel = U[1:4].double() / rho
    p = (gamma - 1.0) * (U[4].double() - 0.5 * (U[1:4].double() * vel).sum(dim=0))
    return float(max(U[1:4].abs().max(), (U[1:4].double() * vel).abs().max() + p.abs().max(),
                     ((U[4].double() + p) * vel).abs().max()))


def _sample_points(o, rng, nblocks):
    pts = []
    for b in rng.choice(len(o.blocks), size=nblocks, replace=False):
        size, org = o.blocks.sizes[b], o.blocks.origins[b]
        sx, sy, sz = size
        cand = [(0, 0, 0), (sx - 1, sy - 1, sz - 1), (0, sy - 1, sz // 2), (sx // 2, 0, sz - 1),
                (1, sy // 2, 1), (sx - 2, 1, sz // 2), (sx // 2, sy // 2, sz // 2),
                tuple(int(rng.integers(0, s)) for s in size)]
        pts += [(int(b), p) for p in cand]
    return pts


def _build(torch, name, nstep):
    w = inputs.WORKLOADS[name]
    o, g = pair(_spec(w), "f32")
    hist = History(torch, w, nstep)
    for m in range(nstep - g.ring_depth + 1, nstep + 1):
        g.set_state(hist.device_level(m), step=m)
    return w, o, g, hist


@pytest.mark.parametrize("name, nblocks, inject", [("vortex3d_128", 8, False), ("tgv_256", 4, False),
                                                   ("tgv_512", 6, True)])
def test_fullsize_rhs_every_stage_sampled_against_pointwise_oracle(name, nblocks, inject):
    """Every RK stage's right-hand side (each stage has its own AT halo
    weights, Eqs. 8-15) on sampled points.  For the 512^3 workload (SAA,
    L = 5) delays at the bound k = 4 are injected on every face and edge slot
    of the sampled blocks, so the largest weights ||W_e(4)||_1 (up to about
    1.5e3) enter the comparison."""
    torch = need_gpu()
    announce("fullsize rhs", name)
    nstep = 21
    w, o, g, hist = _build(torch, name, nstep)
    tiles = g.autotune(reps=2)           # the shape the benchmark would run
    print("tiles", tiles, flush=True)
    rng = np.random.default_rng(5)
    pts = _sample_points(o, rng, nblocks)
    if inject:
        kin = o.delays(nstep).copy()
        for b in {b for b, _ in pts}:
            kin[b, :] = w["L"] - 1
        g.set_delays(nstep, kin[None].astype(np.int8))
        o.set_delays(nstep, kin)
    k = o.delays(nstep)
    assert k is not None and k.max() == w["L"] - 1
    if inject:
        assert all((k[b, :18] == w["L"] - 1).all() for b, _ in pts)
    U = hist.device_level(nstep)
    scale = _flux_scale(torch, U)
    del U
    h = o.cfg.h
    tol = 64 * EPS32 * scale / min(h)
    if w["physics"] == "ns":
        tol *= 1.0 + 1.0 / (o.cfg.gas.re * min(h))
    order = 4
    levels = {m: hist.level(m) for m in range(nstep - 12, nstep + 1)}
    for e in range(o.s):
        R = g.rhs(stage=e)
        worst = 0.0
        for b, p in pts:
            org, size = o.blocks.origins[b], o.blocks.sizes[b]
            get = pointwise.block_accessor(levels[nstep], levels, nstep, org, size, p, k=k[b], W=o.W, e=e,
                                           C=o.cfg.C, mode=w["mode"])
            ref = pointwise.rhs_point(get, h, 3, w["physics"], o.cfg.gas, order)
            gx, gy, gz = ((org[d] + p[d]) % w["n"][d] for d in range(3))
            got = R[:, gz, gy, gx].double().cpu().numpy()
            err = float(np.abs(got - np.array(ref)).max())
            worst = max(worst, err)
            assert err < tol, (name, e, b, p, err, tol)
        del R
        print("fullsize rhs", name, "stage", e, "worst", worst, "tol", tol, flush=True)
    if inject:
        g.set_delays(0, np.zeros((0, g.nblocks, 18), dtype=np.int8))
    g.close()


@pytest.mark.parametrize("name, other", [("vortex3d_128", (16, 16, 8)), ("tgv_256", (32, 8, 16)),
                                         ("tgv_512", (16, 16, 16))])
def test_fullsize_graph_steps_with_tuned_tiles_match_eager(name, other):
    torch = need_gpu()
    announce("fullsize steps", name)
    nstep = 21
    w, o, g, hist = _build(torch, name, nstep)
    tiles = g.autotune(reps=2)
    if tuple(tiles) == tuple(other):
        other = (16, 8, 8)
    box = w["length"]
    U = hist.device_level(nstep)
    dt = 0.25 * inputs.cfl_dt(to_np(U[:, ::4, ::4, ::4]), tuple(x // 4 for x in w["n"]), box, 3, 1.4,
                              w["cfl"])
    g.set_dt(dt)
    g.step(2)                            # graph-captured, tuned tiles
    A = to_np(g.get_state())
    g.close()
    _, _, g2, _ = _build(torch, name, nstep)
    g2.set_graphs(False)
    g2.set_tiles(*other)
    g2.set_dt(dt)
    g2.step(2)
    B = to_np(g2.get_state())
    g2.close()
    assert np.isfinite(A).all()
    assert np.array_equal(A, B), (name, tiles, other, float(np.abs(A - B).max()))
