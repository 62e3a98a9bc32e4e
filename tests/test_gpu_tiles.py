"""Tile shapes and the autotuner: every supported shape (ragged columns
included) gives bit-identical results, and the tuner picks and caches one."""
import math
import os

import numpy as np
import pytest

from gpu_helpers import announce, need_gpu, pair, to_np
from paper_2506_03027_amd import atns, inputs

pytestmark = pytest.mark.gpu

SHAPES = {"euler": [(16, 16), (32, 8), (16, 8), (64, 8), (32, 16)],
          "ns": [(16, 16), (32, 8), (16, 8)]}


GRIDS = {
    # narrow, ragged blocks: partial tiles everywhere
    "ragged": dict(n=(40, 36, 24), length=(6.0, 5.0, 4.0), nblk=(3, 2, 2),
                   split=([20, 12, 8], [20, 16], [13, 11])),
    # one wide block: full tiles of every shape (and a partial z column)
    "wide": dict(n=(64, 48, 20), length=(8.0, 6.0, 2.5), nblk=(1, 1, 1), split=None),
}


@pytest.mark.parametrize("grid", ["ragged", "wide"])
@pytest.mark.parametrize("physics", ["euler", "ns"])
def test_all_tile_shapes_bitwise_equal(physics, grid):
    torch = need_gpu()
    announce("tiles", physics, grid)
    gd = GRIDS[grid]
    n, box = gd["n"], gd["length"]
    U0 = inputs.smooth_random_state(n, box, seed=2)
    dt = inputs.cfl_dt(U0, n, box, 3, 1.4, 0.03)
    ref = None
    for tx, ty in SHAPES[physics]:
        for tz in (4, 7, 16):
            if physics == "ns" and tz < 8 and (tx, ty) != (16, 16):
                continue
            _, g = pair(dict(n=n, length=box, nblk=gd["nblk"], split=gd["split"], physics=physics,
                             mode="at", algo="saa", L=3, seed=5, re=200.0, mach=0.3), "f32", dt=dt)
            g.set_tiles(tx, ty, tz)
            assert g.get_tiles() == (tx, ty, tz)
            g.set_state(torch.from_numpy(U0))
            g.step(8)
            out = to_np(g.get_state())
            g.close()
            assert np.isfinite(out).all(), (tx, ty, tz)
            if ref is None:
                ref = out
            else:
                assert np.array_equal(out, ref), (tx, ty, tz)


def test_bad_tile_shape_rejected():
    need_gpu()
    _, g = pair(dict(n=(16, 16, 16), length=(1.0, 1.0, 1.0), nblk=(1, 1, 1)), "f32")
    with pytest.raises(atns.AtnsError):
        g.set_tiles(8, 8, 4)
    with pytest.raises(atns.AtnsError):
        g.set_tiles(64, 4, 4)
    with pytest.raises(atns.AtnsError):
        g.set_tiles(16, 16, 0)


def test_autotune_picks_and_caches(tmp_path):
    torch = need_gpu()
    announce("autotune")
    n = (64, 64, 64)
    box = (10.0, 10.0, 10.0)
    U0 = inputs.vortex_state(n, box, 3)
    cache = str(tmp_path / "tune.txt")
    _, g = pair(dict(n=n, length=box, nblk=(2, 2, 2), mode="at", algo="saa", L=4), "f32")
    g.set_state(torch.from_numpy(U0))
    best = g.autotune(reps=2, cache=cache)
    assert best[:2] in SHAPES["euler"]
    assert g.get_tiles() == best
    assert os.path.exists(cache) and len(open(cache).read().split()) == 4
    _, g2 = pair(dict(n=n, length=box, nblk=(2, 2, 2), mode="at", algo="saa", L=4), "f32")
    g2.set_state(torch.from_numpy(U0))
    assert g2.autotune(reps=2, cache=cache) == best      # served from the cache
    assert len(open(cache).read().split()) == 4


def test_profiled_steps_count_launches_and_keep_results():
    """Profiling times every step's stage launches (eagerly) and leaves the
    results bit-identical to unprofiled, graph-captured steps."""
    torch = need_gpu()
    announce("profile")
    n, box = (32, 32, 32), (4.0, 4.0, 4.0)
    U0 = inputs.smooth_random_state(n, box, seed=4)
    dt = inputs.cfl_dt(U0, n, box, 3, 1.4, 0.03)
    cfg = dict(n=n, length=box, nblk=(2, 2, 2), physics="euler", mode="at", algo="saa", L=3, seed=2)
    outs = []
    for prof in (False, True):
        _, g = pair(cfg, "f32", dt=dt)
        g.set_state(torch.from_numpy(U0))
        g.step(6)
        g.profile(prof)
        g.step(3)
        if prof:
            launches, ms = g.profile_read()
            assert launches == 3 * 4 and ms > 0.0
            g.step(1)
            assert g.profile_read()[0] == 4        # the read cleared the record
            g.profile(False)
            g.step(1)
        else:
            g.step(2)
        outs.append(to_np(g.get_state()))
        g.close()
    assert np.array_equal(outs[0], outs[1])
