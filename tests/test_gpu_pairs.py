"""Fused RK4 stage pairs (atns_set_fusion): stages 1-2 and 3-4 of a 3-D
Euler step run as two kernels, stage A on the tile plus a 2-point apron and
stage B in the same pass.  They must give the same bits as the four
separate stage kernels, for every halo mode, delay algorithm, tile shape,
ragged tile and uneven block, on graph-captured and eager steps."""
import numpy as np
import pytest

from gpu_helpers import announce, need_gpu, to_np
from paper_2506_03027_amd import atns, inputs

pytestmark = pytest.mark.gpu


def _run(kw, U0, dt, tiles, fuse, graphs, steps):
    torch = need_gpu()
    g = atns.Solver(**kw)
    g.set_graphs(graphs)
    g.set_tiles(*tiles)
    g.set_fusion(fuse)
    g.set_dt(dt)
    g.set_state(torch.from_numpy(U0))
    g.step(steps)
    U = to_np(g.get_state())
    g.close()
    return U


@pytest.mark.parametrize("mode, algo, L", [(atns.SA, atns.CAA, 1), (atns.AT, atns.SAA, 3), (atns.AT, atns.CAA, 4),
                                           (atns.AS, atns.SAA, 2)])
@pytest.mark.parametrize("tiles", [(16, 16, 8), (32, 8, 8), (16, 8, 16), (32, 16, 4)])
def test_fused_pairs_equal_separate_stages(mode, algo, L, tiles):
    need_gpu()
    announce("fused pairs", mode, algo, L, tiles)
    n = (40, 36, 24)
    box = (6.0, 5.0, 4.0)
    kw = dict(n=n, length=box, ndim=3, nblk=(3, 2, 2), split=([20, 12, 8], [20, 16], [13, 11]),
              mode=mode, algo=algo, L=L, seed=9, precision=atns.F32)
    U0 = inputs.smooth_random_state(n, box, seed=4)
    dt = inputs.cfl_dt(U0, n, box, 3, 1.4, 0.02)
    ref = _run(kw, U0, dt, tiles, False, False, 11)
    for graphs in (False, True):
        out = _run(kw, U0, dt, tiles, True, graphs, 11)
        assert np.isfinite(out).all()
        assert np.array_equal(out, ref), (graphs, np.abs(out - ref).max())


def test_fused_pairs_on_the_vortex_workload_grid():
    # the benchmark's block layout (4x4x4 blocks of 32^3) at 64^3 points per
    # block edge halved: 2x2x2 blocks of 32^3, SAA L = 4, graph steps
    need_gpu()
    announce("fused pairs vortex")
    n = (64, 64, 64)
    box = (10.0, 10.0, 10.0)
    kw = dict(n=n, length=box, ndim=3, nblk=(2, 2, 2), mode=atns.AT, algo=atns.SAA, L=4, seed=1,
              precision=atns.F32)
    U0 = inputs.vortex_state(n, box, 3)
    dt = inputs.cfl_dt(U0, n, box, 3, 1.4, 0.02)
    ref = _run(kw, U0, dt, (32, 8, 8), False, True, 20)
    out = _run(kw, U0, dt, (32, 8, 8), True, True, 20)
    assert np.array_equal(out, ref), np.abs(out - ref).max()
