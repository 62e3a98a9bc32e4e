"""Halo assembly inside the first stage kernel (graph-captured Euler steps):
the same bits as the separate halo kernel, for every halo mode and scheme,
with ragged blocks whose last tile is thinner than the 2-point apron (so two
tiles read, and assemble, the same halo points), and in 2-D."""
import numpy as np
import pytest

from gpu_helpers import announce, need_gpu, pair, to_np
from paper_2506_03027_amd import inputs

pytestmark = pytest.mark.gpu

# block sizes 17, 12, 11 / 9, 27 / 13, 11: with 16 x 8 x 6 tiles the last
# tile of a block is 1 point wide in x, y and z
RAGGED = dict(n=(40, 36, 24), length=(6.0, 5.0, 4.0), nblk=(3, 2, 2),
              split=([17, 12, 11], [9, 27], [13, 11]))


def _run(spec, U0, dt, tiles, fused, nsteps, torch):
    _, g = pair(spec, "f32", dt=dt)
    g.set_halo_fusion(fused)
    g.set_tiles(*tiles)
    g.set_state(torch.from_numpy(U0))
    g.step(nsteps)
    out = to_np(g.get_state())
    g.close()
    return out


@pytest.mark.parametrize("rk, mode, algo, L", [("rk4", "at", "saa", 3), ("rk4", "as", "saa", 3),
                                               ("rk4", "at", "caa", 4), ("lserk4", "at", "saa", 2),
                                               ("lserk2", "at", "saa", 3)])
@pytest.mark.parametrize("tiles", [(16, 8, 6), (32, 16, 32)])
def test_fused_halos_bitwise_equal_to_halo_kernel(rk, mode, algo, L, tiles):
    torch = need_gpu()
    announce("halo fusion", rk, mode, algo, L, tiles)
    n, box = RAGGED["n"], RAGGED["length"]
    U0 = inputs.smooth_random_state(n, box, seed=6)
    dt = inputs.cfl_dt(U0, n, box, 3, 1.4, 0.02)
    spec = dict(RAGGED, physics="euler", rk=rk, mode=mode, algo=algo, L=L, seed=13)
    a = _run(spec, U0, dt, tiles, True, 12, torch)
    b = _run(spec, U0, dt, tiles, False, 12, torch)
    assert np.isfinite(a).all()
    assert np.array_equal(a, b), float(np.abs(a - b).max())


def test_fused_halos_2d_and_eager_equal():
    torch = need_gpu()
    announce("halo fusion 2d")
    n, box = (48, 40, 1), (8.0, 6.0, 1.0)
    U0 = inputs.smooth_random_state(n, box, seed=3, ndim=2)
    dt = inputs.cfl_dt(U0, n, box, 2, 1.4, 0.02)
    spec = dict(n=n, length=box, ndim=2, nblk=(3, 2, 1), split=([17, 16, 15], [31, 9], [1]),
                physics="euler", mode="at", algo="saa", L=3, seed=4)
    a = _run(spec, U0, dt, (16, 8, 1), True, 12, torch)
    _, g = pair(spec, "f32", dt=dt)
    g.set_graphs(False)                   # eager: the separate halo kernel
    g.set_tiles(16, 8, 1)
    g.set_state(torch.from_numpy(U0))
    g.step(12)
    b = to_np(g.get_state())
    g.close()
    assert np.array_equal(a, b), float(np.abs(a - b).max())
