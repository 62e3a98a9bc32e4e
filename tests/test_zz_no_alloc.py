"""The allocation-free diagnostics entry point (atns_reduce_noalloc) against
atns_reduce on the same fields, through the C ABI: two calls in a row on one
GPU, the second on a smaller field, and the size limit."""
import math

import numpy as np
import pytest

from gpu_helpers import announce, need_gpu, pair, set_both
from paper_2506_03027_amd import atns, inputs

pytestmark = pytest.mark.gpu

L3 = (2 * math.pi,) * 3


def _case(torch, n, length, precision, physics, seed):
    o, g = pair(dict(n=n, length=length, nblk=(1, 1, 1), physics=physics), precision)
    U = inputs.smooth_random_state(n, length, seed=seed)
    if physics == "ns":
        U = inputs.tgv_state(n) + 0.01 * (U - 1.0)
    set_both(o, g, U)
    ref, ok = g.reduce()
    assert ok
    return g, ref


def test_reduce_noalloc_matches_reduce_on_two_calls():
    torch = need_gpu()
    announce("reduce_noalloc")
    out = torch.full((7,), float("nan"), dtype=torch.float64, device="cuda")
    # first call: a 48 x 40 x 32 single-precision field
    g, ref = _case(torch, (48, 40, 32), L3, "f32", "ns", 3)
    U = g.get_state()
    atns.reduce_noalloc(U, L3, 3, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.array_equal(got, ref), (got, ref)
    g.close()
    # second call, smaller field in double precision: the shared partials are
    # rewritten, nothing of the first call remains
    box = (10.0, 10.0, 10.0)
    g, ref = _case(torch, (20, 16, 12), box, "f64", "euler", 5)
    U = g.get_state()
    out.fill_(float("nan"))
    atns.reduce_noalloc(U, box, 3, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.array_equal(got, ref), (got, ref)
    g.close()


def test_reduce_noalloc_rejects_bad_sizes():
    torch = need_gpu()
    announce("reduce_noalloc sizes")
    U = torch.ones((5, 4, 8, 8), dtype=torch.float32, device="cuda")
    out = torch.zeros(7, dtype=torch.float64, device="cuda")
    with pytest.raises(atns.AtnsError):
        atns.reduce_noalloc(U, L3, 3, out)      # 4 points along z: too few for CD4
    big = torch.empty((5, 1, 1, 1), dtype=torch.float32, device="cuda")
    import ctypes
    n = (ctypes.c_int32 * 3)(2048, 2048, 128)    # 5 n^3 >= 2^31: rejected before any launch
    ln = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    st = atns.lib().atns_reduce_noalloc(ctypes.c_void_p(big.data_ptr()), atns.F32, 3, n, ln,
                                        ctypes.c_void_p(out.data_ptr()), None)
    assert st == -1
