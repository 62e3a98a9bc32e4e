"""GPU parity of the learned halo correction (BF16 MFMA MLP) against the
FP64 reference: forward, gradient, the training sampler, training, and the
corrected asynchronous solver."""
import math

import numpy as np
import pytest

from bounds import bf16_forward_bound
from gpu_helpers import announce, need_gpu, pair, rel_max, set_both, to_np
from oracle import at as oat, delays as odl, mlp as omlp
from paper_2506_03027_amd import atns, inputs
from test_gpu_parity import BOX, smooth_history

pytestmark = pytest.mark.gpu


def small_ctx(torch, precision="f64"):
    o, g = pair(dict(n=(32, 24, 20), length=BOX, nblk=(2, 2, 2), mode="at", algo="saa", L=4, seed=7),
                precision)
    return o, g


def test_mlp_forward_matches_reference():
    torch = need_gpu()
    announce("mlp forward")
    _, g = small_ctx(torch)
    th = omlp.init(5)
    th[omlp.NIN * omlp.NH: omlp.NIN * omlp.NH + 64] = 0.1    # nonzero b1
    th32 = th.astype(np.float32)
    g.mlp_set_params(th32)
    assert np.array_equal(g.mlp_get_params(), th32)
    X = np.random.default_rng(1).standard_normal((1000, 64)).astype(np.float32)
    out = to_np(g.mlp_forward(torch.from_numpy(X)))
    ref, _ = omlp.forward(th32.astype(np.float64), X.astype(np.float64), round_bf16=True)
    err = np.abs(out - ref)
    scale = np.abs(ref).max()
    assert err.max() < 2e-3 * scale, err.max() / scale
    assert np.median(err) < 1e-5 * scale


def test_mlp_forward_within_bf16_bound_of_plain_fp64():
    # The GPU network (BF16 operands on the matrix cores, FP32 accumulation)
    # against the plain FP64 forward pass, element by element, within the
    # bound derived from BF16 operand rounding (tests/bounds.py).
    torch = need_gpu()
    announce("mlp forward vs plain fp64")
    _, g = small_ctx(torch)
    th = omlp.init(8)
    th[omlp.NIN * omlp.NH: omlp.NIN * omlp.NH + 64] = 0.1
    th32 = th.astype(np.float32)
    g.mlp_set_params(th32)
    X = np.random.default_rng(4).standard_normal((2000, 64)).astype(np.float32)
    out = to_np(g.mlp_forward(torch.from_numpy(X)))
    plain, _ = omlp.forward(th32.astype(np.float64), X.astype(np.float64))
    bound = bf16_forward_bound(th32.astype(np.float64), X.astype(np.float64))
    viol = np.abs(out - plain) - bound
    assert viol.max() <= 0.0, float(viol.max())


def test_mlp_gradient_matches_reference():
    torch = need_gpu()
    announce("mlp grad")
    _, g = small_ctx(torch)
    th = omlp.init(6).astype(np.float32)
    g.mlp_set_params(th)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((300, 64)).astype(np.float32)   # ragged last workgroup
    Y = rng.standard_normal((300, 8)).astype(np.float32)
    grad, loss = g.mlp_grad(torch.from_numpy(X), torch.from_numpy(Y))
    grad = to_np(grad)
    lref, gref = omlp.loss_and_grad(th.astype(np.float64), X.astype(np.float64), Y.astype(np.float64))
    assert abs(loss - lref) < 1e-2 * lref
    rel = np.linalg.norm(grad - gref) / np.linalg.norm(gref)
    cos = grad @ gref / (np.linalg.norm(grad) * np.linalg.norm(gref))
    assert rel < 3e-2 and cos > 0.999, (rel, cos)
    # deterministic
    grad2, loss2 = g.mlp_grad(torch.from_numpy(X), torch.from_numpy(Y))
    assert np.array_equal(to_np(grad2), grad) and loss2 == loss


def _face_regions(o):
    out = []
    for b in range(len(o.blocks)):
        for v in o.slots:
            if v < 6:
                out.append((b, v))
    return out


def test_sampler_matches_reference():
    torch = need_gpu()
    announce("mlp sampler")
    o, g = small_ctx(torch)
    nstep = 14
    hist = smooth_history(o.cfg.n, list(range(nstep - g.ring_depth + 1, nstep + 1)))
    for m, U in sorted(hist.items()):
        set_both(o, g, U, step=m)
    s = np.array([1e-3, 2e-3, 2e-3, 2e-3, 5e-3], dtype=np.float32)
    r = np.array([1e-5, 2e-5, 2e-5, 2e-5, 4e-5], dtype=np.float32)
    g.mlp_set_scales(s, r)
    n, seed = 200, 12345
    X, Y = g.mlp_sample(n, seed)
    X, Y = to_np(X), to_np(Y)
    faces = _face_regions(o)
    W0 = oat.halo_table("rk4", "at", 5, 3)[0]
    L = 4
    for i in range(n):
        h1 = odl.splitmix64_draw(seed, 2 * i)
        h2 = odl.splitmix64_draw(seed, 2 * i + 1)
        b, v = faces[h1 % len(faces)]
        rng = o.blocks.region(b, v)
        ex, ey, ez = len(rng[0]), len(rng[1]), len(rng[2])
        pt = (h1 >> 32) % (ex * ey * ez)
        k = h2 % L
        d, mask = omlp.correction_for_region(np.zeros(9360), s, np.ones(5), 1e30, o.history, nstep,
                                             k, L, o.blocks, b, v, o.cfg.H)
        # features at the point, recomputed through the reference path
        pts = omlp.region_points(o.blocks, b, v, o.cfg.H)
        cz, cy, cx = pt // (ex * ey), (pt // ex) % ey, pt % ex
        f32 = np.float32
        feats = []
        for l in range(4):
            for vv in range(5):
                for j in range(3):
                    val = f32(o.history[nstep - k - l][vv][pts[j][0][cz, cy, cx], pts[j][1][cz, cy, cx],
                                                           pts[j][2][cz, cy, cx]])
                    c = f32(o.history[nstep - k][vv][pts[1][0][cz, cy, cx], pts[1][1][cz, cy, cx],
                                                     pts[1][2][cz, cy, cx]])
                    feats.append(f32((val - c) * (f32(1) / f32(s[vv]))))
        assert np.array_equal(X[i, :60].astype(np.float32), np.array(feats, dtype=np.float32)), i
        assert X[i, 60] == pytest.approx(k / 3)
        gi = (pts[1][0][cz, cy, cx], pts[1][1][cz, cy, cx], pts[1][2][cz, cy, cx])
        for vv in range(5):
            ext = sum(W0[k, l] * o.history[nstep - k - l][vv][gi] for l in range(5))
            tgt = (o.history[nstep][vv][gi] - ext) / r[vv]
            assert Y[i, vv] == pytest.approx(tgt, rel=1e-5, abs=1e-4 * abs(1 / r[vv]) * 1e-12 + 1e-6)


@pytest.mark.parametrize("tau", [1e30, 0.0, "mid"])
def test_corrected_solver_matches_reference(tau):
    torch = need_gpu()
    announce("mlp solver", tau)
    o, g = small_ctx(torch)
    nstep = 14
    hist = smooth_history(o.cfg.n, list(range(nstep - g.ring_depth + 1, nstep + 1)))
    for m, U in sorted(hist.items()):
        set_both(o, g, U, step=m)
    dt = 2e-3
    o.cfg.dt = dt
    g.set_dt(dt)
    th = (omlp.init(9) * 0.5).astype(np.float32)
    s = np.array([1e-3, 2e-3, 2e-3, 2e-3, 5e-3], dtype=np.float32)
    r = np.array([1e-4, 2e-4, 2e-4, 2e-4, 4e-4], dtype=np.float32)
    g.mlp_set_params(th)
    g.mlp_set_scales(s, r)
    if tau == "mid":
        # a threshold in a gap of the |out| distribution so both sides decide alike
        X, _ = g.mlp_sample(4000, 3)
        nrm = np.sqrt((to_np(g.mlp_forward(X))[:, :5] ** 2).sum(axis=1))
        qs = np.sort(nrm)
        gaps = np.diff(qs[len(qs) // 4: 3 * len(qs) // 4])
        j = int(np.argmax(gaps)) + len(qs) // 4
        tau = float(0.5 * (qs[j] + qs[j + 1]))
    g.mlp_enable(True, tau)
    o.mlp = dict(theta=th.astype(np.float64), s=s, r=r, tau=tau)
    g.mlp_stats()
    g.step(2)
    o.step(2)
    applied, fallback = g.mlp_stats()
    assert applied + fallback > 0
    if tau == 0.0:
        assert applied == 0
    if tau == 1e30:
        assert fallback == 0
    assert [applied, fallback] == o.mlp_counts
    G = to_np(g.get_state())
    # the correction itself agrees to ~1e-3 relative (BF16 operands, FP32 sums)
    dmax = float(np.max(r)) * 10
    assert np.abs(G - o.U).max() < 1e-12 * np.abs(o.U).max() + 1e-3 * dmax


TRAIN_N = (48, 48, 48)
L3 = (2 * math.pi,) * 3


@pytest.fixture(scope="module")
def trained():
    """Train on a synchronous FP64 Navier-Stokes TGV history (the target, the
    AT extrapolation error, is a truncation error there; in FP32 it sits
    below the rounding noise of the levels and cannot be learned)."""
    torch = need_gpu()
    announce("mlp train")
    n = TRAIN_N
    _, g = pair(dict(n=n, length=L3, nblk=(3, 3, 3), physics="ns", mode="sa", L=4, re=1600.0,
                     mach=0.1), "f64")
    U0 = inputs.tgv_state(n)
    dt = inputs.cfl_dt(U0, n, L3, 3, 1.4, 1.0)
    g.set_dt(dt)
    g.set_state(torch.from_numpy(U0))
    g.step(12)
    g.mlp_set_scales(np.ones(5), np.ones(5))
    X, Y = g.mlp_sample(8192, 1)
    X, Y = to_np(X), to_np(Y)
    s = (np.sqrt((X[:, :60].reshape(-1, 4, 5, 3) ** 2).mean(axis=(0, 1, 3))) + 1e-30).astype(np.float32)
    r = (np.sqrt((Y[:, :5] ** 2).mean(axis=0)) + 1e-30).astype(np.float32)
    g.mlp_set_scales(s, r)
    g.mlp_set_params(omlp.init(0).astype(np.float32) * np.float32(0.5))
    losses = []
    for rnd in range(6):
        g.step(2)
        losses.extend(g.mlp_train(100, 1024, 1e-3, 100 + rnd).tolist())
    X, Y = g.mlp_sample(4096, 999)
    out = to_np(g.mlp_forward(X))[:, :5]
    Yn = to_np(Y)[:, :5]
    res = dict(theta=g.mlp_get_params(), s=s, r=r, dt=dt, losses=losses,
               mse_mlp=float(((out - Yn) ** 2).mean()), mse_at=float((Yn ** 2).mean()))
    g.close()
    return res


def test_training_reduces_loss_and_halo_error(trained):
    ls = trained["losses"]
    print("loss first/last", np.mean(ls[:10]), np.mean(ls[-50:]))
    print("halo error (normalised MSE): AT", trained["mse_at"], "AT+MLP", trained["mse_mlp"])
    assert np.mean(ls[-50:]) < 0.7 * np.mean(ls[:10])
    assert trained["mse_mlp"] < 0.6 * trained["mse_at"]


# The learned halo's gain, on a case shaped like the 512^3 workload's blocks
# (32^3 Navier-Stokes blocks, SAA with L = 5, so delays reach 4) at a time
# step where the AT4 extrapolation error (about 1e-3 relative after 30
# steps) sits far above rounding: FP64 throughout, CFL 1.0.  The network is
# trained on the solver's own synchronous FP64 history (20 rounds of 100
# Adam iterations), then AT and AT + MLP runs are compared with the
# synchronous run of the same steps.  Required: AT + MLP's relative L2
# below (1 - DELTA) times AT's.
GAIN_N = (64, 64, 64)
GAIN_DELTA = 0.05


def test_learned_halo_gain_on_32cubed_blocks_at_delay_bound():
    torch = need_gpu()
    announce("mlp gain, 32^3 blocks, L=5")
    n, L = GAIN_N, 5
    _, g = pair(dict(n=n, length=L3, nblk=(2, 2, 2), physics="ns", mode="sa", L=L, re=1600.0, mach=0.1), "f64")
    U0 = inputs.tgv_state(n)
    dt = inputs.cfl_dt(U0, n, L3, 3, 1.4, 1.0)
    g.set_dt(dt)
    g.set_state(torch.from_numpy(U0))
    g.step(12)
    g.mlp_set_scales(np.ones(5), np.ones(5))
    X, Y = g.mlp_sample(8192, 1)
    X, Y = to_np(X), to_np(Y)
    s = (np.sqrt((X[:, :60].reshape(-1, 4, 5, 3) ** 2).mean(axis=(0, 1, 3))) + 1e-30).astype(np.float32)
    r = (np.sqrt((Y[:, :5] ** 2).mean(axis=0)) + 1e-30).astype(np.float32)
    g.mlp_set_scales(s, r)
    g.mlp_set_params(omlp.init(0).astype(np.float32) * np.float32(0.5))
    for rnd in range(20):
        g.step(2)
        g.mlp_train(100, 1024, 1e-3, 100 + rnd)
    theta = g.mlp_get_params()
    g.close()
    out = {}
    for name, mode, use in (("sa", "sa", False), ("at", "at", False), ("mlp", "at", True)):
        _, h = pair(dict(n=n, length=L3, nblk=(2, 2, 2), physics="ns", mode=mode, algo="saa", L=L, seed=3,
                         re=1600.0, mach=0.1), "f64", dt=dt)
        if use:
            h.mlp_set_params(theta)
            h.mlp_set_scales(s, r)
            h.mlp_enable(True, 10.0)
        h.set_state(torch.from_numpy(U0))
        h.step(30)
        out[name] = to_np(h.get_state())
        if use:
            out["stats"] = h.mlp_stats()
        h.close()
    e_at = np.linalg.norm(out["at"] - out["sa"]) / np.linalg.norm(out["sa"])
    e_mlp = np.linalg.norm(out["mlp"] - out["sa"]) / np.linalg.norm(out["sa"])
    print("rel L2 vs SA after 30 steps: AT %.4e  AT+MLP %.4e  gain %.3f  (applied, fallback) %s"
          % (e_at, e_mlp, 1 - e_mlp / e_at, out["stats"]))
    assert e_at > 1e-5                    # the delay error is far above rounding here
    assert out["stats"][0] > 0
    assert e_mlp < (1.0 - GAIN_DELTA) * e_at
