"""Graph-captured steps and batches.

A captured step reads its step number from a device counter, so one graph
serves every asynchronous step; these tests check that replays give the same
bits as eager steps (with eager work -- state reads, reductions, delay
queries -- between the replays), and that a batch of instances stepped by one
graph per step gives the same bits as each instance stepped alone."""
import numpy as np
import pytest

from gpu_helpers import announce, need_gpu, to_np
from paper_2506_03027_amd import atns, inputs

pytestmark = pytest.mark.gpu


def _solver(kw, graphs=True):
    s = atns.Solver(**kw)
    s.set_graphs(graphs)
    return s


def _case(physics, rk, mode, algo, L):
    n = (40, 36, 24)
    box = (6.0, 5.0, 4.0)
    kw = dict(n=n, length=box, ndim=3, nblk=(3, 2, 2), split=([20, 12, 8], [20, 16], [13, 11]),
              physics=physics, rk=rk, mode=mode, algo=algo, L=L, seed=9, re=200.0, mach=0.3,
              precision=atns.F32)
    U0 = inputs.smooth_random_state(n, box, seed=4)
    dt = inputs.cfl_dt(U0, n, box, 3, 1.4, 0.02)
    return kw, U0, dt


@pytest.mark.parametrize("physics,rk,mode,algo,L", [
    (atns.EULER, atns.RK4, atns.AT, atns.SAA, 3),
    (atns.EULER, atns.LSERK4, atns.AT, atns.CAA, 4),
    (atns.EULER, atns.RK4, atns.AS, atns.SAA, 2),
    (atns.EULER, atns.RK4, atns.SA, atns.CAA, 1),
    (atns.NS, atns.RK4, atns.AT, atns.CAA, 3),
    (atns.NS, atns.LSERK4, atns.AT, atns.SAA, 2),
    (atns.EULER, atns.LSERK2, atns.AT, atns.SAA, 3),
    (atns.NS, atns.LSERK2, atns.AT, atns.CAA, 2),
])
def test_graph_steps_match_eager_bitwise(physics, rk, mode, algo, L):
    torch = need_gpu()
    announce("graph-vs-eager", physics, rk, mode, algo, L)
    kw, U0, dt = _case(physics, rk, mode, algo, L)
    g, e = _solver(kw, True), _solver(kw, False)
    for s in (g, e):
        s.set_dt(dt)
        s.set_state(torch.from_numpy(U0))
    for chunk in (3, 4, 1, 5, 2):      # replays separated by eager work
        g.step(chunk)
        e.step(chunk)
        assert g.step_number() == e.step_number()
        a, b = to_np(g.get_state()), to_np(e.get_state())
        assert np.array_equal(a, b), g.step_number()
        da, oka = g.reduce()
        db, okb = e.reduce()
        assert oka and okb and np.array_equal(da, db)
        if mode != atns.SA:
            assert np.array_equal(g.get_delays(g.step_number() - 1), e.get_delays(e.step_number() - 1))
    # a new state (and step number) mid-run re-seeds the device counter
    U1 = e.get_state()
    for s in (g, e):
        s.set_state(U1, step=40)
        s.step(3)
    assert np.array_equal(to_np(g.get_state()), to_np(e.get_state()))
    g.close()
    e.close()


def test_graph_recaptured_after_dt_and_tile_changes():
    torch = need_gpu()
    announce("graph-recapture")
    kw, U0, dt = _case(atns.EULER, atns.RK4, atns.AT, atns.SAA, 3)
    g, e = _solver(kw, True), _solver(kw, False)
    for s in (g, e):
        s.set_dt(dt)
        s.set_state(torch.from_numpy(U0))
        s.step(7)
        s.set_dt(0.5 * dt)
        s.step(2)
    for s in (g, e):
        s.set_tiles(32, 8, 4)
        s.step(2)
    assert np.array_equal(to_np(g.get_state()), to_np(e.get_state()))
    g.close()
    e.close()


def test_graph_steps_with_learned_halo_match_eager():
    torch = need_gpu()
    announce("graph-mlp")
    from oracle import mlp
    kw, U0, dt = _case(atns.EULER, atns.RK4, atns.AT, atns.CAA, 3)
    theta = (mlp.init(3) * 0.05).astype(np.float32)
    outs = []
    for graphs in (True, False):
        s = _solver(kw, graphs)
        s.set_dt(dt)
        s.mlp_set_params(theta)
        s.mlp_set_scales(np.full(5, 1e-2), np.full(5, 1e-6))
        s.mlp_enable(True, tau=0.5)
        s.set_state(torch.from_numpy(U0))
        s.step(10)
        outs.append((to_np(s.get_state()), s.mlp_stats()))
        s.close()
    assert np.array_equal(outs[0][0], outs[1][0])
    assert outs[0][1] == outs[1][1]
    assert sum(outs[0][1]) > 0          # corrections were evaluated


# ------------------------------------------------------------------ batches
def _batch_configs():
    cfgs = []
    shapes = [((32, 32, 32), (1, 1, 1), None), ((48, 40, 24), (2, 2, 1), ([24, 24], [16, 24], [24])),
              ((40, 32, 32), (2, 1, 2), None), ((24, 24, 16), (1, 2, 1), None)]
    for i, (n, nblk, split) in enumerate(shapes):
        physics = atns.EULER if i % 2 == 0 else atns.NS
        cfgs.append(dict(n=n, length=tuple(0.2 * x for x in n), ndim=3, nblk=nblk, split=split,
                         physics=physics, rk=atns.RK4, mode=atns.AT,
                         algo=atns.SAA if i < 2 else atns.CAA, L=(1, 2, 4, 3)[i], seed=11 + i,
                         re=300.0, mach=0.3, precision=atns.F32))
    return cfgs


def _start(s, kw, i, torch):
    U0 = inputs.smooth_random_state(kw["n"], kw["length"], seed=20 + i)
    dt = inputs.cfl_dt(U0, kw["n"], kw["length"], 3, 1.4, 0.02)
    s.set_dt(dt)
    s.set_state(torch.from_numpy(U0))
    return dt


def test_batch_matches_individual_bitwise():
    torch = need_gpu()
    announce("batch-vs-individual")
    cfgs = _batch_configs()
    b = atns.Batch(cfgs)
    b.set_tiles(atns.EULER, 32, 8, 8)
    b.set_tiles(atns.NS, 16, 8, 16)
    solo = [atns.Solver(**kw) for kw in cfgs]
    for s, kw in zip(solo, cfgs):
        s.set_tiles(*((32, 8, 8) if kw["physics"] == atns.EULER else (16, 8, 16)))
    dts = []
    for i, kw in enumerate(cfgs):
        dts.append(_start(b.members[i], kw, i, torch))
        _start(solo[i], kw, i, torch)
    for chunk in (4, 3, 5):
        b.step(chunk)
        for s in solo:
            s.step(chunk)
        for i in range(len(cfgs)):
            assert b.members[i].step_number() == solo[i].step_number()
            a, c = to_np(b.members[i].get_state()), to_np(solo[i].get_state())
            assert np.isfinite(a).all()
            assert np.array_equal(a, c), (i, solo[i].step_number())
    # a member's dt change is picked up by the batch graph
    b.members[1].set_dt(0.5 * dts[1])
    solo[1].set_dt(0.5 * dts[1])
    b.step(2)
    for s in solo:
        s.step(2)
    for i in range(len(cfgs)):
        assert np.array_equal(to_np(b.members[i].get_state()), to_np(solo[i].get_state())), i
    b.close()
    for s in solo:
        s.close()


@pytest.mark.skip(reason="aborted (SIGABRT inside the former batch autotuner, which re-captured the batch "
                         "graph for every tile shape) with no GPU fault and no cause found by reading; that "
                         "autotuner is removed (the batch now times its stage kernels directly, without any graph capture) and "
                         "this case stays off the GPU")
def test_batch_autotune_and_errors():
    torch = need_gpu()
    announce("batch-autotune")
    cfgs = _batch_configs()[:2]
    b = atns.Batch(cfgs)
    for i, kw in enumerate(cfgs):
        _start(b.members[i], kw, i, torch)
    with pytest.raises(atns.AtnsError):
        b.autotune(1)                       # still in the synchronous start
    b.step(6)
    eu, ns = b.autotune(1)
    assert eu[:2] in [(16, 16), (32, 8), (16, 8)]
    assert ns[:2] in [(16, 16), (32, 8), (16, 8)]
    b.step(2)
    assert all(np.isfinite(to_np(m.get_state())).all() for m in b.members)
    # members at different steps are refused
    b.members[0].step(1)
    with pytest.raises(atns.AtnsError):
        b.step(1)
    b.close()
    bad = dict(cfgs[0], rk=atns.LSERK4)
    with pytest.raises(atns.AtnsError):
        atns.Batch([cfgs[0], bad])


def test_batch_autotune_leaves_states_and_picks_shapes():
    torch = need_gpu()
    announce("batch-autotune-members")
    cfgs = _batch_configs()
    b = atns.Batch(cfgs)
    for i, kw in enumerate(cfgs):
        _start(b.members[i], kw, i, torch)
    before = [to_np(m.get_state()) for m in b.members]
    eu, ns = b.autotune(1)
    assert eu[:2] in [(16, 16), (32, 8), (16, 8), (64, 8), (32, 16)] and eu[2] in (4, 8, 16, 32)
    assert ns[:2] in [(16, 16), (32, 8), (16, 8), (32, 16)] and ns[2] in (8, 16, 32)
    for m, kw, U in zip(b.members, cfgs, before):
        assert m.get_tiles() == (eu if kw["physics"] == atns.EULER else ns)
        assert np.array_equal(to_np(m.get_state()), U)      # timing never touches the state
        assert m.step_number() == 0
    b.step(7)
    assert all(np.isfinite(to_np(m.get_state())).all() for m in b.members)
    b.close()


def test_batch_refuses_members_at_different_steps():
    torch = need_gpu()
    announce("batch-errors")
    cfgs = _batch_configs()[:2]
    b = atns.Batch(cfgs)
    for i, kw in enumerate(cfgs):
        _start(b.members[i], kw, i, torch)
    b.step(6)
    b.members[0].step(1)
    with pytest.raises(atns.AtnsError):
        b.step(1)
    b.close()
    with pytest.raises(atns.AtnsError):
        atns.Batch([cfgs[0], dict(cfgs[0], rk=atns.LSERK4)])
