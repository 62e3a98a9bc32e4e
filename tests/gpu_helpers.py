"""Shared helpers of the GPU parity tests: build matching oracle and library
instances from one specification, and compare fields."""
import math
import sys

import numpy as np
import pytest

from oracle import solver
from paper_2506_03027_amd import atns

PHYS = {"euler": atns.EULER, "ns": atns.NS}
RK = {"rk4": atns.RK4, "lserk4": atns.LSERK4, "lserk2": atns.LSERK2}
MODE = {"sa": atns.SA, "as": atns.AS, "at": atns.AT}
ALGO = {"caa": atns.CAA, "saa": atns.SAA}
EPS32 = 2.0 ** -24


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def announce(*what):
    print("[case]", *what, flush=True)
    sys.stdout.flush()


def pair(spec, precision="f64", dt=None):
    """(oracle, gpu solver) for a spec dict with keys n, length, ndim, nblk,
    physics, rk, mode, algo, L, seed, re, mach, split.  rk "lserk2" is the
    second-order method (CD2, AT2 with three levels) on both sides."""
    s = dict(ndim=3, nblk=(1, 1, 1), physics="euler", rk="rk4", mode="sa", algo="caa", L=1,
             seed=0, re=1600.0, mach=0.1, gamma=1.4, pr=0.71, split=None, filter_alpha=None)
    s.update(spec)
    cfg = solver.Config(s["n"], s["length"], s["ndim"], s["nblk"], s["physics"], gamma=s["gamma"],
                        mach=s["mach"], re=s["re"], pr=s["pr"], rk=s["rk"], mode=s["mode"],
                        algo=s["algo"], L=s["L"], seed=s["seed"], dt=dt, split=s["split"],
                        order=2 if s["rk"] == "lserk2" else 4, C=3 if s["rk"] == "lserk2" else 5,
                        filter_alpha=s["filter_alpha"])
    o = solver.Oracle(cfg)
    g = atns.Solver(n=s["n"], length=s["length"], ndim=s["ndim"], nblk=s["nblk"],
                    physics=PHYS[s["physics"]], gamma=s["gamma"], mach=s["mach"], re=s["re"],
                    pr=s["pr"], rk=RK[s["rk"]], mode=MODE[s["mode"]], algo=ALGO[s["algo"]],
                    L=s["L"], seed=s["seed"], precision=atns.F64 if precision == "f64" else atns.F32,
                    split=s["split"], filter_alpha=s["filter_alpha"])
    if dt is not None:
        g.set_dt(dt)
    return o, g


def set_both(o, g, U, step=0):
    import torch
    o.set_state(U, step)
    g.set_state(torch.from_numpy(np.ascontiguousarray(U)), step)


def to_np(t):
    return t.detach().double().cpu().numpy()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rel_max(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def flux_scale(U, gamma=1.4):
    """Largest magnitude among the inviscid flux components of U."""
    rho = U[0]
    vel = U[1:4] / rho
    p = (gamma - 1.0) * (U[4] - 0.5 * (U[1:4] * vel).sum(axis=0))
    return float(max(np.abs(U[1:4]).max(), np.abs(U[1:4] * vel).max() + np.abs(p).max(),
                     np.abs((U[4] + p) * vel).max()))
