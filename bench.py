"""Throughput benchmark of the AT compressible-flow hot path on one MI355X.

Metric: grid-point x RK-stage updates per second of the FP32 asynchrony-
tolerant solver (one "step" = one RK step of the whole hot path: delay draw,
AT halo assembly from the delayed-level ring, CD4 flux divergence, RK stage
updates, ring write of the new boundary layers), with inputs resident in HBM.
Reported beside it, on the same grid, start and step count: the plain FP64
synchronous (SA) path, and, for the Taylor-Green workloads, the FP32 AT solver
with the learned halo correction; the relative L2 of every path against the
FP64 SA result; the roofline of the dominant (fused stage) kernel from HIP
events recorded around its launches and of the whole step; and the FP64 oracle
timed on the host CPU on a bounded sample of the same workload (with the FP32
GPU result's L2 error against it).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu] [--no-mlp]

NAME is one of the single-instance workloads (default tgv_512: the
Taylor-Green vortex, Re 1600 Mach 0.1, 512^3 in 32^3 blocks, SAA delays up to
4) or batch48, the batched persistent launch of 48 uneven instances.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2506_03027_amd import atns, inputs  # noqa: E402

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E
C_LEVELS = 5              # delayed levels of AT4 (RK4, LSERK4)
RK_ID = {"rk4": atns.RK4, "lserk4": atns.LSERK4, "lserk2": atns.LSERK2}


def n_stages(w):
    return atns.stages(RK_ID[w["rk"]])


def n_levels(w):
    """Delayed levels C of the workload's AT scheme (5 for AT4, 3 for AT2)."""
    return atns.levels(RK_ID[w["rk"]])


def halo_fraction(w):
    """f = halo points per owned point of a block: faces of depth H (2 for
    Euler, 4 for Navier-Stokes) and, for Navier-Stokes, the 2x2 edge prisms."""
    n, nb, ndim = w["n"], w["nblk"], w["ndim"]
    H = 4 if w["physics"] == "ns" else 2
    b = [n[d] // nb[d] for d in range(3)]
    own = b[0] * b[1] * (b[2] if ndim == 3 else 1)
    dims = range(ndim)
    halo = 0
    for d in dims:
        face = 1
        for e in dims:
            if e != d:
                face *= b[e]
        halo += 2 * H * face
    if w["physics"] == "ns":
        for d in dims:
            for e in dims:
                if e > d:
                    other = [x for x in dims if x not in (d, e)]
                    length = b[other[0]] if other else 1
                    halo += 4 * 4 * length
    return halo / own


def algorithmic_bytes_per_point_stage(w, stages, esz):
    """Bytes the method must move per owned point per RK stage, whole step:
    the state in and out plus one RK register (80 B at FP32, averaged over
    the stages), plus, for delayed halos, C ring levels (AT; one level for
    AS) of 5 values per halo point, plus the ring write of the boundary
    layers once per step."""
    f = halo_fraction(w)
    scale = esz / 4.0
    if w["mode"] == "sa":
        return 80.0 * scale, f
    levels = n_levels(w) if w["mode"] == "at" else 1
    return (80.0 + 20.0 * levels * f + 20.0 * f / stages) * scale, f


def stage_kernel_bytes_per_point(w, stages, esz):
    """Bytes the fused stage kernel itself must move per owned point and
    launch: the 80 B of state and RK register, one assembled halo value of
    5 variables per halo point (the sum over the C delayed levels is done
    once per step by the halo kernel), and the ring write of the last stage
    averaged over the stages."""
    f = halo_fraction(w)
    scale = esz / 4.0
    if w["mode"] == "sa":
        return 80.0 * scale
    return (80.0 + 20.0 * f + 20.0 * f / stages) * scale


def filter_bytes_per_point(w):
    """Bytes per owned point the filter of one step with delayed halos must
    move (3-D cubic blocks of side s, FP32): the state read and written once
    (40 B), the 10 halo values per line of each of the three passes (600/s B),
    the ring write of the filtered boundary layers (faces 5 deep, 2-wide edge
    prisms: 30/s + 48/s^2 values per point, 5 variables), and the filter-halo
    slot (5-deep faces, 30/s values per point) that the halo kernel writes
    from the delayed levels it already reads for the stage halos."""
    s = w["n"][0] // w["nblk"][0]
    return 40.0 + 600.0 / s + 20.0 * (30.0 / s + 48.0 / s ** 2) + 20.0 * 30.0 / s


def make_solver(w, precision, mode=None, filter_alpha=None):
    phys = atns.NS if w["physics"] == "ns" else atns.EULER
    m = {"sa": atns.SA, "as": atns.AS, "at": atns.AT}[mode or w["mode"]]
    algo = atns.SAA if w.get("algo", "saa") == "saa" else atns.CAA
    return atns.Solver(n=w["n"], length=w["length"], ndim=w["ndim"], nblk=w["nblk"], physics=phys,
                       mach=w.get("mach", 0.1), re=w.get("re", 1600.0),
                       rk=RK_ID[w["rk"]], mode=m, algo=algo,
                       L=w["L"], seed=w.get("seed", 1), precision=precision, filter_alpha=filter_alpha)


def initial_state(w):
    if w["physics"] == "ns":
        return inputs.tgv_state(w["n"], mach=w.get("mach", 0.1))
    return inputs.vortex_state(w["n"], w["length"], w["ndim"])


def time_steps(torch, g, steps):
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.step(steps)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


TUNE_CACHE = os.environ.get("ATNS_TUNE_CACHE", os.path.join("/tmp", "atns_tune.txt"))


def run_path(torch, w, precision, mode, steps, warmup, dt, U0=None, net=None, filter_alpha=None):
    """One path of the workload from the initial field: the autotuned tiles,
    `warmup` untimed steps, `steps` timed graph-captured steps, then `steps`
    eager steps with the stage kernels bracketed by HIP events.  net (the
    learned halo: theta, s, r, tau) switches the correction on.  Returns the
    timings, the tiles, the learned-halo counts of the timed steps and the
    final state (on the device).  filter_alpha switches the tenth-order
    filter on."""
    g = make_solver(w, precision, mode, filter_alpha)
    g.set_dt(dt)
    if U0 is None:
        g.init_case(atns.CASE_TGV if w["physics"] == "ns" else atns.CASE_VORTEX)
    else:
        g.set_state(torch.from_numpy(U0))
    if net is not None:
        g.mlp_set_params(net["theta"])
        g.mlp_set_scales(net["s"], net["r"])
        g.mlp_enable(True, net["tau"])
    tiles = g.autotune(reps=10, cache=TUNE_CACHE)
    g.step(warmup)
    if net is not None:
        g.mlp_stats()
    ms = time_steps(torch, g, steps)
    stats = g.mlp_stats() if net is not None else (0, 0)
    g.profile(True)
    g.step(steps)
    launches, kms = g.profile_read()
    g.profile(False)
    _, finite = g.reduce()
    U = g.get_state()
    g.close()
    return {"ms": ms, "launches": launches, "kms": kms, "finite": finite, "tiles": tiles, "stats": stats, "U": U}


# Filter coefficient of the Taylor-Green runs of Sec. 5.2.
FILTER_ALPHA = 0.499

# The learned halo runs only if, on held-out training samples, it lowers the
# mean squared halo error of the AT extrapolation by at least this fraction.
MLP_ACCEPT_DELTA = 0.1


def train_halo_net(torch, w, dt, tau=10.0):
    """The learned halo's network, trained on FP64 synchronous Taylor-Green
    runs the solver generates at 256^3 in 16x16x8 blocks with the run's dt
    (the network is the library's; its training kernels run on the GPU)."""
    tw = dict(inputs.WORKLOADS["tgv_256"], mode="sa", L=w["L"])
    tr = make_solver(tw, atns.F64)
    tr.set_dt(dt)
    tr.init_case(atns.CASE_TGV)
    tr.step(C_LEVELS + w["L"] + 2)
    tr.mlp_set_scales(np.ones(5), np.ones(5))
    X, Y = tr.mlp_sample(8192, 1)
    X, Y = X.double().cpu().numpy(), Y.double().cpu().numpy()
    s = (np.sqrt((X[:, :60].reshape(-1, 4, 5, 3) ** 2).mean(axis=(0, 1, 3))) + 1e-30).astype(np.float32)
    r = (np.sqrt((Y[:, :5] ** 2).mean(axis=0)) + 1e-30).astype(np.float32)
    tr.mlp_set_scales(s, r)
    rng = np.random.default_rng(0)
    theta0 = np.concatenate([rng.standard_normal(64 * 64) * math.sqrt(2.0 / 64), np.zeros(64),
                             rng.standard_normal(64 * 64) * math.sqrt(2.0 / 64), np.zeros(64),
                             rng.standard_normal(16 * 64) * math.sqrt(2.0 / 64), np.zeros(16)])
    tr.mlp_set_params((0.5 * theta0).astype(np.float32))
    losses = []
    t0 = time.perf_counter()
    for rnd in range(6):
        tr.step(2)
        losses.extend(tr.mlp_train(100, 1024, 1e-3, 100 + rnd).tolist())
    train_s = time.perf_counter() - t0
    theta = tr.mlp_get_params()
    Xv, Yv = tr.mlp_sample(4096, 999)
    out = tr.mlp_forward(Xv)[:, :5].double().cpu().numpy()
    Yn = Yv[:, :5].double().cpu().numpy()
    tr.close()
    return {"theta": theta, "s": s, "r": r, "tau": tau,
            "training": {"grid": list(tw["n"]), "blocks": list(tw["nblk"]), "precision": "f64", "mode": "sa",
                         "iters": len(losses), "batch": 1024, "seconds": train_s,
                         "loss_first10": float(np.mean(losses[:10])), "loss_last50": float(np.mean(losses[-50:])),
                         "halo_mse_at": float((Yn ** 2).mean()), "halo_mse_mlp": float(((out - Yn) ** 2).mean())}}


PROBE_BYTES = 1 << 30


def hbm_probe(torch, reps=10):
    """Achievable HBM bandwidth from the library's streaming copy of 1 GiB
    (read + write counted)."""
    src = torch.empty(PROBE_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1.0)
    atns.hbm_probe(src, dst, PROBE_BYTES)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        atns.hbm_probe(src, dst, PROBE_BYTES)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"bytes_per_launch": 2 * PROBE_BYTES, "ms": ms, "GBps": 2 * PROBE_BYTES / (ms * 1e-3) / 1e9}


def kernel_source_hash():
    """Hash of the device-code sources (.hip files and the headers they
    include): stored counter results apply only to it."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2506_03027_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp")):
            h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()[:16]


def stored_traffic(workload):
    """Per-launch HBM traffic of the stage kernel from the committed counter
    summary, if it was taken with the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_hash") != kernel_source_hash():
        return None
    return rec.get("traffic_bytes_per_launch")


def traffic_summary(workload, fetch_db, write_db, commands):
    """The counter record profiles/traffic_<workload>.json from two rocprofv3
    runs of this script (--pmc FETCH_SIZE, then --pmc WRITE_SIZE, KiB per
    dispatch): the stage kernel's average per launch and the halo kernel's
    per step, each counter scaled by what it reads for the copy probe's 1 GiB
    copy (1 GiB fetched and 1 GiB written)."""
    import sqlite3

    def per_kernel(db, counter):
        # keyed by (kernel name, workgroups): the tile autotuner launches the
        # stage kernel at other tile shapes and sizes before the timed steps
        c = sqlite3.connect(db)
        rows = c.execute("select kernel_name, grid_size / workgroup_size, dispatch_id, sum(value) "
                         "from counters_collection where counter_name = ? "
                         "group by kernel_name, dispatch_id", (counter,)).fetchall()
        out = {}
        for name, wg, _, v in rows:
            out.setdefault((name.split("(")[0], wg), []).append(v)
        return out

    f, wr = per_kernel(fetch_db, "FETCH_SIZE"), per_kernel(write_db, "WRITE_SIZE")
    pick = lambda d, key: [v for k, vs in d.items() if key in k[0] for v in vs]
    probe_kib = PROBE_BYTES / 1024.0
    fprobe, wprobe = np.mean(pick(f, "copy_probe_kernel")), np.mean(pick(wr, "copy_probe_kernel"))
    fs, ws = probe_kib / fprobe, probe_kib / wprobe
    w = inputs.WORKLOADS[workload]
    kname = "ns_stage_kernel" if w["physics"] == "ns" else "euler_stage_kernel"
    # the benchmark's tile shape and launch size: the group with most dispatches
    groups = {}
    for (k, wg), vs in f.items():
        if kname in k:
            shape = ", ".join(k.split("<", 1)[1].split(">", 1)[0].split(", ")[:3])
            groups.setdefault((shape, wg), []).append(((k, wg), vs))
    best = max(groups, key=lambda g: sum(len(vs) for _, vs in groups[g]))
    per_kind = {}
    fall, wall = [], []
    for key, vs in groups[best]:
        kind = key[0].split("<", 1)[1].split(">", 1)[0]
        per_kind[kind] = {"fetch_kib_raw": float(np.mean(vs)), "dispatches": len(vs),
                          "write_kib_raw": float(np.mean(wr.get(key, [0.0])))}
        fall += vs
        wall += wr.get(key, [])
    fk, wk = np.mean(fall), np.mean(wall)
    npts = w["n"][0] * w["n"][1] * w["n"][2]
    stages = n_stages(w)
    halo = [(a, b) for a, b in zip(pick(f, "halo_kernel"), pick(wr, "halo_kernel"))]
    rec = {"workload": workload, "kernel": "%s<%s> at %d workgroups" % (kname, best[0], best[1]),
           "kernel_hash": kernel_source_hash(), "commands": commands,
           "run_from": "/tmp, with TMPDIR=/tmp", "copy_probe_kib": probe_kib,
           "copy_probe_fetch_kib_raw": float(fprobe), "copy_probe_write_kib_raw": float(wprobe),
           "fetch_scale": fs, "write_scale": ws,
           "fetch_kib_raw_per_dispatch": float(fk), "write_kib_raw_per_dispatch": float(wk), "per_kind": per_kind,
           "traffic_bytes_per_launch": float((fk * fs + wk * ws) * 1024.0),
           "algorithmic_bytes_per_launch": stage_kernel_bytes_per_point(w, stages, 4) * npts}
    if halo:
        rec["halo_kernel_per_step_bytes"] = float(np.mean([(a * fs + b * ws) * 1024.0 for a, b in halo]))
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    with open(path, "w") as fo:
        json.dump(rec, fo, indent=1)
    print(json.dumps({"written": path, "traffic_bytes_per_launch": rec["traffic_bytes_per_launch"],
                      "algorithmic_bytes_per_launch": rec["algorithmic_bytes_per_launch"]}))


SQ_COUNTERS = {
    "a": ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR",
          "SQ_BUSY_CYCLES", "SQ_WAIT_INST_ANY"],
    "b": ["SQ_WAVE_CYCLES", "SQ_ACTIVE_INST_ANY", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS", "SQ_WAIT_ANY",
          "SQ_INST_CYCLES_VMEM_RD", "SQ_LDS_BANK_CONFLICT", "SQ_THREAD_CYCLES_VALU"],
}


def sq_summary(workload, dbs, commands):
    """The counter record profiles/sq_<workload>.json of the stage kernel at
    the benchmark's tile shape and launch size, from two rocprofv3 --pmc runs
    of this script (counter sets SQ_COUNTERS a and b): per-launch averages of
    each counter, the same per owned point, and ratios that say where the
    waves' time goes."""
    import sqlite3
    w = inputs.WORKLOADS[workload]
    npts = w["n"][0] * w["n"][1] * w["n"][2]
    kname = "ns_stage_kernel" if w["physics"] == "ns" else "euler_stage_kernel"
    vals, chosen = {}, None
    for db in dbs:
        c = sqlite3.connect(db)
        rows = c.execute("select kernel_name, grid_size / workgroup_size, dispatch_id, counter_name, sum(value) "
                         "from counters_collection group by kernel_name, dispatch_id, counter_name").fetchall()
        groups = {}
        for name, wg, disp, cn, v in rows:
            if kname not in name:
                continue
            shape = ", ".join(name.split("<", 1)[1].split(">", 1)[0].split(", ")[:3])
            groups.setdefault((shape, wg), {}).setdefault(cn, {})[disp] = v
        best = max(groups, key=lambda g: max(len(d) for d in groups[g].values()))
        chosen = chosen or best
        for cn, d in groups[best].items():
            vals[cn] = float(np.mean(list(d.values())))
    per_pt = {cn: v / npts for cn, v in vals.items()}
    ratios = {}
    if "SQ_WAVE_CYCLES" in vals:
        wc = vals["SQ_WAVE_CYCLES"]
        for cn in ("SQ_ACTIVE_INST_ANY", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS", "SQ_WAIT_ANY",
                   "SQ_WAIT_INST_ANY"):
            if cn in vals:
                ratios[cn + "/SQ_WAVE_CYCLES"] = vals[cn] / wc
    rec = {"workload": workload, "kernel": "%s<%s> at %d workgroups, all stage kinds" % (kname, chosen[0], chosen[1]),
           "kernel_hash": kernel_source_hash(), "commands": commands, "run_from": "/tmp, with TMPDIR=/tmp",
           "owned_points": npts, "per_launch": vals, "per_owned_point": per_pt, "ratios": ratios}
    path = os.path.join(ROOT, "profiles", "sq_%s.json" % workload)
    with open(path, "w") as fo:
        json.dump(rec, fo, indent=1)
    print(json.dumps({"written": path, "ratios": ratios,
                      "valu_per_point": per_pt.get("SQ_INSTS_VALU")}))


def trace_summary(db, top=14):
    """Markdown summary of a rocprofv3 --kernel-trace database: calls, total
    and average duration (microseconds) per kernel and launch size
    (workgroups). A run on a fresh node tunes the tile shape first and
    launches the stage kernel at several shapes and sizes; those launches
    are totalled on one line, and the table keeps the stage kernel at the
    shape and size most used (the benchmark's) beside every other kernel."""
    import sqlite3
    c = sqlite3.connect(db)
    rows = c.execute("select name, grid_x / workgroup_x, count(*), sum(duration), avg(duration) from kernels "
                     "group by name, grid_x / workgroup_x").fetchall()

    def shape_of(name):
        args = name.split("<", 1)[1].split(">", 1)[0].split(", ")
        return ", ".join(args[:3])

    chosen, tuning = {}, []
    for key in ("ns_stage_kernel", "euler_stage_kernel"):
        sel = [r for r in rows if key in r[0]]
        if not sel:
            continue
        groups = {}
        for r in sel:
            groups.setdefault((shape_of(r[0]), r[1]), []).append(r)
        best = max(groups, key=lambda g: sum(r[2] for r in groups[g]))
        chosen[key] = (best, groups[best])
        tuning += [r for g, rs in groups.items() if g != best for r in rs]
    kept = [r for r in rows if r not in tuning]
    tot = sum(r[3] for r in kept)
    kept.sort(key=lambda r: -r[3])
    lines = ["| kernel | workgroups | calls | total us | average us | % |", "|---|---|---|---|---|---|"]
    for name, wg, n, t, a in kept[:top]:
        lines.append("| `%s` | %d | %d | %.1f | %.3f | %.1f |" % (name.split("(")[0], wg, n, t / 1e3, a / 1e3,
                                                                 100.0 * t / tot))
    if tuning:
        lines.append("")
        lines.append("Tile tuning (stage kernel at other shapes and sizes, not in the table): %d launches, %.1f us." % (
            sum(r[2] for r in tuning), sum(r[3] for r in tuning) / 1e3))
    for key, ((shape, wg), grp) in chosen.items():
        n = sum(r[2] for r in grp)
        t = sum(r[3] for r in grp)
        lines.append("")
        lines.append("`%s<%s>` at %d workgroups, all stage kinds: %d calls, average %.3f us per launch." % (
            key, shape, wg, n, t / n / 1e3))
        for r in sorted(grp, key=lambda r: r[0]):
            lines.append("- `%s`: %d calls, average %.3f us" % (r[0].split("(")[0], r[2], r[4] / 1e3))
    print("\n".join(lines))


def host_info():
    """CPU model and core counts of the host the oracle is timed on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0))}


def oracle_sample(w):
    """The bounded oracle sample of a workload: the same block shape, halo
    scheme and delays on a grid of two blocks per axis (at most 64 points),
    started from a delayed history so that every timed step is asynchronous.
    Returns (config, history {step: field}, dt, first timed step)."""
    from oracle import solver
    blk = [w["n"][d] // w["nblk"][d] for d in range(3)]
    n = tuple(w["n"][d] if w["n"][d] <= 64 else max(64, 2 * blk[d]) for d in range(3))
    nblk = tuple(n[d] // blk[d] for d in range(3))
    length = w["length"]
    C = n_levels(w)
    cfg = solver.Config(n, length, w["ndim"], nblk, w["physics"], mach=w.get("mach", 0.1),
                        re=w.get("re", 1600.0), rk=w["rk"], mode=w["mode"], algo=w.get("algo", "saa"),
                        L=w["L"], seed=w.get("seed", 1), C=C, order=2 if w["rk"] == "lserk2" else 4)
    s = dict(w, n=n, nblk=nblk)
    U0 = initial_state(s)
    dt = inputs.cfl_dt(U0, n, length, w["ndim"], 1.4, w["cfl"])
    cfg.dt = dt
    D = C + 2 * w["L"] - 1           # the library's ring depth in the asynchronous modes
    n0 = 2 * D
    hist = {}
    if w["physics"] == "ns":
        # the Taylor-Green field plus smooth perturbations that vary in time
        g1 = 0.02 * (inputs.smooth_random_state(n, length, seed=41) - 1.0)
        g2 = 0.02 * (inputs.smooth_random_state(n, length, seed=42) - 1.0)
        for m in range(n0 - D + 1, n0 + 1):
            hist[m] = U0 + math.sin(0.3 * (m - n0)) * g1 + (1.0 - math.cos(0.3 * (m - n0))) * g2
    else:
        for m in range(n0 - D + 1, n0 + 1):
            hist[m] = inputs.vortex_state(n, length, w["ndim"], t=(m - n0) * dt)
    return cfg, s, hist, dt, n0


def _oracle_steps(args):
    """Worker: run `steps` oracle steps of the sample; (steps, seconds)."""
    w, steps = args
    from oracle import solver
    cfg, _, hist, _, _ = oracle_sample(w)
    o = solver.Oracle(cfg)
    for m in sorted(hist):
        o.set_state(hist[m], step=m)
    t0 = time.perf_counter()
    o.step(steps)
    return steps, time.perf_counter() - t0


def cpu_oracle_timing(w, budget_s=15.0):
    """The FP64 oracle on a bounded sample of the workload (oracle_sample):
    first on one host core until budget_s, then as independent copies on
    every usable core at once (the oracle itself is single-threaded).  Runs
    before the process touches the GPU, so the worker processes it forks
    inherit no device state.  Returns the record and the oracle's final
    state for the GPU comparison (cpu_baseline_l2)."""
    from oracle import solver
    import multiprocessing as mp
    cfg, s, hist, dt, n0 = oracle_sample(w)
    n = cfg.n
    stages = n_stages(w)
    npts = n[0] * n[1] * n[2]
    o = solver.Oracle(cfg)
    for m in sorted(hist):
        o.set_state(hist[m], step=m)
    t0 = time.perf_counter()
    done = 0
    while done < 1 or (time.perf_counter() - t0 < budget_s and done < 64):
        o.step(1)
        done += 1
    elapsed = time.perf_counter() - t0
    one = npts * stages * done / elapsed
    info = host_info()
    procs = max(1, min(16, info["usable_cpus"]))
    k = max(1, done // 2)
    t1 = time.perf_counter()
    with mp.get_context("fork").Pool(procs) as pool:
        pool.map(_oracle_steps, [(w, k)] * procs)
    wall = time.perf_counter() - t1
    allc = npts * stages * k * procs / wall
    sample = ("%s grid %dx%dx%d in %d blocks of %dx%dx%d (the workload's blocks), %s L=%d, asynchronous "
              "RK steps from a delayed history, FP64 numpy oracle" % (
                  w["physics"], n[0], n[1], n[2], cfg.nblk[0] * cfg.nblk[1] * cfg.nblk[2],
                  n[0] // cfg.nblk[0], n[1] // cfg.nblk[1], n[2] // cfg.nblk[2], w.get("algo", "saa").upper(),
                  w["L"]))
    rec = {"value": allc, "unit": "grid-point-stage/s", "cores": procs, "kind": "oracle",
           "sample": sample + "; %d copies at once, one per core, %d steps each" % (procs, k),
           "seconds": wall, "host": info,
           "one_core": {"value": one, "cores": 1, "steps": done, "seconds": elapsed}}
    return rec, o.U, done


def cpu_baseline_l2(torch, w, U_oracle, steps):
    """The oracle sample run through the FP32 GPU path: relative L2 and L-inf
    against the oracle's state after the same steps."""
    cfg, s, hist, dt, n0 = oracle_sample(w)
    g = make_solver(s, atns.F32)
    g.set_dt(dt)
    for m in sorted(hist):
        g.set_state(torch.from_numpy(hist[m]), step=m)
    g.step(steps)
    G = g.get_state().double().cpu().numpy()
    g.close()
    return {"fp32_gpu_rel_l2_vs_oracle": float(np.linalg.norm(G - U_oracle) / np.linalg.norm(U_oracle)),
            "fp32_gpu_rel_linf_vs_oracle": float(np.abs(G - U_oracle).max() / np.abs(U_oracle).max())}


def solver_kwargs(w):
    return dict(n=w["n"], length=w["length"], ndim=w["ndim"], nblk=w["nblk"], split=w.get("split"),
                physics=atns.NS if w["physics"] == "ns" else atns.EULER, mach=w.get("mach", 0.1),
                re=w.get("re", 1600.0), rk=atns.RK4, mode=atns.AT,
                algo=atns.SAA if w.get("algo", "saa") == "saa" else atns.CAA, L=w["L"],
                seed=w.get("seed", 1), precision=atns.F32)


def start_instance(s, w):
    """Analytic initial field computed on the device; dt from the CFL number
    with the wave speeds sampled on a 64-point-per-axis copy of the field."""
    ns = w["physics"] == "ns"
    coarse = tuple(min(64, x) for x in w["n"])
    Uc = inputs.tgv_state(coarse, mach=w.get("mach", 0.1)) if ns else inputs.vortex_state(coarse, w["length"], 3)
    dt = inputs.cfl_dt(Uc, w["n"], w["length"], 3, 1.4, w["cfl"])
    s.set_dt(dt)
    s.init_case(atns.CASE_TGV if ns else atns.CASE_VORTEX)


def batch_main(a, torch):
    """Batched persistent launch: every step of all instances is one graph
    launch; compared with the sum of the same instances run one by one."""
    ws = inputs.batch_instances()
    stages = 4
    pts = [w["n"][0] * w["n"][1] * w["n"][2] for w in ws]
    total = sum(pts)
    b = atns.Batch([solver_kwargs(w) for w in ws])
    for m, w in zip(b.members, ws):
        start_instance(m, w)
    b.step(C_LEVELS + 1)
    eu, nst = b.autotune(reps=10)
    b.step(a.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.step(a.steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    finite = all(m.reduce()[1] for m in b.members)
    b.close()
    solo_ms = 0.0
    for w in ws:
        s = atns.Solver(**solver_kwargs(w))
        start_instance(s, w)
        s.step(C_LEVELS + 1)
        s.autotune(reps=10, cache=TUNE_CACHE)
        s.step(a.warmup)
        solo_ms += time_steps(torch, s, a.steps)
        s.close()
    bytes_step = sum(algorithmic_bytes_per_point_stage(w, stages, 4)[0] * p for w, p in zip(ws, pts)) * stages
    achieved = bytes_step / (ms / a.steps * 1e-3) / 1e9
    out = {
        "metric": "grid-point-stage updates/s (FP32 AT vs FP64 SA)",
        "value": total * stages * a.steps / (ms * 1e-3),
        "unit": "grid-point-stage/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup + C_LEVELS + 1,
        "ms_per_step": ms / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batch48", "instances": len(ws), "points": total,
                   "blocks": sum(w["nblk"][0] * w["nblk"][1] * w["nblk"][2] for w in ws),
                   "euler": sum(1 for w in ws if w["physics"] == "euler"),
                   "scheme": "CD4 + AT halos, RK4", "algo": "SAA", "L": sorted({w["L"] for w in ws}),
                   "tiles": {"euler": list(eu), "ns": list(nst)}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "whole step (euler_batch_kernel, ns_batch_kernel, halo kernels)",
                     "basis": "algorithmic bytes of all instances per step / graph-launch time per step"},
        "finite": finite,
        "solo_sum": {"value": total * stages * a.steps / (solo_ms * 1e-3), "ms_per_step": solo_ms / a.steps,
                     "note": "each instance alone, own autotuned tiles, graph-captured steps"},
        "batch_vs_solo_sum": solo_ms / ms,
        "kernel_hash": kernel_source_hash(),
    }
    print(json.dumps(out))


def free_running_main(a, torch):
    """Free-running asynchronous steps (delays realized by the run) against
    the scheduled SAA steps of the same workload and tiles, both FP32 from
    the same warm state; the free-running run is then replayed on the
    scheduled path with its logged delays, and the two results compared."""
    w = inputs.WORKLOADS[a.workload]
    stages = n_stages(w)
    npts = w["n"][0] * w["n"][1] * w["n"][2]
    U0 = initial_state(w)
    dt = inputs.cfl_dt(U0, w["n"], w["length"], w["ndim"], 1.4, w["cfl"])
    warmup = max(a.warmup, n_levels(w) + w["L"])

    def start():
        g = make_solver(w, atns.F32)
        g.set_dt(dt)
        g.set_state(torch.from_numpy(U0))
        tiles = g.autotune(reps=10, cache=TUNE_CACHE)
        g.step(warmup)
        return g, tiles

    g, tiles = start()
    ms_sched = time_steps(torch, g, a.steps)
    g.close()
    # tile shape of the free-running kernel: one workgroup walks all tiles of
    # its block, so the best shape differs from the scheduled one; the
    # fastest of a few over 5 steps
    bx = w["n"][0] // w["nblk"][0]
    best = None
    cands = (((16, 16, 32), (16, 8, 32), (32, 8, 32), (16, 16, 16)) if w["physics"] == "ns"
             else ((32, 16, 32), (32, 16, 16), (16, 16, 16), (16, 16, 8)))
    for sh in cands:
        if sh[0] > bx:
            continue
        g, _ = start()
        g.set_tiles(*sh)
        g.step_async(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step_async(5)
        el = time.perf_counter() - t0
        g.close()
        if best is None or el < best[0]:
            best = (el, sh)
    free_tiles = best[1]
    g, _ = start()
    g.set_tiles(*free_tiles)
    log0 = g.step_async(2)               # first launch (code load) outside the timing
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    log = g.step_async(a.steps)
    e1.record()
    torch.cuda.synchronize()
    ms_free = e0.elapsed_time(e1)
    A = g.get_state().double()
    g.close()
    r, _ = start()
    r.set_tiles(*free_tiles)
    r.set_delays(warmup, np.concatenate([log0, log]))
    r.step(2 + a.steps)
    B = r.get_state().double()
    r.close()
    used = log[log >= 0]
    hist = np.bincount(used.ravel(), minlength=w["L"]).tolist()
    out = {
        "metric": "grid-point-stage updates/s (FP32, free-running asynchronous steps)",
        "value": npts * stages * a.steps / (ms_free * 1e-3),
        "unit": "grid-point-stage/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": warmup + 2,
        "ms_per_step": ms_free / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": a.workload, "grid": list(w["n"]), "blocks": list(w["nblk"]),
                   "physics": w["physics"], "rk": w["rk"], "mode": w["mode"], "L": w["L"],
                   "tiles": list(free_tiles), "scheduled_tiles": list(tiles),
                   "workgroups": int(np.prod(w["nblk"]))},
        "scheduled_saa": {"value": npts * stages * a.steps / (ms_sched * 1e-3), "ms_per_step": ms_sched / a.steps},
        "realized_delays": {"histogram": hist, "mean": float(used.mean())},
        "replay_rel_max": float((A - B).abs().max() / B.abs().max()),
        "kernel_hash": kernel_source_hash(),
    }
    print(json.dumps(out))


def series_main(a, torch):
    """The workload run for a.series steps with the FP64 diagnostics (conserved
    totals, kinetic energy, enstrophy) reduced on the GPU after every step; or,
    with a.series_t, run to that time with the diagnostics every a.series
    steps (the Taylor-Green runs of Sec. 5.2 through the dissipation peak,
    with the filter when a.series_filter)."""
    w = inputs.WORKLOADS[a.workload]
    if a.series_cfl:
        w = dict(w, cfl=a.series_cfl)
    if a.series_L:
        w = dict(w, L=a.series_L)
    if a.series_mode:
        w = dict(w, mode=a.series_mode, L=w["L"] if a.series_mode != "sa" else 1)
    alpha = FILTER_ALPHA if a.series_filter else None
    g = make_solver(w, atns.F64 if a.series_f64 else atns.F32, filter_alpha=alpha)
    n = w["n"]
    coarse = tuple(min(64, x) for x in n)
    U0 = (inputs.tgv_state(coarse, mach=w.get("mach", 0.1)) if w["physics"] == "ns"
          else inputs.vortex_state(coarse, w["length"], w["ndim"]))
    dt = inputs.cfl_dt(U0, n, w["length"], w["ndim"], 1.4, w["cfl"])
    every = max(1, a.series) if a.series_t else 1
    nsteps = int(math.ceil(a.series_t / dt)) if a.series_t else a.series
    g.set_dt(dt)
    g.init_case(atns.CASE_TGV if w["physics"] == "ns" else atns.CASE_VORTEX)
    g.autotune(reps=10, cache=TUNE_CACHE)
    rows = [(0, 0.0) + tuple(g.reduce()[0])]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    finite = True
    s = 0
    report = max(every, nsteps // 20)
    while s < nsteps:
        k = min(every, nsteps - s)
        g.step(k)
        s += k
        d, ok = g.reduce()
        finite = finite and ok
        rows.append((s, s * dt) + tuple(d))
        if s % report < every:
            print("[series] %s step %d t %.4f K %.6g" % (w["mode"], s, s * dt, d[5]), file=sys.stderr, flush=True)
        if not ok:
            break
    wall = time.perf_counter() - t0
    g.close()
    R = np.array(rows)
    ref = None
    if a.series_ref:
        # the same series from the FP64 synchronous solver (the scheme without
        # delays or FP32 rounding), step for step
        def sa_series(precision):
            r = make_solver(dict(w, mode="sa", L=1), precision, filter_alpha=alpha)
            r.set_dt(dt)
            r.init_case(atns.CASE_TGV if w["physics"] == "ns" else atns.CASE_VORTEX)
            rr = [tuple(r.reduce()[0])]
            step_report = max(1, (len(rows) - 1) // 20)
            for i in range(1, len(rows)):
                r.step(int(rows[i][0] - rows[i - 1][0]))
                rr.append(tuple(r.reduce()[0]))
                if i % step_report == 0:
                    print("[series] sa %s step %d" % ("f64" if precision == atns.F64 else "f32", int(rows[i][0])),
                          file=sys.stderr, flush=True)
            r.close()
            return np.array(rr)

        Q = sa_series(atns.F64)
        Q32 = sa_series(atns.F32)
        ref = {"solver": "FP64 synchronous (SA), same grid and dt",
               "max_rel_diff_kinetic_energy": float(np.abs(R[:, 7] - Q[:, 5]).max() / abs(Q[0, 5])),
               "max_rel_diff_enstrophy": float(np.abs(R[:, 8] - Q[:, 6]).max() / abs(Q[0, 6])),
               "kinetic_energy_end": float(Q[-1, 5]), "enstrophy_end": float(Q[-1, 6]),
               "fp32_sa_max_rel_diff_kinetic_energy": float(np.abs(Q32[:, 5] - Q[:, 5]).max() / abs(Q[0, 5])),
               "fp32_sa_max_rel_diff_enstrophy": float(np.abs(Q32[:, 6] - Q[:, 6]).max() / abs(Q[0, 6]))}
    if a.series_out:
        hdr = "step,t,mass,mom_x,mom_y,mom_z,energy,kinetic_energy,enstrophy"
        np.savetxt(a.series_out, R, delimiter=",", header=hdr, comments="")
        if ref:
            # the FP64 synchronous series beside it, same steps
            root, ext = os.path.splitext(a.series_out)
            np.savetxt(root + "_sa_f64" + (ext or ".csv"), np.hstack([R[:, :2], Q]), delimiter=",", header=hdr,
                       comments="")
    K, E = R[:, 7], R[:, 8]
    out = {"workload": a.workload, "steps": int(R[-1, 0]), "dt": dt, "t_end": float(R[-1, 1]),
           "mode": w["mode"], "L": w["L"], "precision": "f64" if a.series_f64 else "f32", "cfl": w["cfl"],
           "filter_alpha": alpha, "reductions_every": every,
           "finite": bool(finite), "wall_s_with_per_step_reductions": wall,
           "kinetic_energy": {"t0": float(K[0]), "end": float(K[-1]),
                              "monotone_nonincreasing": bool(np.all(np.diff(K) <= 1e-12 * K[0]))},
           "enstrophy": {"t0": float(E[0]), "end": float(E[-1]), "max": float(E.max())},
           "mass_rel_drift": float(abs(R[-1, 2] - R[0, 2]) / abs(R[0, 2])),
           "energy_rel_drift": float(abs(R[-1, 6] - R[0, 6]) / abs(R[0, 6]))}
    if every == 1 and len(R) > 200:
        out["dK_dt_fit_first_200_steps"] = float(np.polyfit(R[:201, 1], K[:201], 1)[0])
    if w["physics"] == "ns":
        # viscous dissipation 2 (1/Re) * enstrophy, and its peak
        re = w.get("re", 1600.0)
        i = int(np.argmax(E))
        out["dissipation_peak"] = {"t": float(R[i, 1]), "value": float(2.0 * E[i] / re)}
        if ref:
            j = int(np.argmax(Q[:, 6]))
            ref["dissipation_peak"] = {"t": float(R[j, 1]), "value": float(2.0 * Q[j, 6] / re)}
            ref["max_abs_diff_dissipation_over_peak"] = float(np.abs(E - Q[:, 6]).max() / Q[:, 6].max())
            ref["max_abs_diff_kinetic_energy_over_k0"] = float(np.abs(K - Q[:, 5]).max() / Q[0, 5])
    if ref:
        out["reference"] = ref
    print(json.dumps(out))


METRIC = "grid-point\u00b7RK-stage updates/s, FP32 AT(+MLP) vs FP64 plain, at stated L2 err"


def coarse_dt(w):
    """dt from the CFL number, with the wave speeds sampled on a copy of the
    initial field at most 64 points per axis (the field is analytic)."""
    coarse = tuple(min(64, x) for x in w["n"])
    if w["physics"] == "ns":
        Uc = inputs.tgv_state(coarse, mach=w.get("mach", 0.1))
    else:
        Uc = inputs.vortex_state(coarse, w["length"], w["ndim"])
    return inputs.cfl_dt(Uc, w["n"], w["length"], w["ndim"], 1.4, w["cfl"])


def equal_accuracy(torch, w, dt, total, U_ref):
    """Discretization error of the FP64 synchronous solution, estimated from
    the same run on the grid coarsened by 2 (twice the step, half the steps;
    the initial field is analytic): e_h ~ |U_2h - U_h| / (2^4 - 1) for a
    fourth-order scheme in space and time."""
    n2 = tuple(x // 2 for x in w["n"])
    if any(x % 2 for x in w["n"]) or total % 2 or min(n2[d] // w["nblk"][d] for d in range(w["ndim"])) < 4:
        return None
    w2 = dict(w, n=n2)
    g = make_solver(dict(w2, mode="sa", L=1), atns.F64)
    g.set_dt(2 * dt)
    g.init_case(atns.CASE_TGV if w["physics"] == "ns" else atns.CASE_VORTEX)
    g.step(total // 2)
    U2 = g.get_state()
    g.close()
    sub = U_ref[:, ::2, ::2, ::2] if w["ndim"] == 3 else U_ref[:, :, ::2, ::2]
    e2h = float(torch.linalg.vector_norm(U2 - sub) / torch.linalg.vector_norm(sub))
    return {"grid_2h": list(n2), "rel_l2_2h_vs_h": e2h, "fp64_sa_disc_err_est": e2h / 15.0}


# Errors against the exact solution within this relative margin of each
# other count as equal accuracy.
EQUAL_ACCURACY_TOL = 0.05


def equal_accuracy_vortex(torch):
    """FP32 AT against FP64 SA where an exact solution exists: the 3-D
    isentropic vortex of the 128^3 Euler workload (4 x 4 x 4 blocks of 32^3,
    SAA L = 4) advanced to T = 1, FP32 AT plain and with compensated steps.
    Every run is compared with the translated exact field; where an FP32
    run's error equals FP64 SA's, the ratio of their step times is a speed-up
    at equal accuracy."""
    w = inputs.WORKLOADS["vortex3d_128"]
    nsteps = int(math.ceil(1.0 / coarse_dt(w)))
    dt = 1.0 / nsteps
    exact = inputs.vortex_state(w["n"], w["length"], 3, t=1.0)
    en = float(np.linalg.norm(exact))
    res = {"workload": "vortex3d_128", "T": 1.0, "steps": nsteps, "dt": dt,
           "reference": "exact translated vortex (periodic images not included)"}
    for key, prec, mode, comp in (("fp32_at", atns.F32, "at", False), ("fp32_at_compensated", atns.F32, "at", True),
                                  ("fp64_sa", atns.F64, "sa", False)):
        g = make_solver(w, prec, mode)
        g.set_compensation(comp)
        g.set_dt(dt)
        g.init_case(atns.CASE_VORTEX)
        g.autotune(reps=5, cache=TUNE_CACHE)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.step(nsteps)
        e1.record()
        torch.cuda.synchronize()
        U = g.get_state().double().cpu().numpy()
        g.close()
        res[key] = {"ms_per_step": e0.elapsed_time(e1) / nsteps,
                    "rel_l2_vs_exact": float(np.linalg.norm(U - exact)) / en}
    es = res["fp64_sa"]["rel_l2_vs_exact"]
    for key in ("fp32_at", "fp32_at_compensated"):
        r = res[key]
        r["error_ratio_vs_fp64_sa"] = r["rel_l2_vs_exact"] / es
        r["equal_accuracy"] = abs(r["error_ratio_vs_fp64_sa"] - 1.0) <= EQUAL_ACCURACY_TOL
        r["speedup_vs_fp64_sa"] = res["fp64_sa"]["ms_per_step"] / r["ms_per_step"]
    res["equal_accuracy_tolerance"] = EQUAL_ACCURACY_TOL
    best = [k for k in ("fp32_at", "fp32_at_compensated") if res[k]["equal_accuracy"]]
    res["speedup_at_equal_accuracy"] = max(res[k]["speedup_vs_fp64_sa"] for k in best) if best else None
    return res


def headline_main(a, torch, cpu):
    """FP32 AT (the metric), FP32 AT with the learned halo and FP64 SA on the
    workload from the same initial field, dt and step count; the L2 of each
    against FP64 SA; rooflines; the CPU baseline."""
    w = inputs.WORKLOADS[a.workload]
    stages = n_stages(w)
    npts = w["n"][0] * w["n"][1] * w["n"][2]
    ns = w["physics"] == "ns"
    dt = coarse_dt(w)
    U0 = None                                 # the analytic initial field, computed on the device
    warmup = max(a.warmup, n_levels(w) + 1)   # the first C steps are synchronous
    warmup += warmup % 2                      # an even total step count (equal_accuracy)
    total = warmup + 2 * a.steps

    at = run_path(torch, w, atns.F32, None, a.steps, warmup, dt, U0)
    value = npts * stages * a.steps / (at["ms"] * 1e-3)
    bpp, f = algorithmic_bytes_per_point_stage(w, stages, 4)
    kbpp = stage_kernel_bytes_per_point(w, stages, 4)
    avg_launch_ms = at["kms"] / max(1, at["launches"])
    achieved = kbpp * npts / (avg_launch_ms * 1e-3) / 1e9
    step_achieved = bpp * npts * stages * a.steps / (at["ms"] * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "grid-point-stage/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": warmup,
        "ms_per_step": at["ms"] / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": a.workload, "grid": list(w["n"]), "blocks": list(w["nblk"]),
                   "physics": w["physics"],
                   "scheme": "%s + %s halos, %s" % ("CD2" if w["rk"] == "lserk2" else "CD4", w["mode"].upper(),
                                                    w["rk"].upper()),
                   "algo": w.get("algo", "saa").upper(), "L": w["L"], "cfl": w["cfl"], "dt": dt,
                   "tiles": list(at["tiles"])},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": stored_traffic(a.workload),
                     "kernel": "%s_stage_kernel" % ("ns" if ns else "euler"),
                     "bytes_per_point_launch": kbpp, "halo_points_per_point": f,
                     "avg_launch_ms": avg_launch_ms, "launches": at["launches"],
                     "basis": "stage-kernel algorithmic bytes (state, RK register, one assembled halo value per "
                              "halo point, ring write) over the kernel's average launch time from HIP events",
                     "step": {"bytes_per_point_stage": bpp, "achieved": step_achieved,
                              "frac": step_achieved / HBM_PEAK_GBS,
                              "basis": "whole-step algorithmic bytes (C delayed levels per halo point and "
                                       "stage) over the graph-launch time per step"}},
        "finite": at["finite"],
    }
    U_at = at.pop("U")
    if ns and not a.no_filter:
        # the same steps with the tenth-order filter after each (Sec. 5.2's
        # alpha_f): one launch per step runs the three line-solve passes of
        # each block and variable and writes the filtered boundary layers to
        # the ring, which the last stage then leaves out
        fl = run_path(torch, w, atns.F32, None, a.steps, warmup, dt, U0, filter_alpha=FILTER_ALPHA)
        fl.pop("U")
        extra = (fl["ms"] - at["ms"]) / a.steps
        fbpp = filter_bytes_per_point(w)
        fbytes = fbpp * npts
        out["at_filtered"] = {"alpha": FILTER_ALPHA, "value": npts * stages * a.steps / (fl["ms"] * 1e-3),
                              "ms_per_step": fl["ms"] / a.steps, "filter_ms_per_step": extra,
                              "filter_bytes_per_point": fbpp, "filter_bytes_per_step": fbytes,
                              "filter_hbm_frac": (fbytes / (extra * 1e-3) / 1e9 / HBM_PEAK_GBS) if extra > 0 else None,
                              "basis": "the filter's algorithmic bytes per step (state in and out once, the "
                                       "filter halo values of the three passes, the ring write of the filtered "
                                       "boundary layers, the filter-halo slot the halo kernel writes) over the "
                                       "filtered step's extra time",
                              "finite": fl["finite"]}
    # the learned halo, trained on the GPU by the library's kernels
    U_mlp = None
    net = None
    if ns and w["rk"] == "rk4" and w["mode"] == "at" and not a.no_mlp:
        net = train_halo_net(torch, w, dt)
        tr = net["training"]
        ratio = tr["halo_mse_mlp"] / tr["halo_mse_at"]
        if not ratio < 1.0 - MLP_ACCEPT_DELTA and not a.force_mlp:
            # nothing to gain: the correction kernel is not run
            out["at_mlp"] = {"accepted": False, "halo_mse_ratio": ratio, "accept_delta": MLP_ACCEPT_DELTA,
                             "ms_per_step": at["ms"] / a.steps, "value": value,
                             "reason": "on held-out samples the trained network does not reduce the AT halo "
                                       "error by the acceptance margin at this time step (the extrapolation "
                                       "error is at the rounding level), so the step runs without it",
                             "training": tr}
            net = None
    if net is not None:
        ml = run_path(torch, w, atns.F32, None, a.steps, warmup, dt, U0, net=net)
        U_mlp = ml.pop("U")
        face_pts = (ml["stats"][0] + ml["stats"][1]) / a.steps
        flops = face_pts * 2.0 * (64 * 64 + 64 * 64 + 16 * 64)
        extra_ms = (ml["ms"] - at["ms"]) / a.steps
        tflops = flops / (extra_ms * 1e-3) / 1e12 if extra_ms > 0 else None
        out["at_mlp"] = {"accepted": not (net["training"]["halo_mse_mlp"] / net["training"]["halo_mse_at"] >=
                                          1.0 - MLP_ACCEPT_DELTA), "forced": bool(a.force_mlp),
                         "halo_mse_ratio": net["training"]["halo_mse_mlp"] /
                         net["training"]["halo_mse_at"], "accept_delta": MLP_ACCEPT_DELTA,
                         "value": npts * stages * a.steps / (ml["ms"] * 1e-3), "ms_per_step": ml["ms"] / a.steps,
                         "tau": net["tau"], "applied": ml["stats"][0], "fallback": ml["stats"][1],
                         "face_points_per_step": face_pts, "flops_per_step": flops,
                         "extra_ms_per_step": extra_ms, "achieved_tflops": tflops,
                         "mfma_frac_of_bf16_peak": (tflops / 2500.0) if tflops else None,
                         "training": net["training"]}
    if not a.no_eqvortex:
        out["equal_accuracy_vortex"] = equal_accuracy_vortex(torch)
    probe = hbm_probe(torch)
    out["hbm_probe"] = probe
    out["roofline"]["frac_of_probe"] = achieved / probe["GBps"]
    out["kernel_hash"] = kernel_source_hash()
    if not a.no_fp64:
        sa = run_path(torch, dict(w, mode="sa", L=1), atns.F64, "sa", a.steps, warmup, dt, U0)
        U_ref = sa.pop("U")
        b64 = stage_kernel_bytes_per_point(dict(w, mode="sa"), stages, 8)
        k64 = sa["kms"] / max(1, sa["launches"])
        out["fp64_sa"] = {"value": npts * stages * a.steps / (sa["ms"] * 1e-3), "ms_per_step": sa["ms"] / a.steps,
                          "avg_launch_ms": k64, "hbm_frac": b64 * npts / (k64 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          "tiles": list(sa["tiles"])}
        nrm = float(torch.linalg.vector_norm(U_ref))
        rel = lambda U: float(torch.linalg.vector_norm(U.double() - U_ref)) / nrm
        relinf = lambda U: float((U.double() - U_ref).abs().max() / U_ref.abs().max())
        l2 = {"steps": total, "reference": "FP64 synchronous GPU run, same grid, initial field and dt",
              "at": rel(U_at), "at_linf": relinf(U_at)}
        if U_mlp is not None:
            l2["at_mlp"] = rel(U_mlp)
            l2["at_mlp_linf"] = relinf(U_mlp)
            l2["at_mlp_minus_at"] = float(torch.linalg.vector_norm(U_mlp - U_at)) / nrm
        out["rel_l2_vs_fp64_sa"] = l2
        out["speedup_vs_fp64_sa"] = value / out["fp64_sa"]["value"]
        del U_at, U_mlp
        eq = equal_accuracy(torch, w, dt, total, U_ref)
        if eq is not None:
            eq["fp32_at_err_vs_fp64_sa"] = l2["at"]
            eq["ratio"] = l2["at"] / eq["fp64_sa_disc_err_est"]
            eq["equal_accuracy"] = eq["ratio"] <= 1.0
            if eq["equal_accuracy"]:
                eq["note"] = ("the FP32 AT path departs from the FP64 synchronous solution by less than the "
                              "latter's own discretization error, so speedup_vs_fp64_sa is a speed-up at equal "
                              "accuracy")
            else:
                eq["note"] = ("over this short horizon the FP64 synchronous solution's discretization error is "
                              "far below FP32 rounding: the FP32 AT path departs from it by `ratio` times that "
                              "error, so the two are not at equal accuracy and speedup_vs_fp64_sa compares equal "
                              "grids and time steps, not equal errors")
            out["equal_accuracy"] = eq
        del U_ref
    if cpu is not None:
        rec, U_or, steps_or = cpu
        rec.update(cpu_baseline_l2(torch, w, U_or, steps_or))
        out["cpu_baseline"] = rec
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=6)
    ap.add_argument("--workload", default="tgv_512")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-mlp", action="store_true", help="skip the learned-halo path")
    ap.add_argument("--no-filter", action="store_true", help="skip the filtered path")
    ap.add_argument("--no-eqvortex", action="store_true",
                    help="skip the equal-accuracy comparison on the vortex with an exact solution")
    ap.add_argument("--force-mlp", action="store_true",
                    help="run the learned halo even when the acceptance test rejects it (to measure its cost)")
    ap.add_argument("--series", type=int, default=0,
                    help="run this many steps with the FP64 diagnostics reduced after every step")
    ap.add_argument("--series-out", default=None, help="CSV file for --series")
    ap.add_argument("--series-ref", action="store_true",
                    help="with --series: also run the FP64 synchronous solver and compare the series")
    ap.add_argument("--series-t", type=float, default=None,
                    help="with --series: run to this time instead (--series then gives the steps between "
                         "reductions)")
    ap.add_argument("--series-cfl", type=float, default=None, help="with --series: CFL number of the run")
    ap.add_argument("--series-mode", choices=["at", "as", "sa"], default=None,
                    help="with --series: halo mode of the run (default: the workload's)")
    ap.add_argument("--series-L", type=int, default=None,
                    help="with --series: delay bound L of the run (delays up to L - 1)")
    ap.add_argument("--series-f64", action="store_true", help="with --series: the run in FP64")
    ap.add_argument("--series-filter", action="store_true",
                    help="with --series: the tenth-order filter (alpha_f = 0.499) after every step, on both "
                         "solvers")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_DB", "WRITE_DB"), default=None,
                    help="write profiles/traffic_<workload>.json from two rocprofv3 --pmc runs (FETCH_SIZE, "
                         "WRITE_SIZE) of this script; no GPU work")
    ap.add_argument("--traffic-commands", nargs="*", default=[], help="the two rocprofv3 commands, for the record")
    ap.add_argument("--sq-summary", nargs=2, metavar=("DB_A", "DB_B"), default=None,
                    help="write profiles/sq_<workload>.json from two rocprofv3 --pmc runs (SQ counter sets a, b)")
    ap.add_argument("--sq-set", choices=sorted(SQ_COUNTERS), default=None,
                    help="print the counters of one SQ set (for the rocprofv3 --pmc list) and exit")
    ap.add_argument("--trace-summary", default=None, metavar="DB",
                    help="print a markdown table of a rocprofv3 --kernel-trace database; no GPU work")
    ap.add_argument("--free-running", action="store_true",
                    help="free-running asynchronous steps (one persistent workgroup per block) next to the "
                         "scheduled graph-captured steps on the same workload")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (--gpus 1 only)",
              file=sys.stderr)
        sys.exit(2)
    if a.trace_summary:
        trace_summary(a.trace_summary)
        return
    if a.traffic_summary:
        traffic_summary(a.workload, a.traffic_summary[0], a.traffic_summary[1], a.traffic_commands)
        return
    if a.sq_set:
        print(" ".join(SQ_COUNTERS[a.sq_set]))
        return
    if a.sq_summary:
        sq_summary(a.workload, a.sq_summary, a.traffic_commands)
        return
    single = a.workload != "batch48" and not a.free_running and not a.series
    # the oracle's timing runs before anything touches the GPU (it forks workers)
    cpu = cpu_oracle_timing(inputs.WORKLOADS[a.workload]) if (single and not a.no_cpu) else None
    import torch
    torch.cuda.set_device(0)
    if a.workload == "batch48":
        batch_main(a, torch)
    elif a.free_running:
        free_running_main(a, torch)
    elif a.series:
        series_main(a, torch)
    else:
        headline_main(a, torch, cpu)


if __name__ == "__main__":
    main()
