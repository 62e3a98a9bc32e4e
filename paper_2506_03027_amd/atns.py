"""ctypes binding of libatns.so (include/atns.h).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch supplies device memory (tensors whose data_ptr() is passed through)
and the HIP stream.  If the library is missing this module raises at import
of the library (``lib()``) -- there is no fallback implementation.
"""
import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libatns.so")

EULER, NS = 0, 1
RK4, LSERK4, LSERK2 = 0, 1, 2
SA, AS, AT = 0, 1, 2
CAA, SAA = 0, 1
F32, F64 = 0, 1
CASE_VORTEX, CASE_TGV = 0, 1
NSLOTS = 18
NDIAG = 7
C_LEVELS = 5


def levels(rk):
    """Delayed levels C of the AT scheme paired with integrator rk: 5 (AT4)
    for RK4 and LSERK4, 3 (AT2) for LSERK2."""
    return 3 if rk == LSERK2 else 5


def stages(rk):
    return {RK4: 4, LSERK4: 5, LSERK2: 2}[rk]

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ESTATE", -5: "ENONFINITE"}

EXPORTS = ["atns_version", "atns_create", "atns_destroy", "atns_last_error", "atns_set_state",
           "atns_get_state", "atns_get_step", "atns_set_dt", "atns_set_delays", "atns_get_delays",
           "atns_rhs", "atns_rk_step", "atns_step_async", "atns_set_fusion", "atns_set_halo_fusion", "atns_set_filter_fusion", "atns_reduce", "atns_reduce_noalloc", "atns_get_layout", "atns_set_graphs", "atns_profile_enable",
           "atns_profile_read", "atns_set_tiles", "atns_get_tiles", "atns_autotune",
           "atns_mlp_set_params", "atns_mlp_get_params", "atns_mlp_set_scales", "atns_mlp_forward",
           "atns_mlp_grad", "atns_mlp_sample", "atns_mlp_train", "atns_mlp_enable", "atns_mlp_stats",
           "atns_hbm_probe", "atns_host_weights", "atns_host_delays", "atns_batch_create",
           "atns_batch_destroy", "atns_batch_last_error", "atns_batch_member", "atns_batch_set_tiles",
           "atns_batch_autotune", "atns_batch_step", "atns_init_case", "atns_checkpoint", "atns_restore",
           "atns_filter_state", "atns_host_filter_coefficients", "atns_set_compensation"]
MLP_PARAMS = 9360


class AtnsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("len", ctypes.c_double * 3),
                ("nblk", ctypes.c_int32 * 3), ("split", ctypes.POINTER(ctypes.c_int32) * 3),
                ("physics", ctypes.c_int32), ("gamma", ctypes.c_double), ("mach", ctypes.c_double),
                ("re", ctypes.c_double), ("pr", ctypes.c_double), ("rk", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("algo", ctypes.c_int32), ("L", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("precision", ctypes.c_int32), ("filter", ctypes.c_int32),
                ("filter_alpha", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libatns.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "atns_version": ([], ctypes.c_char_p),
            "atns_create": ([ctypes.POINTER(Config), vp, ctypes.POINTER(vp)], i32),
            "atns_destroy": ([vp], i32),
            "atns_last_error": ([vp], ctypes.c_char_p),
            "atns_set_state": ([vp, vp, i64], i32),
            "atns_get_state": ([vp, vp, i32], i32),
            "atns_get_step": ([vp, ctypes.POINTER(i64)], i32),
            "atns_set_dt": ([vp, dbl], i32),
            "atns_set_delays": ([vp, i64, i32, vp], i32),
            "atns_get_delays": ([vp, i64, vp, ctypes.POINTER(i32)], i32),
            "atns_rhs": ([vp, i32, vp], i32),
            "atns_rk_step": ([vp, i32], i32),
            "atns_step_async": ([vp, i32, i64, vp], i32),
            "atns_set_fusion": ([vp, i32], i32),
            "atns_set_halo_fusion": ([vp, i32], i32),
            "atns_set_filter_fusion": ([vp, i32], i32),
            "atns_reduce": ([vp, vp], i32),
            "atns_reduce_noalloc": ([vp, i32, i32, vp, vp, vp, vp], i32),
            "atns_get_layout": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
            "atns_set_graphs": ([vp, i32], i32),
            "atns_profile_enable": ([vp, i32], i32),
            "atns_profile_read": ([vp, ctypes.POINTER(i64), ctypes.POINTER(dbl)], i32),
            "atns_set_tiles": ([vp, i32, i32, i32], i32),
            "atns_get_tiles": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
            "atns_autotune": ([vp, i32, ctypes.c_char_p, vp], i32),
            "atns_hbm_probe": ([vp, vp, i64, vp], i32),
            "atns_mlp_set_params": ([vp, vp], i32),
            "atns_mlp_get_params": ([vp, vp], i32),
            "atns_mlp_set_scales": ([vp, vp, vp], i32),
            "atns_mlp_forward": ([vp, vp, i32, vp], i32),
            "atns_mlp_grad": ([vp, vp, vp, i32, vp, ctypes.POINTER(dbl)], i32),
            "atns_mlp_sample": ([vp, i32, ctypes.c_uint64, vp, vp], i32),
            "atns_mlp_train": ([vp, i32, i32, dbl, ctypes.c_uint64, vp], i32),
            "atns_mlp_enable": ([vp, i32, dbl], i32),
            "atns_mlp_stats": ([vp, ctypes.POINTER(i64), ctypes.POINTER(i64)], i32),
            "atns_host_weights": ([i32, i32, i32, vp], i32),
            "atns_filter_state": ([vp], i32),
            "atns_set_compensation": ([vp, i32], i32),
            "atns_host_filter_coefficients": ([dbl, vp], i32),
            "atns_host_delays": ([i32, i32, i64, i32, i32, ctypes.c_uint64, vp, ctypes.POINTER(i32)], i32),
            "atns_batch_create": ([ctypes.POINTER(Config), i32, vp, ctypes.POINTER(vp)], i32),
            "atns_batch_destroy": ([vp], i32),
            "atns_batch_last_error": ([vp], ctypes.c_char_p),
            "atns_batch_member": ([vp, i32, ctypes.POINTER(vp)], i32),
            "atns_batch_set_tiles": ([vp, i32, i32, i32, i32], i32),
            "atns_batch_autotune": ([vp, i32, vp], i32),
            "atns_batch_step": ([vp, i32], i32),
            "atns_init_case": ([vp, i32, vp, i32, i64], i32),
            "atns_checkpoint": ([vp, vp, ctypes.POINTER(ctypes.c_size_t)], i32),
            "atns_restore": ([vp, vp, ctypes.c_size_t], i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(status, ctx=None):
    if status != 0:
        msg = lib().atns_last_error(ctx).decode()
        raise AtnsError(status, msg)


def hbm_probe(src, dst, nbytes, stream=None):
    """Enqueue the library's streaming copy of nbytes from tensor src to dst."""
    _check(lib().atns_hbm_probe(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                int(nbytes), stream))


def reduce_noalloc(U, length, ndim, out, stream=None):
    """atns_reduce_noalloc: the FP64 diagnostics of device field U (torch,
    shape (5, nz, ny, nx), float32 or float64) into device tensor out (7
    float64), enqueued on `stream`; nothing is allocated by the library."""
    nz, ny, nx = U.shape[1:]
    n = (ctypes.c_int32 * 3)(nx, ny, nz)
    ln = (ctypes.c_double * 3)(*[float(x) for x in length])
    prec = F64 if str(U.dtype) == "torch.float64" else F32
    _check(lib().atns_reduce_noalloc(ctypes.c_void_p(U.data_ptr()), prec, int(ndim), n, ln,
                                     ctypes.c_void_p(out.data_ptr()), stream))


def host_weights(rk, mode, L):
    out = np.zeros((stages(rk), L, levels(rk)), dtype=np.float64)
    _check(lib().atns_host_weights(rk, mode, L, out.ctypes.data))
    return out


def host_delays(algo, n, nblocks, L, seed, rk=RK4):
    out = np.zeros((nblocks, NSLOTS), dtype=np.int8)
    sync = ctypes.c_int32(0)
    _check(lib().atns_host_delays(algo, rk, n, nblocks, L, ctypes.c_uint64(seed), out.ctypes.data,
                                  ctypes.byref(sync)))
    return out, bool(sync.value)


def host_filter_coefficients(alpha):
    out = np.zeros(6, dtype=np.float64)
    _check(lib().atns_host_filter_coefficients(float(alpha), out.ctypes.data))
    return out


def make_config(n, length, ndim=3, nblk=(1, 1, 1), physics=EULER, gamma=1.4, mach=0.1, re=1600.0,
                pr=0.71, rk=RK4, mode=SA, algo=CAA, L=1, seed=0, precision=F32, split=None,
                filter_alpha=None):
    cfg = Config()
    cfg.ndim = ndim
    for d in range(3):
        cfg.n[d] = int(n[d])
        cfg.len[d] = float(length[d])
        cfg.nblk[d] = int(nblk[d])
    keep = []
    if split is not None:
        for d in range(3):
            arr = (ctypes.c_int32 * len(split[d]))(*split[d])
            keep.append(arr)
            cfg.split[d] = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32))
    cfg.physics, cfg.gamma, cfg.mach, cfg.re, cfg.pr = physics, gamma, mach, re, pr
    cfg.rk, cfg.mode, cfg.algo, cfg.L, cfg.seed, cfg.precision = rk, mode, algo, L, seed, precision
    # the tenth-order filter after every step when filter_alpha is given
    cfg.filter = 0 if filter_alpha is None else 1
    cfg.filter_alpha = 0.0 if filter_alpha is None else float(filter_alpha)
    return cfg, keep


class Solver:
    """One context of the library; state tensors live on the current device."""

    def __init__(self, stream=None, _ctx=None, _owner=None, **kw):
        import torch
        self.torch = torch
        self.kw = dict(kw)
        self.n = tuple(kw["n"])
        self.dtype = torch.float64 if kw.get("precision", F32) == F64 else torch.float32
        self._owner = _owner     # a Batch owns its members' contexts
        if _ctx is None:
            self.cfg, keep = make_config(**kw)
            ctx = ctypes.c_void_p()
            st = lib().atns_create(ctypes.byref(self.cfg), stream, ctypes.byref(ctx))
            if st != 0:
                raise AtnsError(st, lib().atns_last_error(None).decode())
        else:
            ctx = _ctx
        self.ctx = ctx
        nb, D = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().atns_get_layout(ctx, ctypes.byref(nb), ctypes.byref(D)), ctx)
        self.nblocks, self.ring_depth = nb.value, D.value

    def close(self):
        if getattr(self, "ctx", None):
            if self._owner is None:
                lib().atns_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (5, self.n[2], self.n[1], self.n[0])

    def set_state(self, U, step=0):
        U = U.to(device="cuda", dtype=self.dtype).contiguous()
        if tuple(U.shape) != self.shape:
            raise ValueError("state shape %s, expected %s" % (tuple(U.shape), self.shape))
        self.torch.cuda.synchronize()
        _check(lib().atns_set_state(self.ctx, ctypes.c_void_p(U.data_ptr()), int(step)), self.ctx)
        self.torch.cuda.synchronize()      # U may be freed after return

    def get_state(self):
        out = self.torch.empty(self.shape, dtype=self.dtype, device="cuda")
        _check(lib().atns_get_state(self.ctx, ctypes.c_void_p(out.data_ptr()), 0), self.ctx)
        self.torch.cuda.synchronize()
        return out

    def init_case(self, case, params=(), step=0):
        """Analytic initial field computed on the device (CASE_VORTEX with
        params (t, beta, mach, xc, yc) as a prefix, or CASE_TGV)."""
        pa = np.ascontiguousarray(params, dtype=np.float64)
        self.torch.cuda.synchronize()
        _check(lib().atns_init_case(self.ctx, int(case), pa.ctypes.data if pa.size else None, int(pa.size),
                                    int(step)), self.ctx)

    def checkpoint(self):
        """Restart record (bytes) of the current state, ring, step and dt."""
        n = ctypes.c_size_t(0)
        _check(lib().atns_checkpoint(self.ctx, None, ctypes.byref(n)), self.ctx)
        buf = ctypes.create_string_buffer(n.value)
        self.torch.cuda.synchronize()
        _check(lib().atns_checkpoint(self.ctx, buf, ctypes.byref(n)), self.ctx)
        return buf.raw[:n.value]

    def restore(self, blob):
        self.torch.cuda.synchronize()
        _check(lib().atns_restore(self.ctx, ctypes.c_char_p(blob), len(blob)), self.ctx)

    def set_dt(self, dt):
        _check(lib().atns_set_dt(self.ctx, float(dt)), self.ctx)

    def set_delays(self, step0, k):
        k = np.ascontiguousarray(k, dtype=np.int8)
        nsteps = 0 if k.size == 0 else k.shape[0]
        _check(lib().atns_set_delays(self.ctx, int(step0), nsteps, k.ctypes.data if nsteps else None),
               self.ctx)

    def get_delays(self, step):
        out = np.zeros((self.nblocks, NSLOTS), dtype=np.int8)
        sync = ctypes.c_int32(0)
        _check(lib().atns_get_delays(self.ctx, int(step), out.ctypes.data, ctypes.byref(sync)), self.ctx)
        return None if sync.value else out

    def step_number(self):
        s = ctypes.c_int64()
        _check(lib().atns_get_step(self.ctx, ctypes.byref(s)), self.ctx)
        return s.value

    def rhs(self, stage=0):
        """R(U^n) with the halo values RK stage `stage` of the current step reads."""
        out = self.torch.empty(self.shape, dtype=self.dtype, device="cuda")
        self.torch.cuda.synchronize()
        _check(lib().atns_rhs(self.ctx, int(stage), ctypes.c_void_p(out.data_ptr())), self.ctx)
        self.torch.cuda.synchronize()
        return out

    def step(self, nsteps=1):
        _check(lib().atns_rk_step(self.ctx, int(nsteps)), self.ctx)

    def set_compensation(self, on):
        """Compensated classical RK4 steps (the state update's rounding error
        carried to the next step)."""
        _check(lib().atns_set_compensation(self.ctx, 1 if on else 0), self.ctx)

    def filter_state(self):
        """The configured filter applied to the current state (synchronous halos)."""
        _check(lib().atns_filter_state(self.ctx), self.ctx)

    def step_async(self, nsteps, spin_limit=1 << 20):
        """Free-running asynchronous steps; returns the realized delays
        [nsteps][nblocks][NSLOTS] (-1 for unused slots) as a host array."""
        log = self.torch.full((max(1, nsteps), self.nblocks, NSLOTS), -1, dtype=self.torch.int8, device="cuda")
        self.torch.cuda.synchronize()
        _check(lib().atns_step_async(self.ctx, int(nsteps), int(spin_limit), ctypes.c_void_p(log.data_ptr())),
               self.ctx)
        return log[:nsteps].cpu().numpy()

    def set_fusion(self, on):
        """Fused RK4 stage pairs (3-D Euler, classical RK4, FP32)."""
        _check(lib().atns_set_fusion(self.ctx, 1 if on else 0), self.ctx)

    def set_halo_fusion(self, on):
        """Halo assembly inside the first stage of graph-captured Euler steps
        (default off); results are the same bits either way."""
        _check(lib().atns_set_halo_fusion(self.ctx, 1 if on else 0), self.ctx)

    def set_filter_fusion(self, on):
        """The filter of steps with delayed halos as one launch per step
        (default on); results are the same bits either way."""
        _check(lib().atns_set_filter_fusion(self.ctx, 1 if on else 0), self.ctx)

    def set_graphs(self, on):
        _check(lib().atns_set_graphs(self.ctx, 1 if on else 0), self.ctx)

    def profile(self, on):
        _check(lib().atns_profile_enable(self.ctx, 1 if on else 0), self.ctx)

    def profile_read(self):
        """(number of timed stage-kernel launches, their total ms)."""
        n, ms = ctypes.c_int64(), ctypes.c_double()
        _check(lib().atns_profile_read(self.ctx, ctypes.byref(n), ctypes.byref(ms)), self.ctx)
        return n.value, ms.value

    def set_tiles(self, tx, ty, tz):
        _check(lib().atns_set_tiles(self.ctx, tx, ty, tz), self.ctx)

    def get_tiles(self):
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().atns_get_tiles(self.ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), self.ctx)
        return a.value, b.value, c.value

    def autotune(self, reps=5, cache=None):
        best = np.zeros(3, dtype=np.int32)
        path = cache.encode() if cache else None
        _check(lib().atns_autotune(self.ctx, int(reps), path, best.ctypes.data), self.ctx)
        return tuple(int(x) for x in best)

    # ---------------------------------------------------- learned halo
    def mlp_set_params(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float32)
        if th.size != MLP_PARAMS:
            raise ValueError("expected %d parameters" % MLP_PARAMS)
        _check(lib().atns_mlp_set_params(self.ctx, th.ctypes.data), self.ctx)

    def mlp_get_params(self):
        out = np.zeros(MLP_PARAMS, dtype=np.float32)
        _check(lib().atns_mlp_get_params(self.ctx, out.ctypes.data), self.ctx)
        return out

    def mlp_set_scales(self, feat_scale, targ_scale):
        fs = np.ascontiguousarray(feat_scale, dtype=np.float32)
        ts = np.ascontiguousarray(targ_scale, dtype=np.float32)
        _check(lib().atns_mlp_set_scales(self.ctx, fs.ctypes.data, ts.ctypes.data), self.ctx)

    def mlp_forward(self, X):
        X = X.to(device="cuda", dtype=self.torch.float32).contiguous()
        out = self.torch.empty((X.shape[0], 16), dtype=self.torch.float32, device="cuda")
        self.torch.cuda.synchronize()
        _check(lib().atns_mlp_forward(self.ctx, ctypes.c_void_p(X.data_ptr()), X.shape[0],
                                      ctypes.c_void_p(out.data_ptr())), self.ctx)
        self.torch.cuda.synchronize()
        return out

    def mlp_grad(self, X, Y):
        X = X.to(device="cuda", dtype=self.torch.float32).contiguous()
        Y = Y.to(device="cuda", dtype=self.torch.float32).contiguous()
        g = self.torch.empty(MLP_PARAMS, dtype=self.torch.float32, device="cuda")
        loss = ctypes.c_double()
        self.torch.cuda.synchronize()
        _check(lib().atns_mlp_grad(self.ctx, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
                                   X.shape[0], ctypes.c_void_p(g.data_ptr()), ctypes.byref(loss)), self.ctx)
        self.torch.cuda.synchronize()
        return g, loss.value

    def mlp_sample(self, n, seed):
        X = self.torch.empty((n, 64), dtype=self.torch.float32, device="cuda")
        Y = self.torch.empty((n, 8), dtype=self.torch.float32, device="cuda")
        _check(lib().atns_mlp_sample(self.ctx, int(n), ctypes.c_uint64(seed), ctypes.c_void_p(X.data_ptr()),
                                     ctypes.c_void_p(Y.data_ptr())), self.ctx)
        self.torch.cuda.synchronize()
        return X, Y

    def mlp_train(self, iters, batch, lr, seed):
        losses = np.zeros(iters, dtype=np.float64)
        _check(lib().atns_mlp_train(self.ctx, int(iters), int(batch), float(lr), ctypes.c_uint64(seed),
                                    losses.ctypes.data), self.ctx)
        return losses

    def mlp_enable(self, on, tau=1e30):
        _check(lib().atns_mlp_enable(self.ctx, 1 if on else 0, float(tau)), self.ctx)

    def mlp_stats(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().atns_mlp_stats(self.ctx, ctypes.byref(a), ctypes.byref(b)), self.ctx)
        return a.value, b.value

    def reduce(self):
        out = np.zeros(NDIAG, dtype=np.float64)
        st = lib().atns_reduce(self.ctx, out.ctypes.data)
        if st not in (0, -5):
            _check(st, self.ctx)
        return out, st == 0


class Batch:
    """Many instances stepped together (classical RK4, one precision).

    ``configs`` is a list of keyword dicts as taken by ``Solver``; the members
    are ``Solver`` objects over contexts the batch owns (``members``)."""

    def __init__(self, configs, stream=None):
        import torch
        self.torch = torch
        made = [make_config(**kw) for kw in configs]
        arr = (Config * len(made))(*[m[0] for m in made])
        self._keep = [m[1] for m in made]
        h = ctypes.c_void_p()
        st = lib().atns_batch_create(arr, len(made), stream, ctypes.byref(h))
        if st != 0:
            raise AtnsError(st, lib().atns_batch_last_error(None).decode())
        self.h = h
        self.members = []
        for i, kw in enumerate(configs):
            c = ctypes.c_void_p()
            self._check(lib().atns_batch_member(h, i, ctypes.byref(c)))
            self.members.append(Solver(_ctx=c, _owner=self, **kw))

    def _check(self, st):
        if st != 0:
            raise AtnsError(st, lib().atns_batch_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            for m in self.members:
                m.ctx = None
            lib().atns_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, nsteps=1):
        self.torch.cuda.synchronize()
        self._check(lib().atns_batch_step(self.h, int(nsteps)))

    def set_tiles(self, physics, tx, ty, tz):
        self._check(lib().atns_batch_set_tiles(self.h, int(physics), tx, ty, tz))

    def autotune(self, reps=3):
        """Times every tile shape on the batch (advancing it) and keeps the
        fastest; returns ((Euler tx, ty, tz), (Navier-Stokes tx, ty, tz))."""
        best = np.zeros(6, dtype=np.int32)
        self.torch.cuda.synchronize()
        self._check(lib().atns_batch_autotune(self.h, int(reps), best.ctypes.data))
        return tuple(int(x) for x in best[:3]), tuple(int(x) for x in best[3:])
