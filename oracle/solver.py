"""Blocks, delayed history and the RK step of the asynchronous solver.

The global periodic grid is split into a tensor product of blocks (the
processing elements, PEs, of Sec. 3).  Every stage of every step:

* each block builds an extended copy of itself: its owned points from the
  current stage field, and its halo (buffer points, Sec. 3) from
    SA -- the neighbours' current stage values (Alg. 1: exchange every stage);
    AS -- the neighbours' delayed level U^{n-k} (standard stencils on stale
          data, Table 1 cases 2 and 5);
    AT -- sum_l W[e][k][l] U^{n-k-l}, the AT buffer value of stage e
          (Eqs. 7-15; see ``at.py``);
* the CD4 (or, for the second-order method of Table 1 cases 1-3, CD2)
  right-hand side is evaluated on the extended block (``flow.rhs_extended``),
  and
* the RK update of the owned points follows (classical RK4, LSERK4 or
  LSERK2, Eq. 3).

Halo geometry.  Euler needs faces of depth 2.  Navier-Stokes, with viscous
terms built from repeated first derivatives, needs faces of depth 4 and the
2 x 2 edge regions along each pair of directions (no corners).  Each halo
region belongs to exactly one neighbour block; the neighbour slots are

    0 -x   1 +x   2 -y   3 +y   4 -z   5 +z
    6 (-x,-y)  7 (+x,-y)  8 (-x,+y)  9 (+x,+y)
   10 (-x,-z) 11 (+x,-z) 12 (-x,+z) 13 (+x,+z)
   14 (-y,-z) 15 (+y,-z) 16 (-y,+z) 17 (+y,+z)

and the delay that block b sees from slot v is k[b][v] (``delays.py``).

History.  The oracle keeps whole global fields U^m for every level m the
delays can reach -- the plain definition of "the data a PE received at time
level m".

The ``literal`` halo option runs the buffer recursion of Eq. (8) with the
temporal-derivative coefficients of Eq. (12) on the halo data itself, instead
of the closed-form W.  The two agree to round-off.
"""
import numpy as np

from . import at as atmod
from . import delays as dl
from . import filter as filt
from . import flow
from . import rk as rkmod

SLOTS = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1),
         (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 1, 0),
         (-1, 0, -1), (1, 0, -1), (-1, 0, 1), (1, 0, 1),
         (0, -1, -1), (0, 1, -1), (0, -1, 1), (0, 1, 1)]


def even_split(n, nb):
    base, rem = divmod(n, nb)
    return [base + (1 if i < rem else 0) for i in range(nb)]


class Config:
    def __init__(self, n, length, ndim=3, nblk=(1, 1, 1), physics="euler",
                 gamma=1.4, mach=0.1, re=1600.0, pr=0.71, rk="rk4", mode="sa",
                 algo="caa", L=1, seed=0, C=atmod.AT4_C, dt=None, split=None, order=4,
                 filter_alpha=None):
        self.n = tuple(n)
        self.length = tuple(length)
        self.ndim = ndim
        self.nblk = tuple(nblk)
        self.physics = physics
        self.gas = flow.Gas(gamma, mach, re, pr)
        self.rk = rk
        self.mode = mode
        self.algo = algo
        self.L = L
        self.seed = seed
        self.C = C
        self.order = order          # central-difference order, 4 or 2
        self.dt = dt
        self.split = split or [even_split(self.n[d], self.nblk[d]) for d in range(3)]
        self.h = tuple(self.length[d] / self.n[d] for d in range(3))
        self.H = flow.halo_depth(physics)
        # tenth-order Pade filter after every step (None: off); see filter.py
        self.filter_alpha = filter_alpha


class Blocks:
    """Tensor-product block layout.  Block id b = (iz * nby + iy) * nbx + ix."""

    def __init__(self, cfg):
        self.cfg = cfg
        self.origins = []
        self.sizes = []
        self.index = []
        nb = cfg.nblk
        starts = [np.concatenate([[0], np.cumsum(cfg.split[d])[:-1]]) for d in range(3)]
        for iz in range(nb[2]):
            for iy in range(nb[1]):
                for ix in range(nb[0]):
                    self.index.append((ix, iy, iz))
                    self.origins.append((starts[0][ix], starts[1][iy], starts[2][iz]))
                    self.sizes.append((cfg.split[0][ix], cfg.split[1][iy], cfg.split[2][iz]))
        for s in self.sizes:
            for d in range(cfg.ndim):
                if s[d] < cfg.H:
                    raise ValueError("block smaller than the halo depth")

    def __len__(self):
        return len(self.sizes)

    def slots(self):
        """Slots used by the physics: faces (and edges for Navier-Stokes),
        restricted to the active directions."""
        cfg = self.cfg
        out = []
        for v, off in enumerate(SLOTS):
            if cfg.ndim == 2 and off[2] != 0:
                continue
            nz = sum(1 for o in off if o != 0)
            if nz == 1 or (nz == 2 and cfg.physics == flow.NS):
                out.append(v)
        return out

    def region(self, b, v):
        """Local (x, y, z) index ranges of block b's halo region for slot v."""
        cfg = self.cfg
        off = SLOTS[v]
        nz = sum(1 for o in off if o != 0)
        depth = cfg.H if nz == 1 else 2
        rng = []
        for d in range(3):
            s = self.sizes[b][d]
            if off[d] < 0:
                rng.append(np.arange(-depth, 0))
            elif off[d] > 0:
                rng.append(np.arange(s, s + depth))
            else:
                rng.append(np.arange(0, s))
        return rng

    def global_index(self, b, local):
        """Periodic global (z, y, x) index arrays for local per-axis ranges."""
        cfg = self.cfg
        g = [(self.origins[b][d] + local[d]) % cfg.n[d] for d in range(3)]
        return np.ix_(g[2], g[1], g[0])


class Oracle:
    def __init__(self, cfg):
        self.cfg = cfg
        self.blocks = Blocks(cfg)
        self.slots = self.blocks.slots()
        s = rkmod.n_stages(cfg.rk)
        self.s = s
        self.history = {}
        self.n = 0
        self.U = None
        self.overrides = {}
        self.halo = "closed"
        self.mlp = None        # dict(theta, s, r, tau) for the learned halo correction
        self.mlp_counts = [0, 0]
        if cfg.mode in (atmod.AT, atmod.AS):
            self.W = atmod.halo_table(cfg.rk, cfg.mode, cfg.C, cfg.L - 1)
        if cfg.filter_alpha is not None:
            for b in range(len(self.blocks)):
                for d in range(cfg.ndim):
                    if self.blocks.sizes[b][d] < filt.HALO:
                        raise ValueError("block smaller than the filter's halo depth")
            # weights of the delayed levels for the filter's halo at level n+1
            self.Wf = np.array([[float(x) for x in filt.next_level_weights(k, cfg.C)]
                                for k in range(cfg.L)])
        # float coefficients for the literal Eq. (8) recursion
        self._lit = {}

    # ------------------------------------------------------------------ state
    def set_state(self, U, step=0):
        """U^step := U; also recorded as history level ``step``."""
        self.U = np.array(U, dtype=np.float64)
        self.n = step
        self.history[step] = self.U.copy()

    def set_delays(self, step, k):
        self.overrides[step] = np.array(k, dtype=np.int64)

    def delays(self, n=None):
        cfg = self.cfg
        n = self.n if n is None else n
        if cfg.mode == atmod.SA:
            return None
        return dl.delays(cfg.algo, n, len(self.blocks), cfg.L, cfg.C, cfg.seed,
                         self.overrides.get(n))

    # ------------------------------------------------------------- halo fill
    def _extended(self, b, Y, e, k, bufs):
        cfg = self.cfg
        H = cfg.H
        bx, by, bz = self.blocks.sizes[b]
        hz = 0 if cfg.ndim == 2 else H
        E = np.full((5, bz + 2 * hz, by + 2 * H, bx + 2 * H), np.nan)
        own = (slice(None), slice(hz, hz + bz), slice(H, H + by), slice(H, H + bx))
        E[own] = Y[(slice(None),) + self.blocks.global_index(
            b, [np.arange(bx), np.arange(by), np.arange(bz)])]
        for v in self.slots:
            rng = self.blocks.region(b, v)
            gidx = (slice(None),) + self.blocks.global_index(b, rng)
            if k is None:
                vals = Y[gidx]
            elif self.halo == "literal" and cfg.mode == atmod.AT:
                vals = self._literal(b, v, e, int(k[b, v]), gidx, bufs)
            else:
                kk = int(k[b, v])
                vals = np.zeros((5,) + Y[gidx].shape[1:])
                for l in range(cfg.C):
                    w = self.W[e, kk, l]
                    if w != 0.0:
                        vals = vals + w * self.history[self.n - kk - l][gidx]
                if self.mlp is not None and cfg.mode == atmod.AT and v < 6:
                    key = ("mlp", b, v)
                    if key not in bufs:
                        from . import mlp as mlpmod
                        m = self.mlp
                        bufs[key] = mlpmod.correction_for_region(
                            m["theta"], m["s"], m["r"], m["tau"], self.history, self.n, kk, cfg.L,
                            self.blocks, b, v, cfg.H)
                        ok = bufs[key][1]
                        self.mlp_counts[0] += int(ok.sum())
                        self.mlp_counts[1] += int((~ok).sum())
                    vals = vals + bufs[key][0]
            zr = rng[2] + hz
            yr = rng[1] + H
            xr = rng[0] + H
            E[(slice(None),) + np.ix_(zr, yr, xr)] = vals
        return E

    def _literal(self, b, v, e, kk, gidx, bufs):
        """Eq. (8) buffer recursion on the halo values of (b, v)."""
        cfg = self.cfg
        C = cfg.C
        key = kk
        if key not in self._lit:
            nus = rkmod.nu(cfg.rk)
            ext = [float(x) for x in atmod.boundary_coefficients(kk, C)]
            der = [[float(x) for x in atmod.buffer_derivative(kk, C, nus[j])]
                   for j in range(self.s - 1)]
            self._lit[key] = (ext, der)
        ext, der = self._lit[key]
        levels = [self.history[self.n - kk - l][gidx] for l in range(C)]
        dt = cfg.dt
        st = bufs.setdefault((b, v), {})
        if e == 0:
            u0 = sum(ext[l] * levels[l] for l in range(C))
            st["u0"] = u0
            st["u"] = u0
            st["q"] = np.zeros_like(u0)
            st["d"] = []
            return u0
        # temporal derivative at stage e-1 (Eq. 12), in units of 1/dt
        d = sum(der[e - 1][l] * levels[l] for l in range(C)) / dt
        st["d"].append(d)
        if cfg.rk == rkmod.RK4:
            a, _, _ = rkmod.butcher(cfg.rk)
            u = st["u0"].copy()
            for j in range(e):
                u = u + dt * float(a[e][j]) * st["d"][j]
            return u
        # Eq. (8) with m = e: Q^(m) = A_m Q^(m-1) + dt dU/dt|^(m-1),
        # U^(m) = U^(m-1) + B_m Q^(m)   (A_m, B_m are list entries m-1)
        A, B = rkmod.lserk_coeffs(cfg.rk)
        st["q"] = float(A[e - 1]) * st["q"] + dt * d
        st["u"] = st["u"] + float(B[e - 1]) * st["q"]
        return st["u"]

    # ------------------------------------------------------------------- rhs
    def rhs(self, Y, e=0, k=None, bufs=None):
        """RHS of the stage field Y; halos per mode (k None -> synchronous)."""
        cfg = self.cfg
        bufs = {} if bufs is None else bufs
        R = np.empty_like(Y)
        for b in range(len(self.blocks)):
            E = self._extended(b, Y, e, k, bufs)
            Rb = flow.rhs_extended(E, cfg.H, cfg.ndim, cfg.h, cfg.physics, cfg.gas, cfg.order)
            bx, by, bz = self.blocks.sizes[b]
            R[(slice(None),) + self.blocks.global_index(
                b, [np.arange(bx), np.arange(by), np.arange(bz)])] = Rb
        return R

    # ------------------------------------------------------------------ step
    def step(self, nsteps=1):
        for _ in range(nsteps):
            self._step()

    def _step(self):
        cfg = self.cfg
        dt = cfg.dt
        k = self.delays()
        bufs = {}
        U = self.U
        if cfg.rk == rkmod.RK4:
            a, b, _ = rkmod.butcher(cfg.rk)
            Y = U
            ks = []
            for e in range(4):
                ks.append(self.rhs(Y, e, k, bufs))
                if e < 3:
                    Y = U + dt * sum(float(a[e + 1][j]) * ks[j] for j in range(e + 1))
            Unew = U + dt * sum(float(b[j]) * ks[j] for j in range(4))
        else:
            A, B = rkmod.lserk_coeffs(cfg.rk)
            Q = np.zeros_like(U)
            Y = U
            for m in range(self.s):
                Q = float(A[m]) * Q + dt * self.rhs(Y, m, k, bufs)
                Y = Y + float(B[m]) * Q
            Unew = Y
        if cfg.filter_alpha is not None:
            Unew = self.filter_state(Unew, k)
        self.n += 1
        self.U = Unew
        self.history[self.n] = Unew.copy()
        # keep only the levels the delays can reach
        keep = cfg.C + cfg.L
        for m in list(self.history):
            if m < self.n - keep:
                del self.history[m]

    # ---------------------------------------------------------------- filter
    def filter_state(self, U, k=None):
        """The block-local tenth-order filter of ``filter.py`` applied to the
        new level U (= U^{n+1} of the step in progress, self.n = n): x, y and
        (3-D) z passes; halos synchronous when k is None, else from the
        delayed levels (AT: extrapolated to n+1, AS: the newest level)."""
        V = np.array(U, dtype=np.float64)
        for d in range(self.cfg.ndim):
            V = self._filter_pass(V, d, k)
        return V

    def _filter_pass(self, V, d, k):
        cfg = self.cfg
        Hf = filt.HALO
        ax = 3 - d                     # array axis of grid axis d ([var][z][y][x])
        out = np.empty_like(V)
        for b in range(len(self.blocks)):
            s = self.blocks.sizes[b]
            own = [np.arange(s[0]), np.arange(s[1]), np.arange(s[2])]
            ext = list(own)
            ext[d] = np.arange(-Hf, s[d] + Hf)
            E = V[(slice(None),) + self.blocks.global_index(b, ext)].copy()
            if k is not None:
                for side, v in ((0, 2 * d), (1, 2 * d + 1)):
                    hr = list(own)
                    hr[d] = np.arange(-Hf, 0) if side == 0 else np.arange(s[d], s[d] + Hf)
                    gidx = (slice(None),) + self.blocks.global_index(b, hr)
                    kk = int(k[b, v])
                    if cfg.mode == atmod.AT:
                        vals = np.zeros(V[gidx].shape)
                        for l in range(cfg.C):
                            vals = vals + self.Wf[kk, l] * self.history[self.n - kk - l][gidx]
                    else:
                        vals = self.history[self.n - kk][gidx]
                    pos = [slice(None)] * 4
                    pos[ax] = slice(0, Hf) if side == 0 else slice(s[d] + Hf, s[d] + 2 * Hf)
                    E[tuple(pos)] = vals
            F = filt.filter_block_lines(np.moveaxis(E, ax, -1), cfg.filter_alpha)
            out[(slice(None),) + self.blocks.global_index(b, own)] = np.moveaxis(F, -1, ax)
        return out
