"""FP64 reference of the learned halo correction (not part of the paper).

A small multilayer perceptron predicts, for a face halo point, the error of
the AT buffer extrapolation (Eq. 15) from the delayed levels the extrapolation
itself uses, and the correction is added to every stage's AT halo value:

    Uhat_MLP^(e)(x) = Uhat_AT^(e)(x) + delta(x),   delta_v = r_v * out_v,

unless the correction is implausibly large, |out|_2 > tau, in which case the
AT value is kept (the fallback: the AT stencil decides whether the MLP output is used).

Features (64 per sample).  The halo point x lies in the neighbour's
boundary layer; along the face normal it has layer neighbours j-1, j, j+1
(clamped to the layer).  For the 4 newest delayed levels l = 0..3
(U^{n-k-l}), the 5 conserved variables and those 3 points, the feature is
(U^{n-k-l}_v(point) - U^{n-k}_v(x)) / s_v  (60 values), then k / (L-1), then
3 zeros.  s_v and r_v are per-variable scales.
Target (training only): out_v = (U^n_v(x) - Uhat_AT^(0)_v(x)) / r_v.

Network: 64 -> 64 (ReLU) -> 64 (ReLU) -> 16 (the first 5 outputs used).
Parameters, in this order, row-major [out][in]: W1[64][64], b1[64],
W2[64][64], b2[64], W3[16][64], b3[16]  (9360 values).
Loss: mean over samples and the 5 used outputs of (out - target)^2.

The GPU computes with BF16 operands and FP32 accumulation; ``bf16`` below
rounds to BF16 (round to nearest even) so the oracle can evaluate the same
rounded operands in FP64.
"""
import numpy as np

NIN, NH, NOUT, NUSE = 64, 64, 16, 5
SIZES = [("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
         ("W3", (NOUT, NH)), ("b3", (NOUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SIZES])


def bf16(x):
    """Round float values to the nearest BF16 (ties to even), as float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def init(seed):
    """He-normal weights, zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in SIZES:
        if name.startswith("W"):
            p[name] = rng.standard_normal(shape) * np.sqrt(2.0 / shape[1])
        else:
            p[name] = np.zeros(shape)
    return pack(p)


def forward(theta, X, round_bf16=False):
    """Outputs (n, 16) and the cached activations.  With round_bf16 the
    layer inputs and weights are rounded to BF16 as the GPU does."""
    p = unpack(theta)
    r = bf16 if round_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    Z1 = r(X) @ r(p["W1"]).T + p["b1"]
    H1 = np.maximum(Z1, 0.0)
    Z2 = r(H1) @ r(p["W2"]).T + p["b2"]
    H2 = np.maximum(Z2, 0.0)
    O = r(H2) @ r(p["W3"]).T + p["b3"]
    return O, (X, Z1, H1, Z2, H2)


def loss_and_grad(theta, X, Y):
    """Mean squared error over the 5 used outputs and its exact gradient."""
    p = unpack(theta)
    O, (X, Z1, H1, Z2, H2) = forward(theta, X)
    n = X.shape[0]
    diff = np.zeros_like(O)
    diff[:, :NUSE] = O[:, :NUSE] - np.asarray(Y, dtype=np.float64)[:, :NUSE]
    loss = float((diff[:, :NUSE] ** 2).sum() / (n * NUSE))
    dO = 2.0 * diff / (n * NUSE)
    g = {"W3": dO.T @ H2, "b3": dO.sum(axis=0)}
    dH2 = (dO @ p["W3"]) * (Z2 > 0)
    g["W2"] = dH2.T @ H1
    g["b2"] = dH2.sum(axis=0)
    dH1 = (dH2 @ p["W2"]) * (Z1 > 0)
    g["W1"] = dH1.T @ X
    g["b1"] = dH1.sum(axis=0)
    return loss, pack(g)


# ------------------------------------------------------------ halo samples
def face_features(levels, k, L, j_axis, s):
    """Features of one face-halo point.

    levels[l] : array (5, 3) -- level n-k-l at the points j-1, j, j+1 along
                the face normal (l = 0..3);
    s         : per-variable feature scales (5,).
    """
    f = np.zeros(NIN)
    c = levels[0][:, 1]
    o = 0
    for l in range(4):
        for v in range(5):
            for j in range(3):
                f[o] = (levels[l][v, j] - c[v]) / s[v]
                o += 1
    f[60] = k / max(1, L - 1)
    return f


def correct(out, r, tau):
    """(delta (5,), accepted): delta_v = r_v out_v unless |out|_2 > tau."""
    out = np.asarray(out[:NUSE], dtype=np.float64)
    if np.sqrt((out ** 2).sum()) > tau:
        return np.zeros(NUSE), False
    return np.asarray(r, dtype=np.float64) * out, True


# ------------------------------------------------- solver-side application
def region_points(blocks, b, v, H):
    """Per-point data of block b's face halo region v: (region-local normal
    index, normal axis, depth) and the global (z, y, x) index arrays of the
    point and of its two normal neighbours (clamped to the region), in the
    region's [z][y][x] order."""
    from .solver import SLOTS
    off = SLOTS[v]
    axis = [d for d in range(3) if off[d] != 0][0]
    rng = blocks.region(b, v)
    size = blocks.sizes[b]
    org = blocks.origins[b]
    n = blocks.cfg.n
    Z, Y, X = np.meshgrid(rng[2], rng[1], rng[0], indexing="ij")
    loc = [X, Y, Z]
    # region-local normal index
    ia = loc[axis] + H if off[axis] < 0 else loc[axis] - size[axis]
    pts = []
    for j in (-1, 0, 1):
        ib = np.clip(ia + j, 0, H - 1)
        la = ib - H if off[axis] < 0 else ib + size[axis]
        c = [X, Y, Z]
        c[axis] = la
        pts.append(tuple((org[d] + c[d]) % n[d] for d in (2, 1, 0)))
    return pts


def correction_for_region(theta, s, r, tau, history, n_now, k, L, blocks, b, v, H, ring_f32=False):
    """delta (5, ...) and the accepted mask for every point of a face halo
    region, with the GPU's arithmetic order: features in FP32 from the level
    values (rounded to FP32 when the ring holds FP32), BF16 operands, FP64
    accumulation, FP32 norm test."""
    pts = region_points(blocks, b, v, H)
    shape = pts[1][0].shape
    f32 = np.float32
    inv_s = (f32(1.0) / np.asarray(s, dtype=f32)).astype(f32)
    lev = [history[n_now - k - l] for l in range(4)]
    centre = [lev[0][vv][pts[1]].astype(f32) for vv in range(5)]
    feats = np.zeros(shape + (64,), dtype=np.float32)
    o = 0
    for l in range(4):
        for vv in range(5):
            for j in range(3):
                val = lev[l][vv][pts[j]].astype(f32)
                feats[..., o] = ((val - centre[vv]) * inv_s[vv]).astype(f32)
                o += 1
    feats[..., 60] = f32(k) / f32(L - 1) if L > 1 else 0.0
    Xf = feats.reshape(-1, 64).astype(np.float64)
    out, _ = forward(theta, Xf, round_bf16=True)
    out = out[:, :NUSE]
    n2 = (out.astype(np.float32) ** 2).sum(axis=1, dtype=np.float32)
    ok = n2 <= np.float32(min(tau * tau, 1e30))
    delta = np.asarray(r, dtype=np.float32).astype(np.float64)[None, :] * out
    delta[~ok] = 0.0
    return delta.T.reshape((5,) + shape), ok.reshape(shape)
