"""Tenth-order Pade low-pass filter, applied block by block with delayed halos.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The filter (Sec. 2: Pade-type low-pass filters of up to tenth order with a
coefficient -0.5 < alpha_f <= 0.5; the Taylor-Green runs of Sec. 5.2 use the
tenth-order filter with alpha_f = 0.499).  Along one grid line

    alpha fhat[i-1] + fhat[i] + alpha fhat[i+1]
        = sum_{m=0..5} (a_m / 2) (f[i+m] + f[i-m]),

whose transfer function on a Fourier mode exp(i w j) is

    T(w) = (sum_m a_m cos(m w)) / (1 + 2 alpha cos w).

The six a_m are not printed in the paper.  They follow from six linear
conditions: T(pi) = 0 (the odd-even mode is removed) and 1 - T(w) = O(w^10),
i.e. the w^{2p} Taylor coefficients of numerator and denominator agree for
p = 0..4:

    sum_m a_m m^{2p} = [p == 0] + 2 alpha      (p = 0..4, with 0^0 = 1)
    sum_m a_m (-1)^m = 0.

``coefficients`` solves them over the rationals.

Block-local application (a reading: the paper does not say how the implicit
filter is applied across PE boundaries, nor under delays).
* Every block filters its own lines.  The tridiagonal system is restricted to
  the block's n owned points of the line; the two filtered values just
  outside the block that its first and last rows reference are replaced by
  the unfiltered halo values there (moved to the right-hand side).  The
  right-hand side reads up to five halo points beyond each face.  Blocks
  thus solve independently, which is what lets them run asynchronously.
* The three directions are filtered one after the other (x, then y, then
  z), each pass on the output of the previous one.
* Halo values of a pass along axis d come from the neighbours across the two
  d-faces, five layers deep:
    synchronous steps -- the neighbours' current values of the same pass
                         input (an exchange before every pass);
    AT steps          -- the neighbours' value at the new level n+1,
                         extrapolated from the C delayed levels
                         U^{n-k-l} with the Lagrange weights of Eqs. 14-15
                         taken one step further (delay k+1), the same for all
                         passes;
    AS steps          -- the newest delayed level U^{n-k}.
* The filter acts on the conserved variables once per step, after the last
  stage; the filtered field is the new state and its boundary layers are the
  data the neighbours receive.

With the closure, a polynomial of degree <= 9 passes through a block
unchanged (it satisfies every row exactly), and far from the faces the block
filter equals the periodic one: the closure's perturbation decays into the
block like r^j, r = (-1 + sqrt(1 - 4 alpha^2)) / (2 alpha).
"""
from fractions import Fraction as Fr

import numpy as np

from . import at as atmod

HALO = 5      # right-hand-side half width: the halo depth a pass reads


def _exact(alpha):
    return alpha if isinstance(alpha, Fr) else Fr(alpha)


def coefficients(alpha):
    """[a_0, ..., a_5] as Fractions (alpha converted exactly)."""
    al = _exact(alpha)
    rows, rhs = [], []
    for p in range(5):
        rows.append([Fr(m) ** (2 * p) if (m or p) else Fr(1) for m in range(6)])
        rhs.append((Fr(1) if p == 0 else Fr(0)) + 2 * al)
    rows.append([Fr((-1) ** m) for m in range(6)])
    rhs.append(Fr(0))
    return atmod.solve_exact(rows, rhs)


def transfer(w, alpha):
    """T(w) in float64 from the exact coefficients."""
    a = [float(x) for x in coefficients(alpha)]
    w = np.asarray(w, dtype=np.float64)
    num = sum(a[m] * np.cos(m * w) for m in range(6))
    return num / (1.0 + 2.0 * float(alpha) * np.cos(w))


def _rhs(ext, a):
    """Right-hand side at the owned points of extended lines (last axis:
    HALO points, n owned points, HALO points)."""
    n = ext.shape[-1] - 2 * HALO
    r = a[0] * ext[..., HALO:HALO + n]
    for m in range(1, 6):
        r = r + 0.5 * a[m] * (ext[..., HALO + m:HALO + m + n] + ext[..., HALO - m:HALO - m + n])
    return r


def filter_block_lines(ext, alpha):
    """Block-local filter of lines given with their halos (last axis of
    length n + 2*HALO); returns the n filtered owned values per line."""
    ext = np.asarray(ext, dtype=np.float64)
    a = [float(x) for x in coefficients(alpha)]
    al = float(alpha)
    n = ext.shape[-1] - 2 * HALO
    r = _rhs(ext, a)
    r[..., 0] = r[..., 0] - al * ext[..., HALO - 1]
    r[..., n - 1] = r[..., n - 1] - al * ext[..., HALO + n]
    A = np.eye(n) + al * (np.eye(n, k=1) + np.eye(n, k=-1))
    flat = r.reshape(-1, n).T
    return np.linalg.solve(A, flat).T.reshape(r.shape)


def filter_periodic_lines(f, alpha):
    """The filter on periodic lines (last axis), cyclic tridiagonal system."""
    f = np.asarray(f, dtype=np.float64)
    a = [float(x) for x in coefficients(alpha)]
    al = float(alpha)
    n = f.shape[-1]
    r = a[0] * f
    for m in range(1, 6):
        r = r + 0.5 * a[m] * (np.roll(f, -m, axis=-1) + np.roll(f, m, axis=-1))
    A = np.eye(n)
    for i in range(n):
        A[i, (i - 1) % n] += al
        A[i, (i + 1) % n] += al
    flat = r.reshape(-1, n).T
    return np.linalg.solve(A, flat).T.reshape(r.shape)


def next_level_weights(k, C):
    """Weights of the C delayed levels U^{n-k-l} (l = 0..C-1) that
    extrapolate a halo value to level n+1: the Lagrange extrapolation of
    Eqs. 14-15 at delay k+1."""
    return atmod.lagrange_extrapolation(k + 1, C)
