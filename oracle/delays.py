"""Delay schedules of the asynchronous algorithms (Sec. 4, Alg. 2 and 3).

Steps are numbered n = 0, 1, 2, ...; step n advances U^n to U^{n+1}.  The
first C steps (n < C) are synchronous in both algorithms (Alg. 2 and 3 start
with a synchronous loop of C steps that populates the C buffer levels).

Readings taken where the paper leaves room:

* Delay bound.  Alg. 3 resets the delay once it exceeds L-1, so a used delay
  always satisfies 0 <= k <= L-1.
* CAA (Alg. 2).  Communication happens every L steps and delivers every level
  since the previous exchange; the delay grows by one per step and resets to
  0 at the exchange.  For n >= C:  k(n) = (n - C) mod L, the same on every
  block and every face.  (Alg. 2's test n % L == C-1 never fires when L < C;
  this reading keeps the period-L, uniform delay that the text describes.)
* SAA (Alg. 3).  The delay a block sees from a neighbour is random.  It is
  drawn independently for every (step, block, neighbour slot) from a
  counter-based generator, uniform on {0..L-1}, and held fixed over the RK
  stages of the step.
* Guard (Alg. 3).  A delay larger than L-1, or one that would need levels
  older than the history holds (levels "not consecutive", i.e. k > n-C+1),
  triggers a wait: the delay becomes 0 for that step.

Counter-based generator: SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014).  Draw number i of a
stream seeded with s is mix(s + (i+1)*GOLDEN) with
    mix(z): z = (z ^ (z>>30)) * 0xBF58476D1CE4E5B9
            z = (z ^ (z>>27)) * 0x94D049BB133111EB
            return z ^ (z>>31)
all modulo 2^64.  The draw index for (step n, block b, slot v) is
i = (n * nblocks + b) * NSLOTS + v, and the delay is draw mod L.
"""
import numpy as np

MASK = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
NSLOTS = 18          # 6 faces + 12 edges; Euler uses the first 6

CAA, SAA = "caa", "saa"


def splitmix64_draw(seed, i):
    z = (seed + (i + 1) * GOLDEN) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def raw_delays(algo, n, nblocks, L, C, seed):
    """Delays before the guard, int array [nblocks, NSLOTS]."""
    if algo == CAA:
        return np.full((nblocks, NSLOTS), (n - C) % L, dtype=np.int64)
    out = np.empty((nblocks, NSLOTS), dtype=np.int64)
    for b in range(nblocks):
        for v in range(NSLOTS):
            i = (n * nblocks + b) * NSLOTS + v
            out[b, v] = splitmix64_draw(seed, i) % L
    return out


def apply_guard(k, n, L, C):
    """Alg. 3 guard: delays above L-1 or beyond the available history -> 0."""
    k = np.array(k, dtype=np.int64)
    bad = (k > L - 1) | (k > n - C + 1) | (k < 0)
    k[bad] = 0
    return k


def delays(algo, n, nblocks, L, C, seed, override=None):
    """Used delays for step n, or None for a synchronous step (n < C).

    ``override`` (int array [nblocks, NSLOTS]) replaces the raw draw, as an
    injected schedule does; the guard still applies.
    """
    if n < C:
        return None
    raw = override if override is not None else raw_delays(algo, n, nblocks, L, C, seed)
    return apply_guard(raw, n, L, C)
