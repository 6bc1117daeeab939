"""Counter-based random numbers for the method's own random draws.

The paper draws random numbers in two places and says nothing about how:
the initial KNN lists of Alg. 3 ("initialize with random lists") and the seeds
of every bisection in Alg. 1.  Both the oracle and the HIP library implement the
same published generator independently, so that both sides draw identical
integers:

* SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014).  The generator with state ``s`` returns
  ``mix64(s + (c+1)*GAMMA)`` as its c-th output; here the state is a key derived
  from ``(seed, stream)`` and ``c`` is an explicit counter.
* ``below(r, m)``: an integer in [0, m) from the top 32 bits of ``r`` by
  multiply-shift (Lemire, 2019), without rejection.
* ``floyd_sample``: Floyd's algorithm for ``cnt`` distinct integers from
  [0, m) using exactly ``cnt`` draws (Bentley & Floyd, "Programming pearls:
  a sample of brilliance", CACM 30(9), 1987).

Stream layout: ``purpose << 56 | round << 40 | index``.

Pins: ``mix64`` reproduces the published SplitMix64 sequence for seed 0
(tests/golden/splitmix64_seed0.txt); ``floyd_sample`` is checked for
distinctness, range and uniformity (chi-square) in the CPU tests.
"""
import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB

PURPOSE_GRAPH_INIT = 1
PURPOSE_TWOMEANS = 2
PURPOSE_RANDOM_INIT = 3

ROUND_FIT = 0xFFFF  # round tag of the TwoMeans call that initialises a fit


def stream_id(purpose, rnd, index):
    return ((purpose & 0xFF) << 56) | ((rnd & 0xFFFF) << 40) | (index & ((1 << 40) - 1))


def mix64(z):
    """SplitMix64 output function on a Python int (mod 2**64)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * M1) & MASK64
    z = ((z ^ (z >> 27)) * M2) & MASK64
    return z ^ (z >> 31)


def mix64_np(z):
    """Vectorised ``mix64`` on a numpy uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(M2)
    return z ^ (z >> np.uint64(31))


def stream_key(seed, stream):
    return mix64((seed & MASK64) ^ mix64(stream))


def draw(key, ctr):
    """The ctr-th SplitMix64 output of a generator whose state starts at key."""
    return mix64((key + (ctr + 1) * GAMMA) & MASK64)


def draw_np(keys, ctr):
    keys = np.asarray(keys, dtype=np.uint64)
    with np.errstate(over="ignore"):
        s = keys + np.uint64(((ctr + 1) * GAMMA) & MASK64)
    return mix64_np(s)


def below(r, m):
    return ((r >> 32) * m) >> 32


def below_np(r, m):
    """``below`` for arrays; m may be an array of bounds (all < 2**32)."""
    r = np.asarray(r, dtype=np.uint64)
    m = np.asarray(m, dtype=np.uint64)
    return ((r >> np.uint64(32)) * m) >> np.uint64(32)


def floyd_sample(key, m, cnt):
    """Floyd's algorithm: ``cnt`` distinct values of [0, m), in insertion order.

    For j = m-cnt .. m-1 draw t uniform in [0, j]; insert t unless already
    chosen, in which case insert j.  Draw number c = j - (m - cnt).
    """
    assert 0 <= cnt <= m
    chosen = []
    seen = set()
    base = m - cnt
    for j in range(base, m):
        t = below(draw(key, j - base), j + 1)
        v = j if t in seen else t
        seen.add(v)
        chosen.append(v)
    return chosen


def floyd_sample_rows(keys, m, cnt):
    """``floyd_sample`` for many independent keys at once (one row per key)."""
    keys = np.asarray(keys, dtype=np.uint64)
    rows = keys.shape[0]
    out = np.empty((rows, cnt), dtype=np.int64)
    base = m - cnt
    for c, j in enumerate(range(base, m)):
        t = below_np(draw_np(keys, c), j + 1).astype(np.int64)
        dup = (out[:, :c] == t[:, None]).any(axis=1) if c else np.zeros(rows, bool)
        out[:, c] = np.where(dup, j, t)
    return out
