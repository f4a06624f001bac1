"""Counter-based random streams for the graph of the code (oracle copy).

The paper draws degrees and neighbour sets from a seeded pseudo-random
generator, so that any party holding the seed regenerates the same bipartite
graph (§1, and §2.2 on the per-object seed).  Its generator is a linear
congruential one whose constants are not given, so this implementation uses
a counter-based stream instead, defined as follows:

  mix64(z)   the SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014,
             with the "Mix13" finaliser constants of D. Stafford):
               z ^= z >> 30; z *= 0xBF58476D1CE4E5B9
               z ^= z >> 27; z *= 0x94D049BB133111EB
               z ^= z >> 31          (all mod 2**64)
  key(seed, purpose, a, b) = mix64(mix64(mix64(mix64(seed + G) ^ purpose) ^ a) ^ b)
  draw i >= 0 of a key       = mix64(key + (i + 1) * G),  G = 0x9E3779B97F4A7C15

The graph uses purpose 1 with a = stripe key and b = coded row index, so every
coded row owns its own stream: a row does not depend on n (prefix stability).
Draw 0 of a row picks its degree, draws 1.. feed Floyd's sampler.

Pinned by: the published SplitMix64 sequence for seed 0 (tests), and by the
agreement of the scalar Python-int path with the vectorised numpy path.
"""

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB

PURPOSE_GRAPH = 1


def mix64(z):
    """SplitMix64 output function on a Python int (mod 2**64)."""
    z &= MASK64
    z ^= z >> 30
    z = (z * M1) & MASK64
    z ^= z >> 27
    z = (z * M2) & MASK64
    z ^= z >> 31
    return z


def stream_key(seed, purpose, a, b):
    """Key of the stream (seed, purpose, a, b), by four chained mixes."""
    k = mix64((seed + GOLDEN) & MASK64)
    k = mix64(k ^ (purpose & MASK64))
    k = mix64(k ^ (a & MASK64))
    k = mix64(k ^ (b & MASK64))
    return k


def draw(key, i):
    """Draw number i (i >= 0) of the stream with this key."""
    return mix64((key + (i + 1) * GOLDEN) & MASK64)


def mix64_np(z):
    """Vectorised mix64 on a numpy uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(M1)
        z ^= z >> np.uint64(27)
        z *= np.uint64(M2)
        z ^= z >> np.uint64(31)
    return z


def draws_np(key, start, count):
    """Draws start .. start+count-1 of one stream, as a uint64 array."""
    idx = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(key) + idx * np.uint64(GOLDEN)
    return mix64_np(z)
