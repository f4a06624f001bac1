"""Counter-based generators of synthetic inputs (payloads, erasures, ids)."""

import math

import numpy as np

MASK64 = (1 << 64) - 1
G = 0x9E3779B97F4A7C15
C1 = 0xBF58476D1CE4E5B9
C2 = 0x94D049BB133111EB

DATA, ERASE, REPAIR, UPDATE_IDS, UPDATE_DATA, WORKLOAD, ARRIVAL = 2, 3, 4, 5, 6, 7, 8


def mix64(z):
    z &= MASK64
    z ^= z >> 30
    z = (z * C1) & MASK64
    z ^= z >> 27
    z = (z * C2) & MASK64
    z ^= z >> 31
    return z


def stream_key(seed, purpose, a, b):
    k = mix64((seed + G) & MASK64)
    for v in (purpose, a, b):
        k = mix64(k ^ (v & MASK64))
    return k


def draw(key, i):
    return mix64((key + (i + 1) * G) & MASK64)


def _mix64_np(z):
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(C1)
        z ^= z >> np.uint64(27)
        z *= np.uint64(C2)
        z ^= z >> np.uint64(31)
    return z


def draws_np(key, start, count):
    idx = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(key) + idx * np.uint64(G)
    return _mix64_np(z)


def uniform01(u):
    """53-bit uniform in [0, 1) from a 64-bit draw."""
    return (u >> 11) * (1.0 / (1 << 53))


def payload_slice(seed, stripe, blocks, byte_lo, byte_hi, purpose=DATA):
    """Bytes [byte_lo, byte_hi) of the listed blocks: uint8[len(blocks), hi-lo].

    Word w (8 bytes, little endian) of block i is draw w of
    key(seed, purpose, stripe, i); byte offsets must be multiples of 8.
    """
    assert byte_lo % 8 == 0 and byte_hi % 8 == 0 and byte_hi >= byte_lo
    w0, nw = byte_lo // 8, (byte_hi - byte_lo) // 8
    out = np.empty((len(blocks), nw), dtype=np.uint64)
    for r, i in enumerate(blocks):
        out[r] = draws_np(stream_key(seed, purpose, stripe, int(i)), w0, nw)
    return out.astype("<u8", copy=False).view(np.uint8).reshape(len(blocks), nw * 8)


def payload(seed, stripe, k, t, purpose=DATA):
    """Whole input stripe x: uint8[k, t]."""
    return payload_slice(seed, stripe, range(k), 0, t, purpose)


def sample_distinct(key, m, N):
    """m distinct values of [0, N) (Floyd; multiply-shift reduction), sorted."""
    assert 0 <= m <= N
    chosen = set()
    for s in range(m):
        r = N - m + s
        v = ((draw(key, s + 1) >> 32) * (r + 1)) >> 32
        chosen.add(r if v in chosen else v)
    return sorted(chosen)


def round_half_up(x):
    return int(math.floor(x + 0.5))


def overhead_n(k, eps):
    """Number of coded blocks for k inputs at overhead eps: round(k (1 + eps))."""
    return round_half_up(k * (1.0 + eps))


def erasure_ids(seed, stripe, n, e):
    return sample_distinct(stream_key(seed, ERASE, stripe, 0), e, n)


def erasure_mask(seed, stripe, n, e):
    m = np.zeros(n, dtype=np.uint8)
    m[erasure_ids(seed, stripe, n, e)] = 1
    return m


def repair_lost(seed, stripe, n, max_lost=4):
    """1 + floor(max_lost * U) distinct lost coded rows (capped at n)."""
    key = stream_key(seed, REPAIR, stripe, 0)
    m = 1 + (((draw(key, 0) >> 32) * max_lost) >> 32)
    m = min(m, n)
    # Floyd consumes draws 1..m of the same stream
    return sample_distinct(key, m, n)


def update_ids(seed, stripe, k, count):
    return sample_distinct(stream_key(seed, UPDATE_IDS, stripe, 0), min(count, k), k)


def update_blocks(seed, stripe, ids, t):
    """New contents of the updated inputs: uint8[len(ids), t]."""
    return payload_slice(seed, stripe, ids, 0, t, purpose=UPDATE_DATA)
