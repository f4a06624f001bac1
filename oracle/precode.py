"""Array-LDPC precode (check #1) and the two-stage decode (oracle copy).

Test infrastructure: only the tests, the smoke check and the CPU baseline of
the benchmark use this module; the library never does.

A (b, k, n) code first extends b data blocks to k blocks with k - b parity
blocks of a binary array LDPC code (§2.4, Algorithm 2), then encodes the k
blocks with the LDGM graph (§2.2).  Decoding runs BP at most twice (§2.2):
once on the LDGM graph, and, if inputs are still missing, once on the
precode's check equations.

Functions and the passage each follows
  largest_prime_factor  the helper Algorithm 2 names.
  array_params   p = largest prime factor of k, k' = k / p, j' = k' - b / p
                 (Algorithm 2); b must be a multiple of p with 1 <= j' < k'.
  check_one      Algorithm 2: the k - b rows of L(1), k' - j' symbol indices
                 each, built from the circulant block structure of array
                 codes that Algorithm 2's index formula spells out.
  checks         each check equation as its member set: row r of L(1) plus
                 the parity block b + r it defines (reading below).
  encode         x[0:b] = data; x[b + r] = XOR of x over row r of L(1), in
                 increasing r.
  decode_two_stage  LDGM decode (codec.decode), then level-synchronous BP
                 over the checks: at each level every check with exactly one
                 unknown member names it; the named blocks are recovered from
                 their check of lowest index.
  repair_two_stage  the conventional repair of a precoded code (§4: decode
                 the entire data, then re-run the encoding of the lost
                 chunks): the two-stage decode from the rows neither erased
                 nor lost; with every data block back, the parity blocks are
                 encoded again, so every input is known; a lost row is
                 rebuilt when all its inputs are known.

Readings (the paper states neither explicitly):
  * Row r of L(1) lists the blocks whose XOR is parity block b + r.  The
    indices of a row all lie below b + p*floor(r / p), so the parity blocks
    can be produced block row by block row, which is the linear-time
    encoding the paper attributes to array codes.
  * The second BP does not feed back into the first ("at most twice").
  * Success means all b data blocks recovered; parity blocks left unknown
    do not matter.
"""

import numpy as np

from . import codec


def largest_prime_factor(k):
    assert k >= 2
    best, x, d = 1, k, 2
    while d * d <= x:
        while x % d == 0:
            best, x = d, x // d
        d += 1
    return max(best, x) if x > 1 else best


def array_params(b, k):
    p = largest_prime_factor(k)
    kp = k // p
    assert b % p == 0, "b must be a multiple of the largest prime factor of k"
    jp = kp - b // p
    assert 1 <= jp < kp, "need 1 <= j' < k'"
    return p, kp, jp


def check_one(b, k):
    """L(1) of Algorithm 2 as a list of k - b rows, members ascending.

    Array LDPC codes are built from powers of the p x p cyclic shift P (row i
    of P^s has its one in column (i + s) mod p).  Cut the k blocks into k'
    block columns of p blocks.  Block row j < j' has k' - j' + 1 nonzero
    blocks, at block columns j .. c_j with c_j = j + k' - j'; the block at
    column c is P^s with s = (j' - 1 - j)(c - c_j) mod p, so the last one is
    the identity and names the parity block c_j p + i = b + jp + i of check
    row i + jp.  Row i + jp of L(1) lists the other members: the blocks
    c p + (i + s) mod p for c = j .. c_j - 1.
    """
    p, kp, jp = array_params(b, k)
    w = kp - jp
    j = np.arange(jp).reshape(jp, 1, 1)
    i = np.arange(p).reshape(1, p, 1)
    c = j + np.arange(w).reshape(1, 1, w)        # block columns j .. c_j - 1
    cj = j + w
    s = ((jp - 1 - j) * (c - cj)) % p
    L = (c * p + (i + s) % p).reshape(jp * p, w)
    return [sorted(int(v) for v in row) for row in L]


def checks(b, k):
    """Member sets of the k - b check equations (XOR of members = 0)."""
    return [sorted(set(row) | {b + r}) for r, row in enumerate(check_one(b, k))]


def encode(b, k, data):
    """x[k, t]: the data blocks followed by the k - b parity blocks."""
    data = np.ascontiguousarray(data, dtype=np.uint8)
    assert data.shape[0] == b
    x = np.zeros((k, data.shape[1]), dtype=np.uint8)
    x[:b] = data
    for r, row in enumerate(check_one(b, k)):
        acc = np.zeros(data.shape[1], dtype=np.uint8)
        for i in row:
            acc ^= x[i]
        x[b + r] = acc
    return x


def precode_bp(b, k, x, known, maxit=0):
    """Level-synchronous BP over the checks.  x[k, t] holds the known blocks
    (others ignored); returns (x with the recovered blocks filled in, known
    mask after, levels)."""
    x = x.copy()
    known = np.asarray(known, dtype=bool).copy()
    C = checks(b, k)
    levels = 0
    while maxit == 0 or levels < maxit:
        named = {}
        for ci, members in enumerate(C):
            unknown = [s for s in members if not known[s]]
            if len(unknown) == 1 and unknown[0] not in named:
                named[unknown[0]] = ci
        if not named:
            break
        for s, ci in named.items():
            acc = np.zeros(x.shape[1], dtype=np.uint8)
            for m in C[ci]:
                if m != s:
                    acc ^= x[m]
            x[s] = acc
        for s in named:
            known[s] = True
        levels += 1
    return x, known, levels


def decode_two_stage(G, b, c, erased, maxit=0):
    """Returns (data[b, t], recovered_data[b], status = (ok, unrecovered data
    blocks, LDGM levels, precode levels))."""
    k = G.k
    x, rec, st, _ = codec.decode(G, c, erased, maxit)
    known = rec.astype(bool)
    levels2 = 0
    if not known[:b].all():
        x, known, levels2 = precode_bp(b, k, x, known)
        x[~known] = 0
    data_ok = known[:b]
    return x[:b], data_ok.astype(np.uint8), (int(data_ok.all()), int(b - data_ok.sum()), int(st[2]), int(levels2))


def repair_two_stage(G, b, c, erased, lost, maxit=0):
    """Returns (blocks[m, t], repaired[m]); rows that cannot be rebuilt are
    zero."""
    k = G.k
    erased2 = np.asarray(erased, dtype=bool).copy()
    erased2[list(lost)] = True
    x, rec, _, _ = codec.decode(G, c, erased2, maxit)
    known = rec.astype(bool)
    if not known[:b].all():
        x, known, _ = precode_bp(b, k, x, known)
    if known[:b].all():
        x = encode(b, k, x[:b])
        known[:] = True
    t = c.shape[1]
    out = np.zeros((len(lost), t), dtype=np.uint8)
    ok = np.zeros(len(lost), dtype=np.uint8)
    for r, j in enumerate(lost):
        N = [int(i) for i in G.N(j)]
        if all(known[i] for i in N):
            acc = np.zeros(t, dtype=np.uint8)
            for i in N:
                acc ^= x[i]
            out[r], ok[r] = acc, 1
    return out, ok
