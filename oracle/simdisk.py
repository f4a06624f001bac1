"""Disk-failure reliability sweep ("simDisk") of the LDGM code (oracle copy).

Test infrastructure: only the tests, the smoke check and the CPU baseline of
the benchmark use this module; the library never does.

The utility functions of §2.1 include one that exhausts every combination of
disk failures for given code parameters; §2.2 states what it answers: with the
n coded symbols spread over s drives, which of the f-failure combinations the
code tolerates, i.e. from which the decoder still recovers every input.

Readings (the paper gives no formula for them):
  striping      the coded symbols are spread over the s drives equally and in
                order (the measurements of §5 spread the encoded data over 10
                disks equally): disk d holds rows [floor(d n / s),
                floor((d+1) n / s)), so every disk holds n/s rows when s
                divides n and the sizes differ by at most one otherwise.
  combinations  every f-subset of the s disks, in lexicographic order of the
                sorted disk lists (rank 0 = disks 0..f-1).
  tolerable     the peeling decode (codec.peel_schedule) with the rows of the
                failed disks erased ends with no undecoded input.  The result
                of each combination is the decoder's status triple
                {ok, |F|, levels}.

Functions
  disk_rows       rows of one disk under the striping above.
  combinations    the f-subsets in rank order (a library enumeration).
  erased_mask     the erasure vector of one combination.
  sim_disks       status triples of the combinations of ranks
                  [first, first + count).
  sim_disks_precoded  the same with the array-LDPC precode of b data blocks:
                  tolerable means every data block recovered by the two-stage
                  decode (§2.2); status {ok, data blocks missing, LDGM levels,
                  precode levels}, as precode.decode_two_stage reports it.
"""

import itertools
import math

import numpy as np

from . import codec, precode


def disk_rows(n, s, d):
    """Coded rows on disk d of s (equal, in-order striping of n rows)."""
    assert 1 <= s <= n and 0 <= d < s
    return range(d * n // s, (d + 1) * n // s)


def combinations(s, f):
    """Every f-subset of range(s), in lexicographic order."""
    return list(itertools.combinations(range(s), f))


def erased_mask(n, s, failed):
    er = np.zeros(n, dtype=np.uint8)
    for d in failed:
        er[list(disk_rows(n, s, d))] = 1
    return er


def sim_disks(G, s, f, first=0, count=None, maxit=0):
    """int32[count, 3]: the decoder's status for each failure combination."""
    total = math.comb(s, f)
    count = total - first if count is None else count
    assert 0 <= first and first + count <= total
    combos = combinations(s, f)[first:first + count]
    out = np.zeros((count, 3), dtype=np.int32)
    for r, failed in enumerate(combos):
        sched = codec.peel_schedule(G, erased_mask(G.n, s, failed), maxit)
        out[r] = sched.status()
    return out


def sim_disks_precoded(G, b, s, f, first=0, count=None, maxit=0):
    """int32[count, 4]: the two-stage decoder's status for each combination."""
    total = math.comb(s, f)
    count = total - first if count is None else count
    assert 0 <= first and first + count <= total
    combos = combinations(s, f)[first:first + count]
    out = np.zeros((count, 4), dtype=np.int32)
    for r, failed in enumerate(combos):
        sched = codec.peel_schedule(G, erased_mask(G.n, s, failed), maxit)
        known = np.ones(G.k, dtype=bool)
        known[sched.F] = False
        levels2 = 0
        if not known[:b].all():
            # the second pass on the symbols alone (zero-width blocks)
            _, known, levels2 = precode.precode_bp(b, G.k, np.zeros((G.k, 0), np.uint8), known)
        miss = int(b - known[:b].sum())
        out[r] = (int(miss == 0), miss, int(sched.L), int(levels2))
    return out
