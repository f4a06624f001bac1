"""Check #2 / check #3 generation (CGA) and local-group repair (oracle copy).

Test infrastructure: only the tests, the smoke check and the CPU baseline of
the benchmark use this module; the library never does.

Functions and the passage each follows
  cga            Algorithm 4 (§2.6): columns of the generator matrix B (k x n,
                 column j = the inputs of coded block j) absorb other columns
                 (by XOR) whenever that lowers their weight; L(2,3) (n x n,
                 the identity at the start) records which coded blocks each
                 column has become the sum of.  Sweeps over the columns repeat
                 until B has n - k zero columns or a sweep changes nothing.
  split          §2.6: a column of weight one is a check #2 equation (input i
                 = XOR of the coded blocks of its L column), a column of
                 weight zero a check #3 group (its coded blocks XOR to zero);
                 groups ordered by cardinality, smallest first, ties by
                 column.
  set_xor        §2.5, Eqs. (1)-(4): check #3 groups from a check #1 group
                 and the check #2 sets of its members (symmetric difference).
  extra_groups   §2.5: more check #3 groups from check #2 equations: for a
                 coded block j of degree one with input i, S_i xor {j}
                 (c_j = x_i); for a check #1 set D of precoded blocks (XOR
                 zero) whose members all have check #2 sets, the symmetric
                 difference of those sets (Eqs. (1)-(4)).
  with_extra_groups  the groups held with them: new ones that are empty or
                 equal to a held group are skipped, then all are ordered by
                 cardinality (held ones first on ties).
  check_data     §2.7: the integer array of the check data file.  A check #2
                 equation is the record 1, input, L, then the L coded blocks
                 whose XOR is that input; a check #3 group is 0, L, then its
                 L coded blocks.
  parse_check_data  the records of such an array, in file order.
  from_check_data   what the repair engine keeps from it: the first check #2
                 record per input, and the check #3 groups ordered by
                 cardinality (ties in file order), members as sets.
  extend_local   §2.9's update through local groups: the coded rows
                 n_old..n-1 of a longer code made from the existing rows by
                 local_repair over the longer code's check #3 groups, the
                 new rows taking the place of lost ones.
  local_repair   the repair engine's fast path (§2.3, §2.8, §4): BP over the
                 check #3 groups.  At each level every lost coded block
                 still unknown is rebuilt as the XOR of the other members of
                 the first (smallest) group holding it whose other members
                 are all known (neither erased nor lost, or rebuilt at an
                 earlier level); the loop ends when a level rebuilds
                 nothing.  Blocks left unknown are for the conventional
                 repair.

Readings:
  * Columns are bitsets of the k inputs; w() is their number of ones.  A
    column absorbs another when that lowers its weight; the test is made
    against the column's current value, which changes as it absorbs others
    during the same visit.
  * zero_columns counts the zero columns (the text's "nonzero" contradicts
    the loop bound n - k).
  * The check data array is written check #2 records first (ascending
    input), then the check #3 groups in their stored order; the paper leaves
    the record order open.
  * Local repair takes groups in the stored order (smallest first).  The
    repair engine searches the local sets for one unknown in a loop, as BP
    does (§2.8); here the loop is level-synchronous: a block rebuilt at level
    l becomes known for level l + 1.  The set of blocks rebuilt at the end
    does not depend on the order (it is the closure of the one-unknown
    rule); the group chosen per block does.
"""

import numpy as np


def _w(x):
    return bin(x).count("1")


def _pack(sets, width):
    """0/1 bit matrix with one row per set, packed into uint64 words."""
    words = (width + 63) // 64
    M = np.zeros((len(sets), words * 64), dtype=np.uint8)
    for r, s in enumerate(sets):
        M[r, list(s)] = 1
    return np.packbits(M, axis=1, bitorder="little").view(np.uint64)


def _unpack(row):
    return int.from_bytes(row.tobytes(), "little")


def cga(G, max_sweeps=0):
    """Algorithm 4.  Returns (B columns after, L columns after, sweeps), each
    column an int bitset (B over inputs, L over coded blocks).

    Column j of B lowers its weight by absorbing column i exactly when
    w(b_j ^ b_i) = w(b_j) + w(b_i) - 2|b_j & b_i| < w(b_j), that is when
    w(b_i) < 2|b_j & b_i| (which also gives the paper's first test,
    w(b_i) < 2 w(b_j)).  One sweep visits j = 0 .. n-1; for each j, the other
    columns are offered in increasing i, each tested against the current b_j,
    and each that passes is absorbed (b_j ^= b_i, l_j ^= l_i) before the next
    is offered.  Sweeps repeat until n - k columns are zero, a sweep absorbs
    nothing, or max_sweeps (> 0) sweeps ran.

    B and L are held as packed bit matrices (one row per column of the
    paper's matrices); for column j the test is evaluated for every later
    candidate at once, the first passing one is absorbed, and the search
    resumes after it.
    """
    k, n = G.k, G.n
    Bm = _pack([G.N(j) for j in range(n)], k)
    Lm = _pack([[j] for j in range(n)], n)
    w = np.bitwise_count(Bm).sum(axis=1).astype(np.int64)
    sweeps = 0
    while int((w == 0).sum()) < n - k:
        if max_sweeps and sweeps == max_sweeps:
            break
        absorbed = False
        for j in range(n):
            i = 0
            while i < n:
                overlap = np.bitwise_count(Bm[i:] & Bm[j]).sum(axis=1).astype(np.int64)
                passing = w[i:] < 2 * overlap
                if i <= j:
                    passing[j - i] = False
                hits = np.flatnonzero(passing)
                if len(hits) == 0:
                    break
                i += int(hits[0])
                Bm[j] ^= Bm[i]
                Lm[j] ^= Lm[i]
                w[j] = int(np.bitwise_count(Bm[j]).sum())
                absorbed = True
                i += 1
        sweeps += 1
        if not absorbed:
            break
    return [_unpack(r) for r in Bm], [_unpack(r) for r in Lm], sweeps


def _members(x):
    out, s = [], 0
    while x:
        if x & 1:
            out.append(s)
        x >>= 1
        s += 1
    return out


def split(b, L):
    """(check2, check3): check2 maps input i to the coded blocks of the first
    column whose weight-one b is input i; check3 lists coded-block groups,
    smallest first (ties by column index)."""
    check2 = {}
    groups = []
    for j, (bj, lj) in enumerate(zip(b, L)):
        if bj == 0:
            groups.append((_w(lj), j, _members(lj)))
        elif bj & (bj - 1) == 0:
            i = bj.bit_length() - 1
            check2.setdefault(i, _members(lj))
    groups.sort()
    return check2, [g for _, _, g in groups]


def set_xor(sets):
    """Symmetric difference of the given sets (sorted list)."""
    acc = set()
    for s in sets:
        acc ^= set(s)
    return sorted(acc)


def extra_groups(G, check2, check1=None):
    """Groups from degree-one coded blocks (coded block order), then from the
    check #1 sets in check1 (their order), each a sorted list; empty ones are
    left out."""
    out = []
    for j in range(G.n):
        N = [int(i) for i in G.N(j)]
        if len(N) == 1 and N[0] in check2:
            grp = set_xor([check2[N[0]], [j]])
            if grp:
                out.append(grp)
    for D in check1 or ():
        if all(int(i) in check2 for i in D):
            grp = set_xor([check2[int(i)] for i in D])
            if grp:
                out.append(grp)
    return out


def with_extra_groups(check3, extra):
    groups = [list(g) for g in check3]
    seen = {tuple(g) for g in groups}
    for g in extra:
        if tuple(g) not in seen:
            seen.add(tuple(g))
            groups.append(list(g))
    return sorted(groups, key=len)


def check_data(check2, check3):
    """The check data integer array of check #2 equations {input: [coded
    blocks]} and check #3 groups [[coded blocks], ...]."""
    out = []
    for i in sorted(check2):
        out += [1, int(i), len(check2[i])] + [int(m) for m in check2[i]]
    for grp in check3:
        out += [0, len(grp)] + [int(m) for m in grp]
    return out


def parse_check_data(arr):
    """(check #2 records [(input, [coded blocks])], check #3 groups) in file
    order; ValueError for an unknown flag or a record past the end."""
    arr = [int(v) for v in arr]
    c2, c3 = [], []
    p = 0
    while p < len(arr):
        flag = arr[p]
        if flag == 1:
            if p + 3 > len(arr):
                raise ValueError("check #2 record header past the end")
            i, L = arr[p + 1], arr[p + 2]
            if L < 0 or p + 3 + L > len(arr):
                raise ValueError("check #2 record past the end")
            c2.append((i, arr[p + 3:p + 3 + L]))
            p += 3 + L
        elif flag == 0:
            if p + 2 > len(arr):
                raise ValueError("check #3 record header past the end")
            L = arr[p + 1]
            if L < 0 or p + 2 + L > len(arr):
                raise ValueError("check #3 record past the end")
            c3.append(arr[p + 2:p + 2 + L])
            p += 2 + L
        else:
            raise ValueError("unknown record flag %d" % flag)
    return c2, c3


def from_check_data(arr):
    """(check2 {input: sorted coded blocks}, check3 sorted groups ordered by
    size, ties in file order): the equations as the repair engine holds
    them (§2.8 sorts the check #3 groups by cardinality)."""
    c2, c3 = parse_check_data(arr)
    check2 = {}
    for i, members in c2:
        check2.setdefault(i, sorted(members))
    groups = sorted((sorted(g) for g in c3), key=len)
    return check2, groups


def local_repair(groups, c, lost, erased=None, max_levels=0):
    """Returns (blocks[len(lost), t], repaired[len(lost)], group used per
    lost block or -1, level per lost block or -1, levels run).  max_levels
    > 0 stops after that many levels."""
    n, t = c.shape
    lost = [int(s) for s in lost]
    known = np.ones(n, dtype=bool)
    if erased is not None:
        known &= ~np.asarray(erased, dtype=bool)
    known[lost] = False
    work = np.array(c, dtype=np.uint8, copy=True)
    out = np.zeros((len(lost), t), dtype=np.uint8)
    ok = np.zeros(len(lost), dtype=np.uint8)
    used = np.full(len(lost), -1, dtype=np.int64)
    level_of = np.full(len(lost), -1, dtype=np.int64)
    levels = 0
    while not ok.all() and (max_levels == 0 or levels < max_levels):
        picks = []
        for r, s in enumerate(lost):
            if ok[r]:
                continue
            for gi, grp in enumerate(groups):
                if s in grp and all(known[m] for m in grp if m != s):
                    picks.append((r, gi))
                    break
        if not picks:
            break
        for r, gi in picks:
            acc = np.zeros(t, dtype=np.uint8)
            for m in groups[gi]:
                if m != lost[r]:
                    acc ^= work[m]
            out[r], ok[r], used[r], level_of[r] = acc, 1, gi, levels
        for r, _ in picks:
            known[lost[r]] = True
            work[lost[r]] = out[r]
        levels += 1
    return out, ok, used, level_of, levels


def extend_local(groups, c_old, n, erased=None):
    """(rows[n - n_old, t], made[n - n_old], levels): the new coded rows of a
    code grown from n_old = len(c_old) to n rows, rebuilt from the existing
    rows through the check #3 groups of the n-row code.  erased: uint8[n_old]
    (old rows that are unavailable) or None.  Rows no group reaches stay
    zero with made 0."""
    c_old = np.asarray(c_old, dtype=np.uint8)
    n_old, t = c_old.shape
    c = np.zeros((n, t), dtype=np.uint8)
    c[:n_old] = c_old
    er = np.zeros(n, dtype=np.uint8)
    if erased is not None:
        er[:n_old] = np.asarray(erased, dtype=np.uint8)
    rows, made, _, _, levels = local_repair(groups, c, list(range(n_old, n)), er)
    return rows, made, levels
