"""Encode, peeling decode, repair and update of the LDGM code (oracle copy).

Payloads are byte blocks: x is uint8[k, t] (input symbols), c is uint8[n, t]
(coded symbols), block-major, t % 8 == 0.  All payload arithmetic is bytewise
XOR, i.e. GF(2) (§2.2, "region XOR"), so no rounding is involved anywhere and
every comparison against the library is exact.

Functions and the passage each follows
  encode        §2.2 encoding step 2: c_g = XOR of x_i over N(g).
  peel_schedule Algorithm 5 (DPG) with the level-synchronous ("delayed") BP
                of §3.1: level i uses only symbols decoded at earlier levels;
                each newly decodable input f is paired with ONE degree-1 coded
                symbol, the one of lowest degree.
  replay        §3.1: x_f = c_g XOR (XOR of x_i, i in N(g) minus f), level by
                level in schedule order.
  decode        peel_schedule + replay; unrecovered inputs are zero-filled.
  bp_sequential Algorithm 1 as a queue-driven (Gauss-Seidel) peel, used only
                to cross-check the recovered set (§3.1 states both orders reach
                the same union of decoded sets).
  repair_from_inputs   conventional re-encoding of lost coded rows when the
                inputs are at hand (§4, "re-run partial encoding").
  extend        §2.9: new coded rows n_old..n-1 of a longer (prefix-stable)
                graph, from the inputs or, as repair does, from the existing rows
  repair_conventional  §4: decode the survivors, then re-encode each lost row
                whose neighbours were all recovered.
  update        replace some input blocks; the definition is re-encoding from
                scratch, which by linearity of the region XOR equals adding
                each input delta into every adjacent coded block.

Readings taken where Algorithms 1/5 are silent or garbled:
  * maxit == 0 means no limit (at most k levels); otherwise at most maxit
    levels are run.  The iteration counter of Algorithm 1 is never advanced in
    the listing; it is read as the level count.
  * "g_d is minimum" is the ORIGINAL degree d_g of the coded row; ties go to
    the lowest row index g.  This choice changes only which row decodes f,
    never the value of x_f.
  * |DP| = 2k on success counts the 2k elements of k pairs.
  * Within a level the pairs are listed by ascending f.
  * A decode failure is a result (ok = 0, |F| > 0), not an error.

Pinned by (tests): decode(encode(x)) == x when ok; x restricted to R equals the
input on failure and F is zero; the recovered set agrees with bp_sequential
and with random-order peels; R is contained in the ML-decodable set of the
GF(2) survivor matrix and ok implies rank k, over ALL erasure patterns of tiny
graphs; F is a stopping set; encode equals the dense bit-plane product B^T x.
"""

import numpy as np


def _xor_rows(blocks):
    """XOR-reduce a stack of byte blocks (shape [m, t]) to one block."""
    if len(blocks) == 0:
        raise ValueError("empty XOR")
    return np.bitwise_xor.reduce(np.ascontiguousarray(blocks).view(np.uint64), axis=0).view(np.uint8)


def encode(G, x, rows=None):
    """c[g] = XOR_{i in N(g)} x[i] for every coded row g (or the listed rows)."""
    x = np.ascontiguousarray(x, dtype=np.uint8)
    assert x.shape[0] == G.k and x.shape[1] % 8 == 0
    rows = range(G.n) if rows is None else rows
    out = np.zeros((len(rows), x.shape[1]), dtype=np.uint8)
    for r, g in enumerate(rows):
        out[r] = _xor_rows(x[G.N(g)])
    return out


class Schedule:
    """Result of the peeling schedule.

    levels   list of lists of (f, g) pairs, one list per level, f ascending
    F        sorted array of unrecovered inputs
    """

    def __init__(self, k, levels, F):
        self.k = k
        self.levels = levels
        self.F = np.asarray(sorted(F), dtype=np.int64)

    @property
    def L(self):
        return len(self.levels)

    @property
    def ok(self):
        return len(self.F) == 0

    def recovered_mask(self):
        m = np.ones(self.k, dtype=np.uint8)
        m[self.F] = 0
        return m

    def status(self):
        return (int(self.ok), int(len(self.F)), int(self.L))

    def flat(self):
        """(level_ptr, dp_f, dp_g) in the library's output layout."""
        level_ptr = [0]
        dp_f, dp_g = [], []
        for lev in self.levels:
            for f, g in lev:
                dp_f.append(f)
                dp_g.append(g)
            level_ptr.append(len(dp_f))
        return (np.array(level_ptr, dtype=np.int64), np.array(dp_f, dtype=np.int64),
                np.array(dp_g, dtype=np.int64))


def peel_schedule(G, erased, maxit=0):
    """Algorithm 5 (DPG) with level-synchronous peeling (§3.1).

    At level i, with F the inputs not yet decoded:
      * C keeps the columns of the surviving coded rows with the rows of the
        decoded inputs zeroed, so weight(c_{:,g}) = |N(g) & F|;
      * G_i = surviving rows g with |N(g) & F| == 1, each naming its single
        remaining input f(g);
      * every f named by some row is decoded at this level by the naming row
        of minimum (original degree d_g, row index g);
      * F loses the decoded inputs.
    Stops when F is empty, no surviving row has weight 1, or maxit levels ran.
    """
    k, n = G.k, G.n
    erased = np.asarray(erased, dtype=bool)
    assert erased.shape == (n,)
    survivors = np.flatnonzero(~erased)
    deg = G.degrees()
    in_F = np.ones(k, dtype=bool)
    # row index of every edge, to reduce per coded row
    edge_row = np.repeat(np.arange(n), deg)
    levels = []
    while in_F.any() and (maxit == 0 or len(levels) < maxit):
        # the edges g -> i with i still in F; weight(g) = |N(g) & F|
        live = in_F[G.col]
        weight = np.bincount(edge_row[live], minlength=n)
        # for a row of weight 1, its one live edge names f(g)
        f_of = np.full(n, -1, dtype=np.int64)
        f_of[edge_row[live]] = G.col[live]
        ripple = [g for g in survivors if weight[g] == 1]
        if not ripple:
            break
        best = {}
        for g in ripple:
            f = int(f_of[g])
            key = (int(deg[g]), int(g))
            if f not in best or key < best[f]:
                best[f] = key
        level = [(f, best[f][1]) for f in sorted(best)]
        levels.append(level)
        for f, _ in level:
            in_F[f] = False
    return Schedule(k, levels, np.flatnonzero(in_F))


def replay(G, c, sched, t=None):
    """Numeric pass of the schedule: x_f = c_g ^ XOR(x_i, i in N(g), i != f)."""
    c = np.ascontiguousarray(c, dtype=np.uint8)
    t = c.shape[1] if t is None else t
    x = np.zeros((G.k, t), dtype=np.uint8)
    done = np.zeros(G.k, dtype=bool)
    for level in sched.levels:
        for f, g in level:
            others = [i for i in G.N(g) if i != f]
            assert all(done[i] for i in others), "schedule uses an undecoded input"
            acc = c[g].copy()
            if others:
                acc ^= _xor_rows(x[others])
            x[f] = acc
        for f, _ in level:
            done[f] = True
    # inputs in F stay zero
    return x


def decode(G, c, erased, maxit=0):
    """Peeling decode: returns (x, recovered mask, (ok, |F|, levels), schedule)."""
    sched = peel_schedule(G, erased, maxit)
    x = replay(G, c, sched)
    return x, sched.recovered_mask(), sched.status(), sched


def bp_sequential(G, erased, order=None):
    """Algorithm 1 read as a sequential peel: returns the recovered set.

    A queue holds surviving rows whose residual weight is 1; popping one
    decodes its last unknown input, which lowers the weight of every other
    surviving row on that input.  ``order`` optionally permutes the initial
    queue (any processing order must reach the same set, §3.1).
    """
    k, n = G.k, G.n
    erased = np.asarray(erased, dtype=bool)
    weight = G.degrees().astype(np.int64).copy()
    recovered = np.zeros(k, dtype=bool)
    queue = [g for g in range(n) if not erased[g] and weight[g] == 1]
    if order is not None:
        rng = np.random.default_rng(order)
        rng.shuffle(queue)
    while queue:
        g = queue.pop(0) if order is None else queue.pop(int(rng.integers(len(queue))))
        unknown = [int(i) for i in G.N(g) if not recovered[i]]
        if len(unknown) != 1:
            continue
        f = unknown[0]
        recovered[f] = True
        for h in G.NT(f):
            weight[h] -= 1
            if not erased[h] and weight[h] == 1:
                queue.append(int(h))
    return recovered


def repair_from_inputs(G, x, lost):
    """Re-encode the lost coded rows from the inputs: c_j = XOR_{i in N(j)} x_i."""
    return encode(G, x, rows=list(lost))


def repair_conventional(G, c, erased, lost, maxit=0):
    """§4 conventional repair: decode from the survivors that are not lost,
    then re-encode each lost row whose neighbours were all recovered.

    Returns (blocks[m, t], repaired[m]); rows that cannot be rebuilt are zero.
    """
    erased2 = np.asarray(erased, dtype=bool).copy()
    erased2[list(lost)] = True
    x, rec, _, _ = decode(G, c, erased2, maxit)
    t = c.shape[1]
    out = np.zeros((len(lost), t), dtype=np.uint8)
    ok = np.zeros(len(lost), dtype=np.uint8)
    for r, j in enumerate(lost):
        if all(rec[i] for i in G.N(j)):
            out[r] = _xor_rows(x[G.N(j)])
            ok[r] = 1
    return out, ok


def extend(G, n_old, x=None, c_old=None, erased=None, maxit=0):
    """The paper's update (§2.9): the code gains coded blocks n_old..n-1 of the
    graph G (whose first n_old rows are those of the original graph: rows
    depend only on their own index) without any change to the existing ones.

    With the inputs x the new blocks are their encode.  Without them they are
    made the way the repair engine makes missing blocks (§4): decode from the
    existing blocks c_old[0:n_old] that are not erased, then encode each new
    row whose neighbours were all recovered; the others stay zero.

    Returns (blocks[n - n_old, t], made[n - n_old]).
    """
    new_rows = list(range(n_old, G.n))
    if x is not None:
        return encode(G, x, rows=new_rows), np.ones(len(new_rows), dtype=np.uint8)
    t = c_old.shape[1]
    c = np.zeros((G.n, t), dtype=np.uint8)
    c[:n_old] = c_old[:n_old]
    er = np.zeros(G.n, dtype=bool)
    if erased is not None:
        er[:n_old] = np.asarray(erased, dtype=bool)[:n_old]
    return repair_conventional(G, c, er, new_rows, maxit)


def update(G, x, ids, new_blocks):
    """Definition of the update: replace x[ids] by new_blocks, re-encode all rows."""
    x2 = np.array(x, dtype=np.uint8, copy=True)
    ids = list(ids)
    assert len(set(ids)) == len(ids)
    x2[ids] = new_blocks
    return x2, encode(G, x2)


def affected_rows(G, ids):
    """Coded rows adjacent to at least one updated input (ascending)."""
    s = set()
    for i in ids:
        s.update(int(h) for h in G.NT(i))
    return sorted(s)
