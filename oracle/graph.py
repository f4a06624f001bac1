"""Seeded LDGM bipartite graph (oracle copy).

§2.2 of the paper: each of the n coded symbols ("check node c" in the Omega
passage) gets a degree c_d from the degree distribution and c_d distinct
input symbols chosen pseudo-randomly; the coded symbol is their region XOR.
The graph is a function of the seed alone, so it can be regenerated (§2.2).
The generator matrix B in F_2^{k x n} of Algorithms 1 and 5 has column g equal
to the indicator of the neighbour set N(g) of coded symbol g.

Per coded row j (reading taken for the unspecified sampler):
  key  = stream_key(seed, GRAPH, stripe_key, j)
  d_j  = sample_degree(draw(key, 0), T)
  N(j) = Floyd's sample of d_j distinct values from [0, k) (Bentley & Floyd,
         CACM 1987): for s = 0..d-1, r = k - d + s, v = ((draw(key, s+1) >> 32)
         * (r + 1)) >> 32 (Lemire's multiply-shift range reduction); take r
         if v was already taken, else v.  The row is then sorted ascending.

CSR by coded row (row_ptr[n+1], col[nnz]) and CSC by input (col_ptr[k+1],
rowidx[nnz], rows ascending within a column) describe the same B.

Pinned by: distinctness/sortedness, CSC == transpose of CSR, prefix stability
in n, chi-square of degrees and uniform neighbour marginals (tests), and
bit-exact agreement with the library's independent C++ builder.
"""

from dataclasses import dataclass

import numpy as np

from . import dist, prng


@dataclass
class GraphParams:
    k: int
    n: int
    dist: str = "rsd"            # "rsd" | "finite" | "raptor"
    rsd_c: float = 0.1
    rsd_delta: float = 0.05
    finite_w: tuple = ()         # w_1..w_D for dist == "finite"
    seed: int = 1
    stripe_key: int = 0


@dataclass
class Graph:
    k: int
    n: int
    row_ptr: np.ndarray   # int64[n+1]
    col: np.ndarray       # int64[nnz], ascending within each row
    col_ptr: np.ndarray   # int64[k+1]
    rowidx: np.ndarray    # int64[nnz], ascending within each column

    @property
    def nnz(self):
        return int(self.row_ptr[-1])

    def deg(self, j):
        return int(self.row_ptr[j + 1] - self.row_ptr[j])

    def degrees(self):
        return np.diff(self.row_ptr)

    def N(self, j):
        """Sorted neighbour list of coded row j."""
        return self.col[self.row_ptr[j]:self.row_ptr[j + 1]]

    def NT(self, i):
        """Sorted list of coded rows adjacent to input i."""
        return self.rowidx[self.col_ptr[i]:self.col_ptr[i + 1]]


def degree_weights(p: GraphParams):
    if p.dist == "rsd":
        w, _, _ = dist.rsd_weights(p.k, p.rsd_c, p.rsd_delta)
        return w
    if p.dist == "finite":
        return dist.finite_weights(list(p.finite_w), p.k)
    if p.dist == "raptor":
        return dist.raptor_weights(p.k)
    raise dist.DistError("unknown distribution " + repr(p.dist))


def floyd_sample(key, m, N):
    """m distinct values of [0, N) from draws 1..m of ``key``, sorted."""
    chosen = set()
    for s in range(m):
        r = N - m + s
        v = ((prng.draw(key, s + 1) >> 32) * (r + 1)) >> 32
        chosen.add(r if v in chosen else v)
    return sorted(chosen)


def row_neighbours(p: GraphParams, T, j):
    key = prng.stream_key(p.seed, prng.PURPOSE_GRAPH, p.stripe_key, j)
    d = dist.sample_degree(prng.draw(key, 0), T)
    return floyd_sample(key, d, p.k)


def build(p: GraphParams) -> Graph:
    """Build the graph row by row, then its transpose by counting sort."""
    if p.k < 1 or p.n < 1:
        raise dist.DistError("need k >= 1 and n >= 1")
    T = dist.thresholds(degree_weights(p))
    rows = [row_neighbours(p, T, j) for j in range(p.n)]
    row_ptr = np.zeros(p.n + 1, dtype=np.int64)
    for j, r in enumerate(rows):
        row_ptr[j + 1] = row_ptr[j] + len(r)
    col = np.array([i for r in rows for i in r], dtype=np.int64)
    return with_transpose(p.k, p.n, row_ptr, col)


def with_transpose(k, n, row_ptr, col):
    """Attach the CSC (rows ascending per input) to a CSR description."""
    counts = np.zeros(k + 1, dtype=np.int64)
    for i in col:
        counts[i + 1] += 1
    col_ptr = np.cumsum(counts)
    fill = col_ptr[:-1].copy()
    rowidx = np.zeros(len(col), dtype=np.int64)
    for j in range(n):                       # rows visited in ascending order
        for i in col[row_ptr[j]:row_ptr[j + 1]]:
            rowidx[fill[i]] = j
            fill[i] += 1
    return Graph(k, n, row_ptr, np.asarray(col, dtype=np.int64), col_ptr, rowidx)


def from_rows(k, rows):
    """A graph given explicitly by its neighbour lists (for worked examples)."""
    n = len(rows)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    flat = []
    for j, r in enumerate(rows):
        r = sorted(set(int(i) for i in r))
        assert all(0 <= i < k for i in r)
        flat.extend(r)
        row_ptr[j + 1] = len(flat)
    return with_transpose(k, n, row_ptr, np.array(flat, dtype=np.int64))
