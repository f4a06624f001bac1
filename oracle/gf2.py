"""Dense GF(2) view of the code, for pins on tiny graphs (oracle copy).

Algorithms 1 and 5 of the paper take the generator matrix B in F_2^{k x n};
column g of B is the indicator of N(g), and the coded symbols are c = B^T x
over GF(2), applied independently to every bit of the payload (§2.2).  These
routines are the textbook definitions, kept separate from the sparse code in
``codec`` so that each can check the other:

  dense_B      B as a 0/1 matrix (k x n)
  encode_bits  c = B^T x on the bit planes of x (np.unpackbits, integer
               matrix product reduced mod 2, np.packbits)
  rank         rank over GF(2) by Gaussian elimination on Python-int bitsets
  ml_set       inputs i for which the unit vector e_i lies in the span of the
               surviving columns of B: exactly the inputs any decoder (peeling
               or maximum likelihood) could determine from the survivors

Pinned by (tests): rank and ml_set equal the span listed element by element
(the XOR of every subset of the surviving columns) over every survivor set of
tiny graphs; hand cases where peeling recovers nothing but ML recovers all,
where no unit vector is in the span, and where an input lies in no surviving
row; ml_set is all inputs exactly at full rank.
"""

import numpy as np


def dense_B(G):
    B = np.zeros((G.k, G.n), dtype=np.uint8)
    for g in range(G.n):
        B[G.N(g), g] = 1
    return B


def encode_bits(B, x):
    """c = B^T x over GF(2), bit plane by bit plane."""
    bits = np.unpackbits(np.asarray(x, dtype=np.uint8), axis=1).astype(np.int64)   # k x 8t
    cb = (B.T.astype(np.int64) @ bits) % 2                                          # n x 8t
    return np.packbits(cb.astype(np.uint8), axis=1)


def _col_bitsets(B, cols):
    out = []
    for g in cols:
        v = 0
        for i in np.flatnonzero(B[:, g]):
            v |= 1 << int(i)
        out.append(v)
    return out


def _reduce_basis(vectors):
    """Row-echelon basis keyed by leading bit."""
    basis = {}
    for v in vectors:
        while v:
            h = v.bit_length() - 1
            if h in basis:
                v ^= basis[h]
            else:
                basis[h] = v
                break
    return basis


def rank(B, cols):
    return len(_reduce_basis(_col_bitsets(B, cols)))


def in_span(basis, v):
    while v:
        h = v.bit_length() - 1
        if h not in basis:
            return False
        v ^= basis[h]
    return True


def ml_set(B, cols):
    """Inputs determinable from the listed coded columns (sorted list)."""
    basis = _reduce_basis(_col_bitsets(B, cols))
    k = B.shape[0]
    return [i for i in range(k) if in_span(basis, 1 << i)]
