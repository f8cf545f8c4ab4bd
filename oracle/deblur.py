"""FP64 oracle pieces for the compressed-deblurring shape of Section 7.

Test infrastructure only (like the rest of `oracle/`): the product never
imports it.

Section 7 models the blur as a circulant B obtained by right-circulating a
row vector b whose first L entries are 1/L (b_j = 1/L for j < L, else 0), so
B[i, j] = b[(j - i) mod n], and composes it with the circulant sensing
matrix: A = P C B.  A product of circulants is circulant; its generator
(first column) is C times the first column of B, beta[i] = B[i, 0] =
b[(-i) mod n].  This module writes that definition out.
"""
import numpy as np


def box_first_column(n, L):
    """First column of B: beta[i] = b[(-i) mod n] with b_j = 1/L for j < L."""
    b = np.zeros(n)
    b[:L] = 1.0 / L
    return b[(-np.arange(n)) % n]


def composite_generator(c, L):
    """Generator of C B: (C beta)[k] = sum_i c[(k - i) mod n] beta[i], summed
    over the L nonzeros of beta (FP64)."""
    c = np.asarray(c, dtype=np.float64)
    n = c.size
    beta = box_first_column(n, L)
    out = np.zeros(n)
    k = np.arange(n)
    for i in np.flatnonzero(beta):
        out += c[(k - i) % n] * beta[i]
    return out


def dense_circulant(col):
    """Dense circulant with the given first column: M[i, j] = col[(i - j) mod n]."""
    col = np.asarray(col, dtype=np.float64)
    n = col.size
    idx = (np.arange(n)[:, None] - np.arange(n)[None, :]) % n
    return col[idx]


def dense_box_blur(n, L):
    """B from its definition: right-circulated rows of b."""
    b = np.zeros(n)
    b[:L] = 1.0 / L
    idx = (np.arange(n)[None, :] - np.arange(n)[:, None]) % n
    return b[idx]
