"""Fold of a symmetric system into two quarter-size systems, and back (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

0-based forms of the paper's formulas (Section 2, the definitions of A(1),
A(2), p(1), p(2) after eqs. (3)-(4); Theorem 1, eq. (5)), with m = M/2 and
n = N/2:

    A1[i, j] = A[i, j] - A[M-1-i, j],   A2[i, j] = A[i, j] + A[M-1-i, j]
    p1[i]    = p[i] - p[M-1-i],         p2[i]    = p[i] + p[M-1-i]
    f[j]     = (f2[j] + f1[j]) / 2,     f[N-1-j] = (f2[j] - f1[j]) / 2

for i < m, j < n.  The inverse of (5), used to split a start image, is the
transform from the proof of Theorem 1: f1[j] = f[j] - f[N-1-j],
f2[j] = f[j] + f[N-1-j].

Stored pattern: A1 and A2 are kept on one shared pattern, the union of the
stored positions of A[i, j] and A[M-1-i, j]; an absent term counts as +0.0,
and entries of A1 that cancel are kept as explicit zeros.  Rows and columns
ascend in both the CSR and the CSC copies.

Two precisions of the folded values are provided: ``fold64`` keeps them in
FP64 (exact, since each is one sum of two FP32 numbers), and ``fold32`` rounds
that FP64 result once to FP32.  An FP64 add of two FP32 operands followed by
one rounding to FP32 equals the FP32 add itself (double rounding is innocuous
for +, -, *, / and sqrt when the wider format has at least 2p+2 bits:
Figueroa, "When is double rounding innocuous?", 1995), so ``fold32`` is what a
correctly rounded FP32 fold produces bit for bit.

Normalisation sums for SART on the split pair are those of A itself:
W_i = sum_j A[i, j] and V_j = sum_i A[i, j], which equal the row sums and
column sums of A2 (substitute eq. (2) into the definition of A2).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class Split:
    m: int
    n: int
    # shared pattern, CSR order (row-major, ascending columns)
    indptr: np.ndarray
    indices: np.ndarray
    v1: np.ndarray
    v2: np.ndarray
    # same entries in CSC order (column-major, ascending rows)
    cindptr: np.ndarray
    cindices: np.ndarray
    cv1: np.ndarray
    cv2: np.ndarray
    W: np.ndarray  # (m,) FP64 row sums of A restricted to rows < m
    V: np.ndarray  # (n,) FP64 column sums of A restricted to cols < n

    @property
    def nnz(self) -> int:
        return int(self.indices.shape[0])

    def A1(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.v1, self.indices, self.indptr),
                             shape=(self.m, self.n))

    def A2(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.v2, self.indices, self.indptr),
                             shape=(self.m, self.n))


def _fold_terms(A: sp.csr_matrix):
    """For every position (i, j) of the shared pattern, the two FP64 terms
    a = A[i, j] and b = A[M-1-i, j] (0 where not stored), in CSR order."""
    M, N = A.shape
    assert M % 2 == 0 and N % 2 == 0, "M and N must be even"
    m, n = M // 2, N // 2
    C = A.tocoo()
    r = C.row.astype(np.int64)
    c = C.col.astype(np.int64)
    v = C.data.astype(np.float64)
    top = (r < m) & (c < n)       # A[i, j],       i < m
    bot = (r >= m) & (c < n)      # A[M-1-i, j],   row M-1-r -> i
    rows = np.concatenate([r[top], M - 1 - r[bot]])
    cols = np.concatenate([c[top], c[bot]])
    a = np.concatenate([v[top], np.zeros(int(bot.sum()))])
    b = np.concatenate([np.zeros(int(top.sum())), v[bot]])
    key = rows * n + cols
    uniq, inv = np.unique(key, return_inverse=True)
    a_u = np.bincount(inv, weights=a, minlength=uniq.shape[0])
    b_u = np.bincount(inv, weights=b, minlength=uniq.shape[0])
    # each position receives at most one term of each kind
    assert np.all(np.bincount(inv, weights=(a != 0)) <= 1)
    return m, n, uniq // n, uniq % n, a_u, b_u


def fold(A: sp.csr_matrix, precision: str = "fp64") -> Split:
    """A -> (A1, A2) on the shared pattern; ``precision`` is 'fp64' (exact)
    or 'fp32' (each value rounded once to FP32)."""
    m, n, i, j, a, b = _fold_terms(A)
    v1 = a - b
    v2 = a + b
    if precision == "fp32":
        v1 = v1.astype(np.float32)
        v2 = v2.astype(np.float32)
    else:
        assert precision == "fp64"
    indptr = np.zeros(m + 1, np.int64)
    np.add.at(indptr, i + 1, 1)
    indptr = np.cumsum(indptr)
    corder = np.lexsort((i, j))
    cindptr = np.zeros(n + 1, np.int64)
    np.add.at(cindptr, j + 1, 1)
    cindptr = np.cumsum(cindptr)
    W = np.bincount(i, weights=a + b, minlength=m)
    V = np.bincount(j, weights=a + b, minlength=n)
    return Split(m=m, n=n, indptr=indptr, indices=j.astype(np.int32),
                 v1=v1, v2=v2, cindptr=cindptr,
                 cindices=i[corder].astype(np.int32), cv1=v1[corder],
                 cv2=v2[corder], W=W, V=V)


def fold_p(p: np.ndarray, precision: str = "fp64"):
    """p -> (p1, p2)."""
    p = np.asarray(p, dtype=np.float64)
    M = p.shape[0]
    assert M % 2 == 0
    m = M // 2
    top = p[:m]
    mir = p[::-1][:m]  # p[M-1-i]
    p1, p2 = top - mir, top + mir
    if precision == "fp32":
        return p1.astype(np.float32), p2.astype(np.float32)
    return p1, p2


def reciprocal(s: np.ndarray, precision: str = "fp64") -> np.ndarray:
    """1/s with 0 where s == 0 (a ray missing the grid, or a voxel no ray
    crosses, is left out of the update)."""
    s = np.asarray(s, dtype=np.float64)
    out = np.zeros_like(s)
    nz = s != 0
    out[nz] = 1.0 / s[nz]
    return out.astype(np.float32) if precision == "fp32" else out


def recombine(f1: np.ndarray, f2: np.ndarray, precision: str = "fp64"):
    """Theorem 1, eq. (5): f from the half-solutions."""
    f1 = np.asarray(f1, dtype=np.float64)
    f2 = np.asarray(f2, dtype=np.float64)
    n = f1.shape[0]
    if precision == "fp32":
        hi = (f2 + f1).astype(np.float32) * np.float32(0.5)
        lo = (f2 - f1).astype(np.float32) * np.float32(0.5)
    else:
        hi = (f2 + f1) / 2
        lo = (f2 - f1) / 2
    f = np.empty(2 * n, dtype=hi.dtype)
    f[:n] = hi
    f[n:] = lo[::-1]  # f[N-1-j] = (f2[j] - f1[j]) / 2
    return f


def image_fold(f: np.ndarray, precision: str = "fp64"):
    """Inverse of eq. (5) (the f-transform in the proof of Theorem 1)."""
    f = np.asarray(f, dtype=np.float64)
    N = f.shape[0]
    assert N % 2 == 0
    n = N // 2
    top = f[:n]
    mir = f[::-1][:n]
    f1, f2 = top - mir, top + mir
    if precision == "fp32":
        return f1.astype(np.float32), f2.astype(np.float32)
    return f1, f2


def round_storage(v32: np.ndarray, dtype: str) -> np.ndarray:
    """FP32 values rounded to nearest-even 16-bit storage, returned as FP64
    numbers (dtype 'bf16' or 'f16').

    bf16 keeps FP32's exponent and 8 significand bits: the two bf16 numbers
    bracketing x are x's FP32 bits truncated to the top 16 (toward zero) and
    the next bf16 away from zero; the nearer wins, and on a tie the one whose
    last kept bit is 0.  f16 uses numpy's IEEE binary16 conversion, which
    rounds to nearest-even."""
    v32 = np.asarray(v32, dtype=np.float32)
    if dtype == "f16":
        with np.errstate(over="ignore"):  # beyond the binary16 range: +-inf, as intended
            return v32.astype(np.float16).astype(np.float64)
    assert dtype == "bf16"
    bits = v32.view(np.uint32).astype(np.uint64)
    lo_bits = (bits & 0xFFFF0000).astype(np.uint32)
    hi_bits = (lo_bits.astype(np.uint64) + 0x10000).astype(np.uint32)
    lo = lo_bits.view(np.float32).astype(np.float64)
    hi = hi_bits.view(np.float32).astype(np.float64)
    x = v32.astype(np.float64)
    dlo, dhi = np.abs(x - lo), np.abs(hi - x)
    lo_even = (lo_bits & 0x10000) == 0
    pick_lo = (dlo < dhi) | ((dlo == dhi) & lo_even)
    return np.where(pick_lo, lo, hi)


def storage_bits(v32: np.ndarray, dtype: str) -> np.ndarray:
    """uint16 bit patterns of ``round_storage``."""
    r = round_storage(v32, dtype)
    if dtype == "f16":
        return r.astype(np.float16).view(np.uint16)
    return (r.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
