"""Simultaneous SART on the full system and on the split pair (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper names SART as the standard iterative reconstruction (Section 1,
its ref. [001], Andersen & Kak 1984) without writing the iteration out.  The
form used here is the simultaneous one, every ray in every iteration (the
form whose convergence for 0 < lambda < 2 is shown in the paper's ref. [003],
Jiang & Wang 2003):

    f^{k+1} = f^k + lambda * V^{-1} A^T W^{-1} (p - A f^k),

W_i = sum_j w_ij (ray lengths), V_j = sum_i w_ij, a zero sum giving a zero
reciprocal; f^0 = 0 unless a start is given; no clamping.

Split form: the same update on each half-system (3), (4) with the sums of A
(equal to the row and column sums of A2) for both halves.  By the
block-diagonal identity behind Theorem 1 (fold(A f) = (A1 f1, A2 f2) for
(f1, f2) = image_fold(f)) and the mirror symmetry of W and V, the split
iterates recombined by eq. (5) are exactly the full iterates, and

    ||p - A f||^2 = (||p1 - A1 f1||^2 + ||p2 - A2 f2||^2) / 2,
    ||p||^2       = (||p1||^2 + ||p2||^2) / 2,

so the relative residual of the full system can be tracked on the halves.

``res[k]`` is ||p - A f^k|| / ||p|| for k = 0..iters (f^k before the k-th
update; res[iters] belongs to the returned image).

Non-negativity (``nonneg``): after every update the image is projected onto
f >= 0, i.e. every voxel is clamped at 0 (the Euclidean projection onto the
non-negative orthant).  On the split pair, voxels j and N-1-j are
f_j = (f2_j + f1_j) / 2 and f_{N-1-j} = (f2_j - f1_j) / 2 by eq. (5), so the
same projection is: clamp both at 0 and map back, f1 = a - b, f2 = a + b.  It
couples the two halves voxel pair by voxel pair only (f2_j >= |f1_j|), and
the split iterates stay exactly the full ones.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .split import Split, reciprocal


def nonneg_pair(f1, f2):
    """The projection onto f >= 0 in split coordinates (see the header)."""
    a = np.maximum(0.5 * (f2 + f1), 0.0)
    b = np.maximum(0.5 * (f2 - f1), 0.0)
    return a - b, a + b


def sart_full(A: sp.csr_matrix, p, lam: float, iters: int, f0=None, sums=None, nonneg=False):
    """``sums`` = (W, V) overrides the row and column sums of A; the 16-bit
    storage variant keeps the sums of the FP32 weights while iterating with
    the rounded ones."""
    A = sp.csr_matrix(A, dtype=np.float64)
    At = A.T.tocsr()
    p = np.asarray(p, dtype=np.float64)
    if sums is None:
        sums = (np.asarray(A.sum(axis=1)).ravel(), np.asarray(A.sum(axis=0)).ravel())
    invW = reciprocal(sums[0])
    invV = reciprocal(sums[1])
    f = np.zeros(A.shape[1]) if f0 is None else np.array(f0, dtype=np.float64)
    pn = np.linalg.norm(p)
    res = np.empty(iters + 1)
    for k in range(iters):
        r = p - A @ f
        res[k] = np.linalg.norm(r) / pn
        f = f + lam * invV * (At @ (invW * r))
        if nonneg:
            f = np.maximum(f, 0.0)
    res[iters] = np.linalg.norm(p - A @ f) / pn
    return f, res


def sart_split(S: Split, p1, p2, lam: float, iters: int, f10=None, f20=None, nonneg=False):
    A1 = sp.csr_matrix((S.v1.astype(np.float64), S.indices, S.indptr),
                       shape=(S.m, S.n))
    A2 = sp.csr_matrix((S.v2.astype(np.float64), S.indices, S.indptr),
                       shape=(S.m, S.n))
    A1t, A2t = A1.T.tocsr(), A2.T.tocsr()
    invW = reciprocal(S.W)
    invV = reciprocal(S.V)
    p1 = np.asarray(p1, dtype=np.float64)
    p2 = np.asarray(p2, dtype=np.float64)
    f1 = np.zeros(S.n) if f10 is None else np.array(f10, dtype=np.float64)
    f2 = np.zeros(S.n) if f20 is None else np.array(f20, dtype=np.float64)
    pn = np.sqrt(0.5 * (p1 @ p1 + p2 @ p2))
    res = np.empty(iters + 1)
    for k in range(iters):
        r1 = p1 - A1 @ f1
        r2 = p2 - A2 @ f2
        res[k] = np.sqrt(0.5 * (r1 @ r1 + r2 @ r2)) / pn
        f1 = f1 + lam * invV * (A1t @ (invW * r1))
        f2 = f2 + lam * invV * (A2t @ (invW * r2))
        if nonneg:
            f1, f2 = nonneg_pair(f1, f2)
    r1 = p1 - A1 @ f1
    r2 = p2 - A2 @ f2
    res[iters] = np.sqrt(0.5 * (r1 @ r1 + r2 @ r2)) / pn
    return f1, f2, res
