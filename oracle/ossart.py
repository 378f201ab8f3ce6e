"""Ordered-subset SART with mirror-paired subsets (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper lists ordered subsets of projection data (its ref. [004], Hudson &
Larkin 1994) among the ways of speeding SART up (Section 1).  Applied to SART
(ref. [001]): the rays are partitioned into subsets T_1 .. T_S, and one pass
applies, for s = 1 .. S in this order,

    f <- f + lambda * V_s^{-1} A_s^T W_s^{-1} (p_s - A_s f),

where A_s holds the rows of T_s, W_s their row sums (the same W_i as in
SART) and V_s[j] = sum_{i in T_s} w_ij; a zero sum gives a zero reciprocal.
With one subset this is simultaneous SART.

Mirror pairing.  If every subset is closed under the ray mirror i -> M-1-i
(for the symmetric scan: the rays of sources k and K-1-k), the fold sends
T_s to a set of rows of the folded system, and the subset column sums of A
equal those of A(2) over the folded rows (substitute eq. (2), as for the
full sums).  The block-diagonal identity behind Theorem 1 then holds for
every sub-step, so split OS-SART with those sums, recombined by eq. (5), is
full OS-SART at every sub-step.  Subsets that are not closed under the mirror
have no split counterpart.

``res[k]`` is ||p - A f^k|| / ||p|| for f^k the image after k passes,
k = 0 .. passes.

Behaviour (observed with this oracle, not a claim of the paper): every
subset step uses its own column weights V_s, so the pass map is not a
projection in one common metric.  For a consistent overdetermined system of
full rank the passes converge to the solution, but on underdetermined
systems they can settle at a fixed point of the pass map with a nonzero
residual (0.019 for a random 40 x 100 system; the noise-free 64 x 64 scan is
still at 2.5e-3 after 3000 passes, where SART reaches 3e-4), while the first
passes lower the residual several times faster than SART iterations do.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .sart import nonneg_pair
from .split import Split, reciprocal


def mirror_paired_views(K: int, B: int):
    """Subsets for a scan of K sources (K even) and B bins, rays ordered
    i = k*B + b: subset s holds the rays of sources s and K-1-s (s < K/2).
    Returns (full, folded): row-index arrays of A, and of the folded system
    (rows s*B .. s*B+B-1 of m = K*B/2)."""
    assert K % 2 == 0
    full, folded = [], []
    for s in range(K // 2):
        a = np.arange(s * B, (s + 1) * B)
        b = np.arange((K - 1 - s) * B, (K - s) * B)
        full.append(np.concatenate([a, b]))
        folded.append(a.copy())
    return full, folded


def _subset_sums(A: sp.csr_matrix, rows):
    sub = A[rows, :]
    return sub, sub.T.tocsr(), reciprocal(np.asarray(sub.sum(axis=0)).ravel())


def os_sart_full(A: sp.csr_matrix, p, lam: float, passes: int, subsets, f0=None, nonneg=False):
    """``nonneg``: clamp the image at 0 after every subset step."""
    A = sp.csr_matrix(A, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    invW = reciprocal(np.asarray(A.sum(axis=1)).ravel())
    parts = [(rows,) + _subset_sums(A, rows) for rows in subsets]
    f = np.zeros(A.shape[1]) if f0 is None else np.array(f0, dtype=np.float64)
    pn = np.linalg.norm(p)
    res = np.empty(passes + 1)
    for k in range(passes):
        res[k] = np.linalg.norm(p - A @ f) / pn
        for rows, As, Ast, invVs in parts:
            r = p[rows] - As @ f
            f = f + lam * invVs * (Ast @ (invW[rows] * r))
            if nonneg:
                f = np.maximum(f, 0.0)
    res[passes] = np.linalg.norm(p - A @ f) / pn
    return f, res


def os_sart_split(S: Split, p1, p2, lam: float, passes: int, folded_subsets, f10=None, f20=None,
                  nonneg=False):
    """Both halves of the folded pair, normalised by A(2)'s row sums and
    A(2)'s column sums over each folded subset."""
    A1 = sp.csr_matrix((S.v1.astype(np.float64), S.indices, S.indptr), shape=(S.m, S.n))
    A2 = sp.csr_matrix((S.v2.astype(np.float64), S.indices, S.indptr), shape=(S.m, S.n))
    invW = reciprocal(S.W)
    parts = []
    for rows in folded_subsets:
        A1s, A2s = A1[rows, :], A2[rows, :]
        invVs = reciprocal(np.asarray(A2s.sum(axis=0)).ravel())
        parts.append((rows, A1s, A1s.T.tocsr(), A2s, A2s.T.tocsr(), invVs))
    p1 = np.asarray(p1, dtype=np.float64)
    p2 = np.asarray(p2, dtype=np.float64)
    f1 = np.zeros(S.n) if f10 is None else np.array(f10, dtype=np.float64)
    f2 = np.zeros(S.n) if f20 is None else np.array(f20, dtype=np.float64)
    pn = np.sqrt(0.5 * (p1 @ p1 + p2 @ p2))

    def rel():
        r1, r2 = p1 - A1 @ f1, p2 - A2 @ f2
        return np.sqrt(0.5 * (r1 @ r1 + r2 @ r2)) / pn
    res = np.empty(passes + 1)
    for k in range(passes):
        res[k] = rel()
        for rows, A1s, A1st, A2s, A2st, invVs in parts:
            z1 = invW[rows] * (p1[rows] - A1s @ f1)
            z2 = invW[rows] * (p2[rows] - A2s @ f2)
            f1 = f1 + lam * invVs * (A1st @ z1)
            f2 = f2 + lam * invVs * (A2st @ z2)
            if nonneg:
                f1, f2 = nonneg_pair(f1, f2)
    res[passes] = rel()
    return f1, f2, res
