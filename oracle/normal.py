"""The direct path: normal equations of the full system and of the split
pair (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Theorem 2: the normal pseudo-solutions of systems (3) and (4), recombined by
eq. (5), are the normal pseudo-solution of (1).  When A has full column rank
that is the least-squares solution, the unique solution of the normal
equations A^T A f = A^T p; the paper's remark after eq. (13) gives the split
normal matrices as B(k) = A(k)^T A(k) (the fold of B = A^T A).  The paper's
Table 1 times a direct method on these systems; here the normal equations are
solved by a Cholesky factorisation (a library routine, used as one step).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .split import Split, recombine


def normal_solve(A, p):
    """f = (A^T A)^{-1} A^T p by Cholesky, FP64."""
    A = sp.csr_matrix(A, dtype=np.float64)
    B = (A.T @ A).toarray()
    c = A.T @ np.asarray(p, dtype=np.float64)
    return sla.cho_solve(sla.cho_factor(B, lower=True), c)


def normal_solve_split(S: Split, p1, p2):
    """Both halves' normal equations B(k) f(k) = A(k)^T p(k), recombined by
    eq. (5); also returns the halves."""
    A1 = sp.csr_matrix((S.v1.astype(np.float64), S.indices, S.indptr), shape=(S.m, S.n))
    A2 = sp.csr_matrix((S.v2.astype(np.float64), S.indices, S.indptr), shape=(S.m, S.n))
    f1 = normal_solve(A1, p1)
    f2 = normal_solve(A2, p2)
    return recombine(f1, f2), f1, f2
