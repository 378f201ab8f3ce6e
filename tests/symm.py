"""Test helpers: random matrices that satisfy the symmetry (2) of the paper,
w[i, j] == w[M-1-i, N-1-j] (0-based), built by mirroring a random top half."""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def random_symmetric_dense(rng, M: int, N: int, density: float = 1.0,
                           positive: bool = False, integer: bool = False):
    assert M % 2 == 0 and N % 2 == 0
    m = M // 2
    if integer:
        top = rng.integers(-9, 10, size=(m, N)).astype(np.float64)
    elif positive:
        top = rng.uniform(0.1, 1.0, size=(m, N))
    else:
        top = rng.standard_normal((m, N))
    if density < 1.0:
        top = top * (rng.random((m, N)) < density)
    return np.vstack([top, top[::-1, ::-1]])


def random_symmetric_sparse(rng, M: int, N: int, density: float,
                            dtype=np.float32) -> sp.csr_matrix:
    """Positive weights (like ray lengths), FP32-valued, CSR with ascending
    columns; rows and columns may be empty."""
    A = random_symmetric_dense(rng, M, N, density=density, positive=True)
    A = sp.csr_matrix(A.astype(dtype))
    A.eliminate_zeros()
    A.sort_indices()
    return A
