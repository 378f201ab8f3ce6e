"""Helpers for the GPU parity tests: problems built by the oracle, handed to
the library through its C ABI, and results read back for comparison."""
from __future__ import annotations

import dataclasses
import functools
import sys

import numpy as np
import scipy.sparse as sp

from oracle import geometry as G
from oracle import split as OSp
from paper_1902_10559_amd import inputs, native


def banner(msg: str) -> None:
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@dataclasses.dataclass
class Problem:
    A: sp.csr_matrix   # FP32 weights
    p: np.ndarray      # FP32
    f_true: np.ndarray


@functools.lru_cache(maxsize=None)
def problem(cfg: int, item: int = 0) -> Problem:
    g = inputs.geometry_for(cfg)
    A = G.to_fp32(G.system_matrix(g))
    f_true = G.image_to_snake(inputs.phantom_for(cfg, item, g))
    wl = inputs.WORKLOADS[cfg]
    q = A.astype(np.float64) @ f_true
    p = inputs.add_noise(q, inputs.noise_draws(cfg, item, g.M), G.row_sums(A) > 0, wl.noise)
    return Problem(A, p, f_true)


def random_problem(seed: int, M: int, N: int, density: float) -> Problem:
    from symm import random_symmetric_sparse
    rng = np.random.default_rng(seed)
    A = random_symmetric_sparse(rng, M, N, density)
    # a few empty rows and columns, kept symmetric
    D = A.toarray()
    for i in rng.choice(M // 2, size=min(3, M // 2 - 1), replace=False):
        D[i, :] = 0
        D[M - 1 - i, :] = 0
    for j in rng.choice(N // 2, size=min(3, N // 2 - 1), replace=False):
        D[:, j] = 0
        D[:, N - 1 - j] = 0
    A = sp.csr_matrix(D.astype(np.float32))
    A.eliminate_zeros()
    A.sort_indices()
    f_true = rng.uniform(0, 1, N)
    p = (A.astype(np.float64) @ f_true + 0.01 * rng.standard_normal(M)).astype(np.float32)
    return Problem(A, p, f_true)


def host_matrix(A: sp.csr_matrix) -> native.HostMatrix:
    A = sp.csr_matrix(A, dtype=np.float32)
    A.sort_indices()
    Ac = A.tocsc()
    Ac.sort_indices()
    return native.HostMatrix(A.shape[0], A.shape[1], A.nnz, A.indptr.astype(np.int64),
                             A.indices.astype(np.int32), A.data, Ac.indptr.astype(np.int64),
                             Ac.indices.astype(np.int32), Ac.data)


def device(A: sp.csr_matrix):
    return native.to_device(host_matrix(A), "cuda")


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def split_values(S: native.System, csc: bool = False):
    """(v1, v2) of a folded system as FP64, decoding 16-bit storage."""
    raw = to_np(S.val_t if csc else S.val)
    if S.wdtype == "f32":
        v = raw.reshape(-1, 2).astype(np.float64)
        return v[:, 0], v[:, 1]
    bits = raw.view(np.uint16).reshape(-1, 2)
    if S.wdtype == "f16":
        v = bits.view(np.float16).astype(np.float64)
    else:
        v = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return v[:, 0], v[:, 1]


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_fold32(A: sp.csr_matrix):
    return OSp.fold(A, "fp32")


def assert_res_close(got, want):
    """Residual histories agree to 1e-5 relative, down to the FP32 floor: the
    GPU forms r = p - q in FP32, so |r| carries an absolute error of order
    eps32 * |p| (eps32 = 6e-8) times a small growth factor; 1e-6 in units of
    ||p|| covers it."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    assert got.shape == want.shape
    assert np.all(np.abs(got - want) <= 1e-5 * np.abs(want) + 1e-6), (got, want)
