"""Oracle pins for the fold, Theorem 1, Theorem 2, eq. (13) and the identities
behind them, on random matrices satisfying eq. (2)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import geometry as G
from oracle import split
from symm import random_symmetric_dense, random_symmetric_sparse


@pytest.mark.parametrize("M,N", [(10, 6), (12, 8), (20, 4)])
def test_theorem1_recovers_f_true_from_exact_half_solutions(M, N):
    rng = np.random.default_rng(M * 100 + N)
    for _ in range(5):
        A = random_symmetric_dense(rng, M, N)
        f_true = rng.standard_normal(N)
        p = A @ f_true
        S = split.fold(sp.csr_matrix(A))
        p1, p2 = split.fold_p(p)
        f1 = np.linalg.lstsq(S.A1().toarray(), p1, rcond=None)[0]
        f2 = np.linalg.lstsq(S.A2().toarray(), p2, rcond=None)[0]
        f = split.recombine(f1, f2)
        assert np.max(np.abs(f - f_true)) < 1e-10
        assert np.max(np.abs(A @ f - p)) < 1e-10


@pytest.mark.parametrize("M,N", [(6, 10), (10, 6), (8, 8), (4, 12)])
def test_theorem2_recombined_pseudo_solutions_are_the_full_one(M, N):
    rng = np.random.default_rng(M * 31 + N)
    for rank_deficient in (False, True):
        A = random_symmetric_dense(rng, M, N, integer=True)
        if rank_deficient:
            A[:, 1] = A[:, 0]
            A[:, N - 2] = A[:, N - 1]   # keeps eq. (2)
        assert np.array_equal(A, A[::-1, ::-1])
        p = rng.standard_normal(M)  # inconsistent in general
        S = split.fold(sp.csr_matrix(A))
        p1, p2 = split.fold_p(p)
        f1 = np.linalg.pinv(S.A1().toarray()) @ p1
        f2 = np.linalg.pinv(S.A2().toarray()) @ p2
        f = split.recombine(f1, f2)
        assert np.allclose(f, np.linalg.pinv(A) @ p, atol=1e-11, rtol=0)
        # the norm identity used in the proof of Theorem 2
        assert np.isclose(f @ f, 0.5 * (f1 @ f1) + 0.5 * (f2 @ f2), rtol=1e-13)


def test_fold_block_identity_and_inverse_pair():
    rng = np.random.default_rng(3)
    A = random_symmetric_dense(rng, 14, 10)
    S = split.fold(sp.csr_matrix(A))
    for _ in range(5):
        f = rng.standard_normal(10)
        f1, f2 = split.image_fold(f)
        q1, q2 = split.fold_p(A @ f)
        assert np.allclose(S.A1() @ f1, q1, atol=1e-13)
        assert np.allclose(S.A2() @ f2, q2, atol=1e-13)
        assert np.allclose(split.recombine(f1, f2), f, atol=1e-15)
        g1, g2 = split.image_fold(split.recombine(f1, f2))
        assert np.allclose(g1, f1, atol=1e-15) and np.allclose(g2, f2, atol=1e-15)


@pytest.mark.parametrize("n", [2, 4, 6, 10])
def test_eq13_determinant_factorises(n):
    rng = np.random.default_rng(n)
    for _ in range(4):
        A = random_symmetric_dense(rng, n, n)
        S = split.fold(sp.csr_matrix(A))
        d = np.linalg.det(A)
        d12 = np.linalg.det(S.A1().toarray()) * np.linalg.det(S.A2().toarray())
        assert np.isclose(d, d12, rtol=1e-10, atol=1e-12)


def test_normal_matrix_is_symmetric_and_folds_into_half_normal_matrices():
    rng = np.random.default_rng(11)
    A = random_symmetric_dense(rng, 12, 8)
    B = A.T @ A
    assert np.allclose(B, B[::-1, ::-1], atol=1e-13)
    SA = split.fold(sp.csr_matrix(A))
    SB = split.fold(sp.csr_matrix(B))
    A1, A2 = SA.A1().toarray(), SA.A2().toarray()
    assert np.allclose(SB.A1().toarray(), A1.T @ A1, atol=1e-12)
    assert np.allclose(SB.A2().toarray(), A2.T @ A2, atol=1e-12)


def test_fold_sums_equal_the_sums_of_A_and_of_A2():
    rng = np.random.default_rng(5)
    A = random_symmetric_sparse(rng, 40, 30, density=0.2)
    S = split.fold(A, "fp64")
    m, n = 20, 15
    assert np.allclose(S.W, G.row_sums(A)[:m], rtol=1e-14, atol=0)
    assert np.allclose(S.V, G.col_sums(A)[:n], rtol=1e-14, atol=0)
    assert np.allclose(S.W, np.asarray(S.A2().sum(axis=1)).ravel(), rtol=1e-14)
    assert np.allclose(S.V, np.asarray(S.A2().sum(axis=0)).ravel(), rtol=1e-14)
    # symmetric halves of the sums: W[M-1-i] = W[i]
    WA = G.row_sums(A)
    assert np.allclose(WA, WA[::-1], rtol=1e-14)


def test_fp32_fold_is_the_correctly_rounded_fp32_add_and_subtract():
    rng = np.random.default_rng(9)
    # FP32 values spanning many binades, with exact cancellations mixed in
    a = (rng.standard_normal(200000) * 10.0 ** rng.integers(-8, 8, 200000)).astype(np.float32)
    b = (rng.standard_normal(200000) * 10.0 ** rng.integers(-8, 8, 200000)).astype(np.float32)
    b[::7] = a[::7]
    d64 = (a.astype(np.float64) - b.astype(np.float64)).astype(np.float32)
    s64 = (a.astype(np.float64) + b.astype(np.float64)).astype(np.float32)
    with np.errstate(over="ignore"):
        d32 = a - b
        s32 = a + b
    assert np.array_equal(d64.view(np.uint32), d32.view(np.uint32))
    assert np.array_equal(s64.view(np.uint32), s32.view(np.uint32))
    # and the oracle's fold32 goes through exactly that path
    A = random_symmetric_sparse(rng, 16, 12, density=0.5)
    S = split.fold(A, "fp32")
    D = A.toarray()
    want1 = D[:8, :6] - D[::-1][:8, :6]
    assert np.array_equal(S.A1().toarray().view(np.uint32),
                          want1.astype(np.float32).view(np.uint32))


def test_shared_pattern_keeps_cancelled_entries_and_csc_matches_csr():
    rng = np.random.default_rng(21)
    A = random_symmetric_sparse(rng, 24, 18, density=0.3).toarray()
    A[3, 4] = A[24 - 1 - 3, 4] = 0.75  # A1[3,4] cancels to +0.0
    A[24 - 1 - 3, 18 - 1 - 4] = A[3, 18 - 1 - 4] = 0.75   # keep eq. (2)
    A = sp.csr_matrix(A.astype(np.float32))
    assert G.is_symmetric(A)
    S = split.fold(A, "fp32")
    D = A.toarray()
    union = (D[:12, :9] != 0) | (D[::-1][:12, :9] != 0)
    assert S.nnz == union.sum()
    k = S.indptr[3] + np.searchsorted(S.indices[S.indptr[3]:S.indptr[4]], 4)
    assert S.indices[k] == 4 and S.v1[k] == 0 and not np.signbit(S.v1[k])
    # CSC copy holds the same entries
    rows = np.repeat(np.arange(S.m), np.diff(S.indptr))
    csr = sorted(zip(rows, S.indices, S.v1, S.v2))
    cols = np.repeat(np.arange(S.n), np.diff(S.cindptr))
    csc = sorted(zip(S.cindices, cols, S.cv1, S.cv2))
    assert csr == csc
    for j in range(S.n):
        seg = S.cindices[S.cindptr[j]:S.cindptr[j + 1]]
        assert np.all(np.diff(seg) > 0)


def test_bf16_and_f16_rounding_match_library_conversions():
    import torch
    rng = np.random.default_rng(13)
    v = (rng.standard_normal(100000) * 10.0 ** rng.integers(-6, 6, 100000)).astype(np.float32)
    # exact ties: bf16 values plus half a bf16 ulp
    base = (v.view(np.uint32) & 0xFFFF0000).view(np.float32)
    ties = (base.view(np.uint32) | 0x8000).view(np.float32)
    v = np.concatenate([v, ties, np.float32([0.0, -0.0, 1.0, 3.0e38, -1.5e-40])])
    want = torch.from_numpy(v).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(split.storage_bits(v, "bf16"), want)
    with np.errstate(over="ignore"):  # 3e38 rounds to inf in binary16
        assert np.array_equal(split.storage_bits(v, "f16"), v.astype(np.float16).view(np.uint16))
    # rounding is to nearest: error at most half an ulp of 8 (bf16) bits
    r = split.round_storage(v[:100000], "bf16")
    nz = v[:100000] != 0
    assert np.max(np.abs(r[nz] - v[:100000][nz]) / np.abs(v[:100000][nz])) <= 2.0 ** -8
