"""Oracle pins for SART: closed forms, the limit, and the exact equivalence of
full and split iterations."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import geometry as G
from oracle import sart, split
from paper_1902_10559_amd import inputs
from symm import random_symmetric_sparse


@pytest.mark.parametrize("lam", [0.5, 1.0, 1.7])
def test_identity_system_has_the_geometric_closed_form(lam):
    rng = np.random.default_rng(0)
    p = rng.standard_normal(6)
    A = sp.identity(6, format="csr")
    for k in (0, 1, 2, 5, 13):
        f, res = sart.sart_full(A, p, lam, k)
        assert np.allclose(f, (1 - (1 - lam) ** k) * p, rtol=1e-14, atol=1e-15)
        assert np.isclose(res[k], abs(1 - lam) ** k, rtol=1e-12)


@pytest.mark.parametrize("M,N", [(8, 6), (6, 10)])
def test_limit_is_the_weighted_minimum_norm_least_squares_solution(M, N):
    rng = np.random.default_rng(M + N)
    A = rng.uniform(0.0, 0.3, (M, N)) + np.eye(M, N)
    p = rng.standard_normal(M)
    W = A.sum(axis=1)
    V = A.sum(axis=0)
    Bm = A / np.sqrt(W)[:, None] / np.sqrt(V)[None, :]
    closed = (np.linalg.pinv(Bm) @ (p / np.sqrt(W))) / np.sqrt(V)
    s = np.linalg.svd(Bm, compute_uv=False)
    assert abs(s[0] - 1.0) < 1e-12      # the SART-normalised matrix has norm 1
    lam = 1.0
    smin = s[s > 1e-10].min()
    iters = int(np.ceil(np.log(1e-14) / np.log(1 - lam * smin ** 2)))
    assert iters < 200000
    f, _ = sart.sart_full(sp.csr_matrix(A), p, lam, iters)
    assert np.max(np.abs(f - closed)) < 1e-10


def _random_problem(seed, M=40, N=30, density=0.25):
    rng = np.random.default_rng(seed)
    A = random_symmetric_sparse(rng, M, N, density)
    p = rng.standard_normal(M).astype(np.float32)  # inconsistent data
    return A, p


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_split_sart_equals_full_sart_at_every_iteration(seed):
    A, p = _random_problem(seed)
    S = split.fold(A)
    p1, p2 = split.fold_p(p)
    f, res = sart.sart_full(A, p, 0.5, 50)
    f1, f2, res_s = sart.sart_split(S, p1, p2, 0.5, 50)
    assert np.max(np.abs(res - res_s)) < 1e-13
    assert np.max(np.abs(split.recombine(f1, f2) - f)) < 1e-12 * np.abs(f).max()
    for k in (1, 7, 23):
        fk, _ = sart.sart_full(A, p, 0.5, k)
        g1, g2, _ = sart.sart_split(S, p1, p2, 0.5, k)
        assert np.max(np.abs(split.recombine(g1, g2) - fk)) < 1e-12 * max(1, np.abs(fk).max())


def test_split_needs_the_sums_of_A_not_the_absolute_sums_of_A1():
    # the reading the split rests on: both halves use W, V of A (= A2's);
    # normalising A1 by its own absolute sums gives a different iteration
    A, p = _random_problem(4)
    S = split.fold(A)
    p1, p2 = split.fold_p(p)
    f, _ = sart.sart_full(A, p, 0.5, 50)
    rows = np.repeat(np.arange(S.m), np.diff(S.indptr))
    alt = split.Split(**{**S.__dict__,
                         "W": np.bincount(rows, weights=np.abs(S.v1), minlength=S.m),
                         "V": np.bincount(S.indices, weights=np.abs(S.v1),
                                          minlength=S.n)})
    a1, _, _ = sart.sart_split(alt, p1, p2, 0.5, 50)
    _, a2, _ = sart.sart_split(S, p1, p2, 0.5, 50)
    assert np.max(np.abs(split.recombine(a1, a2) - f)) > 1e-3 * np.abs(f).max()


def test_residual_identity_of_the_halves():
    A, p = _random_problem(5)
    S = split.fold(A)
    rng = np.random.default_rng(5)
    f = rng.standard_normal(A.shape[1])
    f1, f2 = split.image_fold(f)
    p1, p2 = split.fold_p(p)
    r = p - A @ f
    r1 = p1 - S.A1() @ f1
    r2 = p2 - S.A2() @ f2
    assert np.isclose(r @ r, 0.5 * (r1 @ r1 + r2 @ r2), rtol=1e-13)
    pp = p.astype(np.float64)
    assert np.isclose(pp @ pp, 0.5 * (p1 @ p1 + p2 @ p2), rtol=1e-13)


def test_warm_start_resume_equals_one_long_run():
    A, p = _random_problem(6)
    S = split.fold(A)
    p1, p2 = split.fold_p(p)
    f1, f2, _ = sart.sart_split(S, p1, p2, 0.5, 20)
    h1, h2, _ = sart.sart_split(S, p1, p2, 0.5, 10)
    g1, g2, _ = sart.sart_split(S, p1, p2, 0.5, 10, h1, h2)
    assert np.array_equal(f1, g1) and np.array_equal(f2, g2)


def test_cfg1_full_and_split_agree_and_the_residual_falls():
    g = inputs.geometry_cfg1()
    A = G.to_fp32(G.system_matrix(g))
    f_true = G.image_to_snake(inputs.phantom_for(1, 0, g))
    q = A.astype(np.float64) @ f_true
    p = inputs.add_noise(q, inputs.noise_draws(1, 0, g.M), G.row_sums(A) > 0, 0.005)
    S = split.fold(A)
    p1, p2 = split.fold_p(p)
    f, res = sart.sart_full(A, p, 0.5, 20)
    f1, f2, res_s = sart.sart_split(S, p1, p2, 0.5, 20)
    assert np.max(np.abs(res - res_s)) < 1e-13
    assert np.max(np.abs(split.recombine(f1, f2) - f)) < 1e-12 * np.abs(f).max()
    assert res[0] == pytest.approx(1.0) and res[-1] < 0.1
    assert np.all(np.diff(res) < 0)


def test_explicit_sums_equal_default_sums_when_they_are_the_matrix_sums():
    A, p = _random_problem(7)
    W = np.asarray(A.astype(np.float64).sum(axis=1)).ravel()
    V = np.asarray(A.astype(np.float64).sum(axis=0)).ravel()
    f, r = sart.sart_full(A, p, 0.5, 15)
    g, s = sart.sart_full(A, p, 0.5, 15, sums=(W, V))
    assert np.array_equal(f, g) and np.array_equal(r, s)
    # and they matter: scaled sums give a different iterate
    h, _ = sart.sart_full(A, p, 0.5, 15, sums=(2 * W, V))
    assert np.max(np.abs(h - f)) > 1e-3 * np.abs(f).max()


@pytest.mark.parametrize("lam", [0.5, 1.2])
def test_nonnegative_identity_system_closed_form(lam):
    """A = I: a voxel with p_j < 0 stays at 0 (every step would go
    negative), the others follow the unconstrained closed form."""
    p = np.array([0.7, -0.4, 1.3, -2.0, 0.0, 0.25])
    A = sp.identity(6, format="csr")
    for k in (1, 2, 9):
        f, _ = sart.sart_full(A, p, lam, k, nonneg=True)
        want = np.where(p > 0, (1 - (1 - lam) ** k) * p, 0.0)
        assert np.allclose(f, want, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("seed", [4, 5])
def test_nonnegative_split_sart_equals_clamped_full_sart(seed):
    A, p = _random_problem(seed)            # inconsistent data: the clamp is active
    S = split.fold(A)
    p1, p2 = split.fold_p(p)
    f, res = sart.sart_full(A, p, 0.5, 40, nonneg=True)
    f_free, _ = sart.sart_full(A, p, 0.5, 40)
    assert f.min() >= 0.0 and f_free.min() < -1e-3      # the constraint binds
    f1, f2, res_s = sart.sart_split(S, p1, p2, 0.5, 40, nonneg=True)
    assert np.max(np.abs(res - res_s)) < 1e-13
    assert np.max(np.abs(split.recombine(f1, f2) - f)) < 1e-12 * np.abs(f).max()
    assert np.all(f2 >= np.abs(f1) - 1e-15)


def test_nonneg_pair_is_the_clamp_of_the_recombined_image():
    rng = np.random.default_rng(9)
    f = rng.standard_normal(20)
    f1, f2 = split.image_fold(f)
    g1, g2 = sart.nonneg_pair(f1, f2)
    assert np.allclose(split.recombine(g1, g2), np.maximum(f, 0.0), atol=1e-15)
