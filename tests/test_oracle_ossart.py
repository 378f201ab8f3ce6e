"""Oracle pins for ordered-subset SART (ref. [004] applied to SART): closed
forms, a hand-written single-ray rule, the fixed point of consistent data,
and the exact equivalence of full and split passes when the subsets are
mirror-paired views."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import geometry as G
from oracle import ossart, sart, split
from paper_1902_10559_amd import inputs
from symm import random_symmetric_sparse


@pytest.mark.parametrize("lam", [0.5, 1.3])
def test_identity_system_has_the_geometric_closed_form(lam):
    rng = np.random.default_rng(4)
    p = rng.standard_normal(9)
    A = sp.identity(9, format="csr")
    subsets = [np.array([0, 4, 8]), np.array([1, 2]), np.array([3, 5, 6, 7])]
    for k in (0, 1, 3, 11):
        f, res = ossart.os_sart_full(A, p, lam, k, subsets)
        assert np.allclose(f, (1 - (1 - lam) ** k) * p, rtol=1e-14, atol=1e-15)
        assert np.isclose(res[k], abs(1 - lam) ** k, rtol=1e-12)


def test_one_subset_is_simultaneous_sart():
    rng = np.random.default_rng(5)
    A = random_symmetric_sparse(rng, 30, 22, 0.3)
    p = rng.standard_normal(30)
    f, res = ossart.os_sart_full(A, p, 0.7, 12, [np.arange(30)])
    fr, rr = sart.sart_full(A, p, 0.7, 12)
    assert np.max(np.abs(f - fr)) < 1e-13 and np.max(np.abs(res - rr)) < 1e-13


def test_single_ray_subsets_follow_the_hand_rule():
    """One ray per subset: V_s[j] = a_ij, so every voxel the ray crosses
    moves by lambda * (p_i - a_i . f) / W_i and the others stay."""
    rng = np.random.default_rng(6)
    D = rng.uniform(0, 1, (4, 5)) * (rng.uniform(0, 1, (4, 5)) < 0.7)
    D[:, 0] += 0.5                       # no empty row
    p = rng.standard_normal(4)
    lam = 0.6
    f_ref = np.zeros(5)
    for _ in range(3):
        for i in range(4):
            W = D[i].sum()
            step = lam * (p[i] - D[i] @ f_ref) / W
            for j in range(5):
                if D[i, j] != 0.0:
                    f_ref[j] += step
    f, _ = ossart.os_sart_full(sp.csr_matrix(D), p, lam, 3, [np.array([i]) for i in range(4)])
    assert np.max(np.abs(f - f_ref)) < 1e-14


def test_consistent_data_converge_to_the_solution():
    rng = np.random.default_rng(7)
    A = rng.uniform(0.0, 0.4, (12, 6)) + np.eye(12, 6)
    f_true = rng.standard_normal(6)
    p = A @ f_true
    subsets = [np.arange(0, 4), np.arange(4, 8), np.arange(8, 12)]
    f, res = ossart.os_sart_full(sp.csr_matrix(A), p, 0.5, 3000, subsets)
    assert np.max(np.abs(f - f_true)) < 1e-10 and res[-1] < 1e-11


def test_mirror_paired_views_are_closed_under_the_ray_mirror():
    full, folded = ossart.mirror_paired_views(8, 5)
    M = 40
    assert sorted(np.concatenate(full).tolist()) == list(range(M))
    for T, F in zip(full, folded):
        assert sorted((M - 1 - T).tolist()) == sorted(T.tolist())
        assert np.all(F < M // 2) and set(F.tolist()) <= set(T.tolist())


@pytest.mark.parametrize("seed", [1, 2])
def test_split_os_sart_equals_full_os_sart(seed):
    rng = np.random.default_rng(seed)
    A = random_symmetric_sparse(rng, 40, 30, 0.25)
    p = rng.standard_normal(40)
    full, folded = ossart.mirror_paired_views(8, 5)
    S = split.fold(A)
    p1, p2 = split.fold_p(p)
    for passes in (1, 4, 15):
        f, res = ossart.os_sart_full(A, p, 0.5, passes, full)
        f1, f2, rs = ossart.os_sart_split(S, p1, p2, 0.5, passes, folded)
        assert np.max(np.abs(res - rs)) < 1e-13
        assert np.max(np.abs(split.recombine(f1, f2) - f)) < 1e-12 * max(1.0, np.abs(f).max())


def test_split_os_sart_equals_full_on_the_64x64_scan():
    g = inputs.geometry_for(1)
    A = G.to_fp32(G.system_matrix(g))
    p = A.astype(np.float64) @ G.image_to_snake(inputs.phantom_for(1, 0, g))
    full, folded = ossart.mirror_paired_views(g.K, g.B)
    f, res = ossart.os_sart_full(A, p, 0.5, 6, full)
    S = split.fold(A)
    p1, p2 = split.fold_p(p)
    f1, f2, rs = ossart.os_sart_split(S, p1, p2, 0.5, 6, folded)
    assert np.max(np.abs(res - rs)) < 1e-12
    assert np.max(np.abs(split.recombine(f1, f2) - f)) < 1e-11 * np.abs(f).max()
    # informative: ordered subsets lower the residual faster per pass than SART
    _, rr = sart.sart_full(A, p, 0.5, 6)
    assert res[6] < rr[6]


def test_underdetermined_passes_settle_above_zero_residual():
    """Documents the limit of ordered subsets with subset column weights: on a
    consistent underdetermined system SART converges to a solution, the
    two-subset passes settle at a fixed point of the pass map instead."""
    rng = np.random.default_rng(0)
    A = sp.csr_matrix(rng.uniform(0, 1, (40, 100)) * (rng.uniform(0, 1, (40, 100)) < 0.3))
    p = A @ rng.uniform(0, 1, 100)
    f, res = ossart.os_sart_full(A, p, 0.5, 3000, [np.arange(0, 20), np.arange(20, 40)])
    _, rs = sart.sart_full(A, p, 0.5, 3000)
    assert rs[-1] < 1e-12 and 1e-3 < res[-1] and abs(res[-1] - res[-500]) < 1e-12
    # a fixed point of the pass map: one more pass leaves the image unchanged
    f2, _ = ossart.os_sart_full(A, p, 0.5, 1, [np.arange(0, 20), np.arange(20, 40)], f0=f)
    assert np.max(np.abs(f2 - f)) < 1e-10 * np.abs(f).max()


def test_nonnegative_split_os_sart_equals_clamped_full():
    rng = np.random.default_rng(3)
    A = random_symmetric_sparse(rng, 40, 30, 0.25)
    p = rng.standard_normal(40)
    full, folded = ossart.mirror_paired_views(8, 5)
    S = split.fold(A)
    p1, p2 = split.fold_p(p)
    f, res = ossart.os_sart_full(A, p, 0.5, 12, full, nonneg=True)
    f1, f2, rs = ossart.os_sart_split(S, p1, p2, 0.5, 12, folded, nonneg=True)
    assert f.min() >= 0.0
    assert np.max(np.abs(res - rs)) < 1e-13
    assert np.max(np.abs(split.recombine(f1, f2) - f)) < 1e-12 * np.abs(f).max()
