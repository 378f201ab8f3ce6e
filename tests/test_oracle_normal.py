"""Oracle pins for the direct (normal-equation) path: the Cholesky solve is
the least-squares solution (checked against an SVD-based solver), the split
solve recombines to the full one (Theorem 2), and the Table 1 geometry has
full column rank."""
import numpy as np
import pytest

from oracle import geometry as G
from oracle import normal, split
from paper_1902_10559_amd import inputs
from symm import random_symmetric_sparse


def _full_rank_problem(seed, M=60, N=24):
    rng = np.random.default_rng(seed)
    A = random_symmetric_sparse(rng, M, N, 0.4)
    assert np.linalg.matrix_rank(A.toarray()) == N
    return A, rng.standard_normal(M)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_cholesky_solve_is_the_least_squares_solution(seed):
    A, p = _full_rank_problem(seed)
    f = normal.normal_solve(A, p)
    f_ls = np.linalg.lstsq(A.toarray(), p, rcond=None)[0]
    assert np.max(np.abs(f - f_ls)) < 1e-11 * max(1.0, np.abs(f_ls).max())


@pytest.mark.parametrize("seed", [4, 5])
def test_split_normal_solution_recombines_to_the_full_one(seed):
    A, p = _full_rank_problem(seed)
    S = split.fold(A)
    p1, p2 = split.fold_p(p)
    f_split, f1, f2 = normal.normal_solve_split(S, p1, p2)
    f = normal.normal_solve(A, p)
    assert np.max(np.abs(f_split - f)) < 1e-11 * max(1.0, np.abs(f).max())
    # Theorem 2's norm identity
    assert np.isclose(f @ f, 0.5 * (f1 @ f1 + f2 @ f2), rtol=1e-12)


def test_table1_geometry_has_full_column_rank_and_mirror_symmetry():
    g = inputs.geometry_normal(32)
    A = G.system_matrix(g)
    assert A.shape == (2304, 1024) and G.is_symmetric(A)
    w = np.linalg.eigvalsh((A.T @ A).toarray())
    assert w[0] > 1e-9 * w[-1]            # positive definite: cond(B) ~ 1e7
    S = split.fold(A)
    for A_half in (S.A1(), S.A2()):
        wh = np.linalg.eigvalsh((A_half.T @ A_half).toarray())
        assert wh[0] > 1e-9 * wh[-1]
