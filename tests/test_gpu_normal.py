"""GPU direct path (ss_normal_solve) against the FP64 oracle on the same
FP32 matrices: the solution within 1e-7 relative L2 (both sides solve the
same FP64 normal equations; Cholesky rounding grows with cond(B) ~ 1e7),
for the split pair (recombined) and for A itself; and Theorem 2 on the GPU:
the split and unsplit solutions, and the phantom for consistent data, agree
up to the FP32 rounding of the folded values.  Repeated and interleaved
calls (the look-ahead stream and events are reused) are bitwise reproducible."""
import numpy as np
import pytest

from gpu_util import banner, device, rel_l2, to_np
from oracle import geometry as G
from oracle import normal as ON
from oracle import split as OSp
from paper_1902_10559_amd import inputs, native

pytestmark = pytest.mark.gpu


def _table1_problem(n):
    g = inputs.geometry_normal(n)
    A = G.to_fp32(G.system_matrix(g))
    f_true = G.image_to_snake(inputs.phantom_for(6, 0, g))
    p = (A.astype(np.float64) @ f_true).astype(np.float32)
    return A, p, f_true


def _solve(A, p, split):
    import torch
    Ad = device(A)
    pd = torch.from_numpy(np.ascontiguousarray(p, dtype=np.float32)).cuda()
    S = native.fold(Ad, pd) if split else native.unsplit(Ad, pd)
    return to_np(native.normal_solve(S))


def _oracle_split(A, p):
    S32 = OSp.fold(A, "fp32")
    p1, p2 = OSp.fold_p(p.astype(np.float64), "fp32")
    f, _, _ = ON.normal_solve_split(S32, p1.astype(np.float32).astype(np.float64),
                                    p2.astype(np.float32).astype(np.float64))
    return f


def test_split_and_full_normal_solutions_match_the_oracle():
    banner("normal equations 32x32")
    A, p, f_true = _table1_problem(32)
    fs = _solve(A, p, True)
    assert rel_l2(fs, _oracle_split(A, p)) <= 1e-7
    fu = _solve(A, p, False)
    assert rel_l2(fu, ON.normal_solve(A, p.astype(np.float64))) <= 1e-7
    # Theorem 2 on the GPU, up to the FP32 rounding of the folded values and
    # of p (the oracle: 9e-6 apart, both within 1e-5 of the phantom)
    assert rel_l2(fs, fu) <= 1e-4 and rel_l2(fs, f_true) <= 1e-4 and rel_l2(fu, f_true) <= 1e-4


def test_random_full_rank_systems_with_ragged_blocks():
    """Sizes that end in a partial 64-block (n = 1, 65, 133 for the halves;
    2, 130, 266 unsplit), so the factorisation's panel solves and trailing
    updates run with ragged tiles."""
    banner("normal equations random")
    from symm import random_symmetric_sparse
    for seed, M, N in [(41, 4, 2), (42, 300, 130), (43, 600, 266)]:
        rng = np.random.default_rng(seed)
        A = random_symmetric_sparse(rng, M, N, 0.3 if N > 2 else 1.0)
        p = (A.astype(np.float64) @ rng.uniform(0, 1, N) + 0.01 * rng.standard_normal(M)).astype(np.float32)
        S32 = OSp.fold(A, "fp32")
        assert np.linalg.matrix_rank(A.toarray()) == N
        assert np.linalg.matrix_rank(S32.A1().toarray()) == N // 2
        assert rel_l2(_solve(A, p, True), _oracle_split(A, p)) <= 1e-7
        assert rel_l2(_solve(A, p, False), ON.normal_solve(A, p.astype(np.float64))) <= 1e-7


def test_singular_normal_matrix_is_reported():
    """A voxel pair no ray crosses (a zero column of A, and of A(1), A(2))
    gives an exactly zero pivot: SS_E_SHAPE, for both forms."""
    banner("normal equations singular")
    import torch
    A, p, _ = _table1_problem(32)
    N = A.shape[1]
    D = A.tocsc(copy=True)
    for j in (40, N - 1 - 40):
        D.data[D.indptr[j]:D.indptr[j + 1]] = 0
    D.eliminate_zeros()
    D = D.tocsr()
    D.sort_indices()
    pd = torch.from_numpy(np.ascontiguousarray(p)).cuda()
    for split in (True, False):
        Ad = device(D)
        S = native.fold(Ad, pd) if split else native.unsplit(Ad, pd)
        with pytest.raises(native.SSError) as e:
            native.normal_solve(S)
        assert e.value.code == -4


def test_repeated_and_interleaved_solves_are_reproducible():
    """The factorisation's second stream and its events are reused from call
    to call: solves of different sizes and forms, interleaved, give bitwise
    the same results as the first time."""
    import torch
    banner("normal equations repeated")
    A32, p32, _ = _table1_problem(32)
    rng = np.random.default_rng(7)
    from symm import random_symmetric_sparse
    Ar = random_symmetric_sparse(rng, 600, 266, 0.3)
    pr = (Ar.astype(np.float64) @ rng.uniform(0, 1, 266)).astype(np.float32)
    cases = [(A32, p32, True), (Ar, pr, False), (A32, p32, False), (Ar, pr, True)]
    first = [_solve(A, p, split) for A, p, split in cases]
    for (A, p, split), want in zip(cases[::-1], first[::-1]):
        got = _solve(A, p, split)
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
    # on a side stream of the caller's
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        got = _solve(A32, p32, True)
    torch.cuda.synchronize()
    assert np.array_equal(got.view(np.uint64), first[0].view(np.uint64))


def test_replayed_solve_reads_the_current_system():
    """A solve is captured once per shape, workspace and image and then
    replayed: systems with the same n but other rays (m, entries, values),
    solved in turn into the same output, each match their own oracle
    solution, so a replay reads the system it is given."""
    import torch
    banner("normal equations replay with other systems")
    from symm import random_symmetric_sparse
    cases = []
    for seed, M in [(51, 600), (52, 900)]:
        rng = np.random.default_rng(seed)
        A = random_symmetric_sparse(rng, M, 266, 0.3 if M == 600 else 0.2)
        assert np.linalg.matrix_rank(A.toarray()) == 266
        p = (A.astype(np.float64) @ rng.uniform(0, 1, 266)).astype(np.float32)
        cases.append((A, p, _oracle_split(A, p)))
    out = torch.empty(266, dtype=torch.float64, device="cuda")
    for _ in range(2):
        for A, p, want in cases:
            Ad = device(A)
            pd = torch.from_numpy(np.ascontiguousarray(p, dtype=np.float32)).cuda()
            got = to_np(native.normal_solve(native.fold(Ad, pd), out=out))
            assert rel_l2(got, want) <= 1e-7


def test_split_solve_with_large_trailing_updates():
    """Halves of 4864 columns: the first panels' near and far trailing
    updates span more than 4096 rows and take the 128 x 128 tiles (smaller
    updates take 64 x 64 tiles, which the other tests cover)."""
    banner("normal equations with 128 x 128 trailing tiles (halves of 4864)")
    from symm import random_symmetric_sparse
    rng = np.random.default_rng(61)
    A = random_symmetric_sparse(rng, 19456, 9728, 0.01)
    p = (A.astype(np.float64) @ rng.uniform(0, 1, 9728)).astype(np.float32)
    assert rel_l2(_solve(A, p, True), _oracle_split(A, p)) <= 1e-7
