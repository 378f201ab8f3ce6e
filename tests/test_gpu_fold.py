"""GPU fold (ss_fold_size / ss_fold / ss_unsplit) against the oracle.

Bar: the shared pattern and every folded value bit-exact (one FP32 add or
subtract per entry, then round-to-nearest-even for 16-bit storage), p1/p2
bit-exact, and the reciprocal sums within one FP32 ulp (the FP64 sums are
taken in a different order on each side)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from conftest import GOLDEN
from gpu_util import banner, device, oracle_fold32, problem, random_problem, split_values, to_np
from oracle import split as OSp
from paper_1902_10559_amd import native

pytestmark = pytest.mark.gpu


def _fold(A, p, wdtype="f32"):
    import torch
    Ad = device(A)
    pd = torch.from_numpy(np.ascontiguousarray(p, dtype=np.float32)).cuda()
    return Ad, pd, native.fold(Ad, pd, wdtype)


def _ulps(a, b):
    a = np.asarray(a, np.float32).view(np.int32).astype(np.int64)
    b = np.asarray(b, np.float32).view(np.int32).astype(np.int64)
    return np.abs(a - b)


def _check_against_oracle(A, p, S, wdtype="f32"):
    ref = oracle_fold32(A)
    assert S.nnz == ref.nnz
    assert np.array_equal(to_np(S.row_ptr), ref.indptr)
    assert np.array_equal(to_np(S.col_idx), ref.indices)
    assert np.array_equal(to_np(S.col_ptr), ref.cindptr)
    assert np.array_equal(to_np(S.row_idx), ref.cindices)
    v1, v2 = split_values(S)
    c1, c2 = split_values(S, csc=True)
    if wdtype == "f32":
        want = [ref.v1, ref.v2, ref.cv1, ref.cv2]
        got = [v1, v2, c1, c2]
        for g, w in zip(got, want):
            assert np.array_equal(g.astype(np.float32).view(np.uint32), w.view(np.uint32))
    else:
        for g, w in zip([v1, v2, c1, c2], [ref.v1, ref.v2, ref.cv1, ref.cv2]):
            assert np.array_equal(g, OSp.round_storage(w, wdtype))
    p1, p2 = OSp.fold_p(p, "fp32")
    pp = to_np(S.p).reshape(-1, 2)
    assert np.array_equal(pp[:, 0].view(np.uint32), p1.view(np.uint32))
    assert np.array_equal(pp[:, 1].view(np.uint32), p2.view(np.uint32))
    inv_r = OSp.reciprocal(ref.W, "fp32")
    inv_c = OSp.reciprocal(ref.V, "fp32")
    assert _ulps(to_np(S.inv_row), inv_r).max() <= 1
    assert _ulps(to_np(S.inv_col), inv_c).max() <= 1
    assert np.array_equal(to_np(S.inv_row) == 0, inv_r == 0)


def test_fold_example1_reproduces_the_printed_systems():
    banner("fold example 1")
    ex = json.load(open(os.path.join(GOLDEN, "example1.json")))
    A = sp.csr_matrix(np.array(ex["A"], np.float32))
    p = np.array(ex["p"], np.float32)
    _, _, S = _fold(A, p)
    v1, v2 = split_values(S)
    rows = np.repeat(np.arange(S.m), np.diff(to_np(S.row_ptr)))
    D1 = np.zeros((S.m, S.n))
    D2 = np.zeros((S.m, S.n))
    D1[rows, to_np(S.col_idx)] = v1
    D2[rows, to_np(S.col_idx)] = v2
    assert np.array_equal(D1, ex["A1"]) and np.array_equal(D2, ex["A2"])
    pp = to_np(S.p).reshape(-1, 2)
    assert np.array_equal(pp[:, 0], ex["p1"]) and np.array_equal(pp[:, 1], ex["p2"])


@pytest.mark.parametrize("seed,M,N,density", [(1, 18, 22, 0.3), (2, 130, 98, 0.1),
                                              (3, 1002, 514, 0.02), (4, 64, 4, 0.9)])
def test_fold_random_symmetric_systems_bit_exact(seed, M, N, density):
    banner(f"fold random seed={seed} M={M} N={N}")
    pr = random_problem(seed, M, N, density)
    Ad, pd, S = _fold(pr.A, pr.p)
    _check_against_oracle(pr.A, pr.p, S)


@pytest.mark.parametrize("cfg", [1, 2])
def test_fold_full_size_configs_bit_exact(cfg):
    banner(f"fold cfg{cfg}")
    pr = problem(cfg)
    Ad, pd, S = _fold(pr.A, pr.p)
    _check_against_oracle(pr.A, pr.p, S)


@pytest.mark.parametrize("wdtype", ["bf16", "f16"])
def test_fold_16bit_storage_is_rne_of_the_fp32_fold(wdtype):
    banner(f"fold 16-bit {wdtype}")
    pr = problem(1)
    Ad, pd, S = _fold(pr.A, pr.p, wdtype)
    _check_against_oracle(pr.A, pr.p, S, wdtype)


def test_fold_is_deterministic():
    banner("fold determinism")
    pr = random_problem(5, 300, 200, 0.05)
    _, _, S1 = _fold(pr.A, pr.p)
    _, _, S2 = _fold(pr.A, pr.p)
    for a, b in [(S1.val, S2.val), (S1.val_t, S2.val_t), (S1.inv_row, S2.inv_row),
                 (S1.inv_col, S2.inv_col)]:
        assert np.array_equal(to_np(a).view(np.uint32), to_np(b).view(np.uint32))


def _expect_error(A_host, p, code):
    import torch
    Ad = native.to_device(A_host, "cuda")
    pd = torch.from_numpy(p).cuda()
    with pytest.raises(native.SSError) as e:
        native.fold_size(Ad, pd)
    assert e.value.code == code, str(e.value)


def test_fold_size_rejects_bad_inputs():
    from gpu_util import host_matrix
    banner("fold error paths")
    pr = random_problem(6, 40, 30, 0.2)
    base = host_matrix(pr.A)
    # eq. (2) violated by one weight
    h = host_matrix(pr.A)
    h.val = h.val.copy()
    h.val[3] = np.nextafter(h.val[3], np.float32(10))
    _expect_error(h, pr.p, -3)
    # CSC copy symmetric but holding other values than the CSR copy
    h = host_matrix(pr.A)
    h.val_t = h.val_t.copy()
    N = h.N
    j = int(np.argmax(np.diff(h.col_ptr) > 0))
    q = h.col_ptr[j]
    jm = N - 1 - j
    qm = h.col_ptr[jm + 1] - 1 - (q - h.col_ptr[j])
    h.val_t[q] *= 2
    h.val_t[qm] *= 2
    _expect_error(h, pr.p, -4)
    # CSC copy breaking eq. (2)
    h = host_matrix(pr.A)
    h.val_t = h.val_t.copy()
    h.val_t[q] *= 2
    _expect_error(h, pr.p, -3)
    # NaN in p
    p = pr.p.copy()
    p[7] = np.nan
    _expect_error(base, p, -5)
    # unsorted row
    h = host_matrix(pr.A)
    h.col_idx = h.col_idx.copy()
    s = h.row_ptr[1]
    if h.row_ptr[2] - s >= 2:
        h.col_idx[s], h.col_idx[s + 1] = h.col_idx[s + 1], h.col_idx[s]
        _expect_error(h, pr.p, -4)
    # offsets past nnz
    h = host_matrix(pr.A)
    h.row_ptr = h.row_ptr.copy()
    h.row_ptr[-1] += 5
    _expect_error(h, pr.p, -4)


def test_unsplit_sums_match_oracle():
    import torch
    banner("unsplit sums")
    pr = problem(1)
    Ad = device(pr.A)
    pd = torch.from_numpy(pr.p).cuda()
    S = native.unsplit(Ad, pd)
    W = np.asarray(pr.A.astype(np.float64).sum(axis=1)).ravel()
    V = np.asarray(pr.A.astype(np.float64).sum(axis=0)).ravel()
    assert _ulps(to_np(S.inv_row), OSp.reciprocal(W, "fp32")).max() <= 1
    assert _ulps(to_np(S.inv_col), OSp.reciprocal(V, "fp32")).max() <= 1
    assert np.array_equal(to_np(S.p), pr.p)
    Sb = native.unsplit(Ad, pd, "bf16")
    bits = to_np(Sb.val).view(np.uint16)
    assert np.array_equal(bits, OSp.storage_bits(pr.A.data, "bf16"))


def test_empty_matrix_folds_and_solves():
    import torch
    banner("empty matrix")
    A = sp.csr_matrix((8, 6), dtype=np.float32)
    p = np.arange(8, dtype=np.float32)
    Ad, pd, S = _fold(A, p)
    assert S.nnz == 0
    assert np.array_equal(to_np(S.row_ptr), np.zeros(5)) and np.array_equal(to_np(S.inv_row), np.zeros(4))
    f = [S.new_image()]
    h = [torch.zeros(6, dtype=torch.float64, device="cuda")]
    status, it = native.Solver([S], native.SartOptions(max_iter=5)).solve(f, h)
    assert it == [5] and np.all(to_np(f[0]) == 0) and np.allclose(to_np(h[0]), 1.0)
    # the interleaved form (copies, and a stored order) on a system with no entries
    S2 = native.fold(Ad, pd, row_lanes=8, col_lanes=4)
    for sys_, ch in ((S, 12), (S2, 0)):
        f = [sys_.new_image()]
        h = [torch.zeros(6, dtype=torch.float64, device="cuda")]
        status, it = native.Solver([sys_], native.SartOptions(max_iter=5, chunked=ch)).solve(f, h)
        assert it == [5] and np.all(to_np(f[0]) == 0) and np.allclose(to_np(h[0]), 1.0)


def _poison(S):
    """Fills every output array with a pattern the fold never writes."""
    for t in (S.row_ptr, S.col_ptr, S.col_idx, S.row_idx):
        t.fill_(-7)
    for t in (S.val, S.val_t):
        t.fill_(float("nan") if t.dtype.is_floating_point else 0x7fc1)
    for t in (S.p, S.inv_row, S.inv_col):
        t.fill_(float("nan"))


@pytest.mark.parametrize("wdtype,lanes", [("f32", 0), ("bf16", 0), ("f32", 8)])
def test_batch_fold_equals_single_folds_bitwise(wdtype, lanes):
    """ss_fold_batch over matrices of different sizes (cfg1, ragged random
    ones, a 2 x 2) writes exactly what one ss_fold per matrix writes, also
    in the interleaved line order."""
    import torch
    banner(f"batch fold {wdtype} lanes={lanes}")
    probs = [problem(1), random_problem(21, 1002, 514, 0.05), random_problem(22, 66, 130, 0.3),
             random_problem(23, 2, 2, 0.3), problem(1, 3)]
    As = [device(pr.A) for pr in probs]
    ps = [torch.from_numpy(np.ascontiguousarray(pr.p, dtype=np.float32)).cuda() for pr in probs]
    kw = dict(row_lanes=lanes, col_lanes=lanes // 2)
    singles = [native.fold(A, p, wdtype, **kw) for A, p in zip(As, ps)]
    batch = [native.fold(A, p, wdtype, **kw) for A, p in zip(As, ps)]
    for S in batch:
        _poison(S)
    native.FoldBatch(As, ps, batch)()
    for a, b in zip(singles, batch):
        for name in ("row_ptr", "col_idx", "val", "col_ptr", "row_idx", "val_t", "p", "inv_row", "inv_col"):
            x, y = to_np(getattr(a, name)), to_np(getattr(b, name))
            assert x.shape == y.shape and np.array_equal(x.view(np.uint8), y.view(np.uint8)), name


def test_batch_recombine_equals_single():
    import torch
    banner("batch recombine")
    g = torch.Generator().manual_seed(3)
    # more images than one launch takes (32), sizes from 1 to a few blocks
    sizes = [1, 7, 2048] + [int(v) for v in torch.randint(1, 1500, (67,), generator=g)]
    f12 = [torch.randn(n, 2, generator=g).cuda() for n in sizes]
    want = [native.recombine(f) for f in f12]
    outs = [torch.full((2 * f.shape[0],), float("nan"), device="cuda") for f in f12]
    native.RecombineBatch(f12, outs)()
    for w, o in zip(want, outs):
        assert np.array_equal(to_np(w), to_np(o))


def _interleaved_positions(ptr, L):
    """Stored position of every entry of every line, written out from the
    order documented with ss_system: blocks of 4L entries (the last one r
    long); entry e of a block (lane g = e mod L, q = r // L) sits at
    g*q + min(g, r mod L) + e // L within it."""
    pos = np.empty(int(ptr[-1]), np.int64)
    B = 4 * L
    for t in range(len(ptr) - 1):
        lo, n = int(ptr[t]), int(ptr[t + 1] - ptr[t])
        e = np.arange(n)
        b = e // B
        s_ = e - b * B
        r = np.minimum(B, n - b * B)
        q, rem, g = r // L, r % L, s_ % L
        pos[lo + e] = lo + b * B + g * q + np.minimum(g, rem) + s_ // L
    return pos


@pytest.mark.parametrize("rl,cl", [(8, 8), (16, 4), (64, 32)])
def test_fold_writes_interleaved_lines(rl, cl):
    """With row_lanes / col_lanes set, every line holds the entries of the
    ascending fold at the documented interleaved positions (bitwise), and
    the offsets, p and the sums are unchanged."""
    import torch
    banner(f"interleaved fold rl={rl} cl={cl}")
    for pr in [problem(1), random_problem(21, 1002, 514, 0.05), random_problem(23, 2, 2, 0.3)]:
        Ad = device(pr.A)
        pd = torch.from_numpy(np.ascontiguousarray(pr.p, dtype=np.float32)).cuda()
        S0 = native.fold(Ad, pd)
        S1 = native.fold(Ad, pd, row_lanes=rl, col_lanes=cl)
        for name in ("row_ptr", "col_ptr", "p", "inv_row", "inv_col"):
            assert np.array_equal(to_np(getattr(S0, name)).view(np.uint8), to_np(getattr(S1, name)).view(np.uint8))
        nnz = S0.nnz
        for ptr, idx, val, L in [("row_ptr", "col_idx", "val", rl), ("col_ptr", "row_idx", "val_t", cl)]:
            pos = _interleaved_positions(to_np(getattr(S0, ptr)), L)
            assert np.array_equal(np.sort(pos), np.arange(nnz))
            i0, i1 = to_np(getattr(S0, idx))[:nnz], to_np(getattr(S1, idx))[:nnz]
            assert np.array_equal(i1[pos], i0)
            v0 = to_np(getattr(S0, val)).reshape(-1).view(np.uint64)[:nnz]
            v1 = to_np(getattr(S1, val)).reshape(-1).view(np.uint64)[:nnz]
            assert np.array_equal(v1[pos], v0)


def test_batched_validation_equals_single_calls_and_names_the_bad_matrix():
    """ss_fold_size_batch gives each matrix the size ss_fold_size gives it,
    and a batch holding one matrix that violates eq. (2) fails with that
    error, naming that matrix."""
    import torch
    from gpu_util import host_matrix
    banner("batched validation")
    probs = [problem(1), random_problem(61, 1002, 514, 0.05), random_problem(62, 40, 30, 0.2),
             random_problem(63, 2, 2, 1.0)]
    As = [device(pr.A) for pr in probs]
    ps = [torch.from_numpy(np.ascontiguousarray(pr.p, np.float32)).cuda() for pr in probs]
    sizes = native.FoldCheckBatch(As, ps)()
    assert sizes == [native.fold_size(A, p) for A, p in zip(As, ps)]
    assert sizes == [oracle_fold32(pr.A).nnz for pr in probs]
    assert native.FoldCheckBatch(As, None)() == sizes
    h = host_matrix(probs[2].A)
    h.val = h.val.copy()
    h.val[3] = np.nextafter(h.val[3], np.float32(10))
    bad = As[:2] + [native.to_device(h, "cuda")] + As[3:]
    with pytest.raises(native.SSError) as e:
        native.FoldCheckBatch(bad, ps)()
    assert e.value.code == -3 and "matrix 2" in str(e.value)
    p_bad = [p.clone() for p in ps]
    p_bad[1][5] = float("nan")
    with pytest.raises(native.SSError) as e:
        native.FoldCheckBatch(As, p_bad)()
    assert e.value.code == -5 and "matrix 1" in str(e.value)
