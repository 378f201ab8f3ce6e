"""The allocation-free fold (ss_fold_noalloc) against ss_fold.

Bar: bit-exact (the fold is one FP32 add or subtract per entry), on two
calls in a row through the C ABI, the second on a smaller matrix, so that the
scratch array the entry point keeps between calls is reused."""
import numpy as np
import pytest
import torch

from gpu_util import banner, device, problem, random_problem, to_np
from paper_1902_10559_amd import native

pytestmark = pytest.mark.gpu

FIELDS = ("row_ptr", "col_idx", "val", "col_ptr", "row_idx", "val_t", "p", "inv_row", "inv_col")


def _poisoned_like(S):
    """A system with S's sizes whose arrays hold a NaN pattern."""
    T = native.System(S.m, S.n, S.nnz, S.nvals, S.wdtype,
                      *[torch.empty_like(getattr(S, k)) for k in FIELDS], S.row_lanes, S.col_lanes)
    for k in FIELDS:
        t = getattr(T, k)
        t.view(torch.uint8).fill_(0xFF)
    return T


def _same(S, T):
    for k in FIELDS:
        a, b = to_np(getattr(S, k)), to_np(getattr(T, k))
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), k


@pytest.mark.parametrize("wdtype,lanes", [("f32", (0, 0)), ("bf16", (0, 0)), ("f32", (8, 4))])
def test_noalloc_fold_equals_fold_on_two_calls(wdtype, lanes):
    cases = [problem(1), random_problem(7, 130, 98, 0.1)]   # the second is smaller
    for k, pr in enumerate(cases):
        banner(f"ss_fold_noalloc call {k}: M={pr.A.shape[0]} N={pr.A.shape[1]} {wdtype} lanes={lanes}")
        Ad = device(pr.A)
        pd = torch.from_numpy(np.ascontiguousarray(pr.p, dtype=np.float32)).cuda()
        ref = native.fold(Ad, pd, wdtype, row_lanes=lanes[0], col_lanes=lanes[1])
        got = _poisoned_like(ref)
        native.fold_noalloc_into(Ad, pd, got)
        torch.cuda.synchronize()
        _same(ref, got)


def test_noalloc_fold_rejects_bad_arguments_before_any_work():
    banner("ss_fold_noalloc argument errors")
    pr = problem(1)
    Ad = device(pr.A)
    pd = torch.from_numpy(np.ascontiguousarray(pr.p, dtype=np.float32)).cuda()
    S = native.fold(Ad, pd)
    bad = native.System(S.m + 1, *[getattr(S, k) for k in ("n", "nnz", "nvals", "wdtype")],
                        *[getattr(S, k) for k in FIELDS])
    with pytest.raises(native.SSError) as e:
        native.fold_noalloc_into(Ad, pd, bad)
    assert e.value.code == -1
