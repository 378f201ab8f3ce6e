"""16-bit weight storage (BF16, FP16) for the split pair and the unsplit A.

Two bars per storage type:
* arithmetic: the GPU result against the FP64 oracle run on the SAME rounded
  values (and the FP32-derived sums), which isolates FP32 accumulation:
  1e-5 relative L2 after 20 iterations;
* storage: the GPU result against the FP64 oracle on the exact FP32 weights,
  which measures what 16-bit storage costs: 1e-2 relative L2 after 100
  iterations on the 64x64 slice workload.
"""
import dataclasses

import numpy as np
import pytest

from gpu_util import assert_res_close, banner, device, problem, rel_l2, to_np
from oracle import sart as OS
from oracle import split as OSp
from paper_1902_10559_amd import native

pytestmark = pytest.mark.gpu


def _rounded_split(A, dtype):
    S = OSp.fold(A, "fp32")
    return dataclasses.replace(S, v1=OSp.round_storage(S.v1, dtype),
                               v2=OSp.round_storage(S.v2, dtype))


def _gpu_split_solve(pr, dtype, iters):
    import torch
    Ad = device(pr.A)
    pd = torch.from_numpy(pr.p).cuda()
    S = native.fold(Ad, pd, dtype)
    f = [S.new_image()]
    h = [torch.zeros(iters + 1, dtype=torch.float64, device="cuda")]
    native.Solver([S], native.SartOptions(max_iter=iters)).solve(f, h)
    return to_np(native.recombine(f[0])), to_np(h[0])


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_16bit_split_arithmetic_matches_oracle_on_the_same_values(dtype):
    banner(f"16-bit arithmetic {dtype}")
    pr = problem(3)
    img, hist = _gpu_split_solve(pr, dtype, 20)
    R = _rounded_split(pr.A, dtype)
    p1, p2 = OSp.fold_p(pr.p)
    g1, g2, res = OS.sart_split(R, p1, p2, 0.5, 20)
    assert rel_l2(img, OSp.recombine(g1, g2)) <= 1e-5
    assert_res_close(hist, res)


@pytest.mark.parametrize("dtype,bar", [("f32", 1e-4), ("bf16", 1e-2), ("f16", 1e-2)])
def test_storage_error_against_exact_oracle_after_100_iterations(dtype, bar):
    banner(f"storage error {dtype}")
    pr = problem(3)
    img, _ = _gpu_split_solve(pr, dtype, 100)
    f_ref, _ = OS.sart_full(pr.A, pr.p, 0.5, 100)
    err = rel_l2(img, f_ref)
    banner(f"{dtype}: image rel L2 vs FP64 oracle after 100 iterations = {err:.3e}")
    assert err <= bar


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_16bit_unsplit_matches_oracle_on_the_same_values(dtype):
    import scipy.sparse as sp
    import torch
    banner(f"16-bit unsplit {dtype}")
    pr = problem(3)
    Ad = device(pr.A)
    pd = torch.from_numpy(pr.p).cuda()
    U = native.unsplit(Ad, pd, dtype)
    f = [U.new_image()]
    native.Solver([U], native.SartOptions(max_iter=20)).solve(f)
    # oracle: rounded values, sums of the FP32 values
    Ar = sp.csr_matrix((OSp.round_storage(pr.A.data, dtype), pr.A.indices, pr.A.indptr),
                       shape=pr.A.shape)
    W = np.asarray(pr.A.astype(np.float64).sum(axis=1)).ravel()
    V = np.asarray(pr.A.astype(np.float64).sum(axis=0)).ravel()
    fr, _ = OS.sart_full(Ar, pr.p, 0.5, 20, sums=(W, V))
    assert rel_l2(to_np(f[0]), fr) <= 1e-5
