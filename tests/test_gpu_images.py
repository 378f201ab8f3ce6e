"""GPU recombination (Theorem 1, eq. (5)), its inverse and the forward
projection against the oracle."""
import numpy as np
import pytest

from gpu_util import banner, device, problem, to_np
from oracle import split as OSp
from paper_1902_10559_amd import native

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1, 3, 255, 256, 257, 32768])
def test_recombine_and_image_fold_bit_exact(n):
    import torch
    banner(f"recombine n={n}")
    rng = np.random.default_rng(n)
    f12 = rng.standard_normal((n, 2)).astype(np.float32)
    got = to_np(native.recombine(torch.from_numpy(f12).cuda()))
    want = OSp.recombine(f12[:, 0], f12[:, 1], "fp32")
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    f = rng.standard_normal(2 * n).astype(np.float32)
    got = to_np(native.image_fold(torch.from_numpy(f).cuda()))
    w1, w2 = OSp.image_fold(f, "fp32")
    assert np.array_equal(got[:, 0].view(np.uint32), w1.view(np.uint32))
    assert np.array_equal(got[:, 1].view(np.uint32), w2.view(np.uint32))


def test_project_matches_oracle():
    import torch
    banner("project")
    pr = problem(1)
    Ad = device(pr.A)
    q = to_np(native.project(Ad, torch.from_numpy(pr.f_true.astype(np.float32)).cuda()))
    want = pr.A.astype(np.float64) @ pr.f_true.astype(np.float32).astype(np.float64)
    assert np.max(np.abs(q - want)) <= 1e-5 * np.abs(want).max()
