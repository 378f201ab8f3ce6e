"""The polar grid of the closing example (Fig. 4, renumbered so that eq. (2)
holds): the fold, split SART and the direct path run on it unchanged.

Inputs: the oracle's polar matrix (FP32) and noise-free projections of a
seeded phantom.  Bars as for the Cartesian scans: the fold bit-exact; split
SART within 1e-5 (image) of the FP64 oracle after 20 iterations, residual
history within 1e-5 relative + 1e-6; split and unsplit GPU images within
1e-5 of each other (Theorem 1); ordered subsets over the mirror-paired
views within 1e-5 of the oracle after 10 passes; the direct path within 1e-7 of the oracle's
Cholesky solution on the 72-voxel system, which has full column rank."""
import functools

import numpy as np
import pytest

from gpu_util import assert_res_close, banner, device, rel_l2, to_np
from oracle import geometry as G
from oracle import normal as ON
from oracle import polar as P
from oracle import sart as OS
from oracle import split as OSp
from paper_1902_10559_amd import inputs, native
from test_gpu_fold import _check_against_oracle

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def _problem(which):
    cfg, g = (7, inputs.geometry_tgs()) if which == "tgs" else (8, inputs.geometry_polar_large())
    A = G.to_fp32(P.system_matrix(g))
    f_true = inputs.polar_phantom(cfg, 0, g)
    p = (A.astype(np.float64) @ f_true).astype(np.float32)
    return g, A, f_true, p


def _systems(A, p):
    import torch
    Ad = device(A)
    pd = torch.from_numpy(np.ascontiguousarray(p)).cuda()
    return Ad, pd, native.fold(Ad, pd), native.unsplit(Ad, pd)


def _sart(S, iters):
    import torch
    sol = native.Solver([S], native.SartOptions(lam=0.5, max_iter=iters))
    f = [S.new_image()]
    h = [torch.full((iters + 1,), -1.0, dtype=torch.float64, device="cuda")]
    status, it = sol.solve(f, h)
    assert status == 0 and it == [iters]
    return f[0], to_np(h[0])


@pytest.mark.parametrize("which", ["tgs", "large"])
def test_polar_fold_is_bit_exact(which):
    banner(f"polar fold {which}")
    g, A, _, p = _problem(which)
    _, _, S, _ = _systems(A, p)
    _check_against_oracle(A, p, S)


@pytest.mark.parametrize("which", ["tgs", "large"])
def test_polar_split_sart_matches_oracle_and_unsplit(which):
    banner(f"polar SART {which}")
    g, A, _, p = _problem(which)
    _, _, S, U = _systems(A, p)
    f12, h = _sart(S, 20)
    img = to_np(native.recombine(f12))
    f_ref, res_ref = OS.sart_full(A, p, 0.5, 20)
    assert rel_l2(img, f_ref) <= 1e-5
    assert_res_close(h, res_ref)
    fu, hu = _sart(U, 20)
    assert rel_l2(img, to_np(fu)) <= 1e-5


def test_polar_direct_path_matches_oracle():
    banner("polar direct path tgs")
    g, A, f_true, p = _problem("tgs")
    _, _, S, U = _systems(A, p)
    fs = to_np(native.normal_solve(S))
    S32 = OSp.fold(A, "fp32")
    p1, p2 = OSp.fold_p(p.astype(np.float64), "fp32")
    want, _, _ = ON.normal_solve_split(S32, p1.astype(np.float64), p2.astype(np.float64))
    assert rel_l2(fs, want) <= 1e-7
    fu = to_np(native.normal_solve(U))
    assert rel_l2(fu, ON.normal_solve(A, p.astype(np.float64))) <= 1e-7
    assert rel_l2(fs, f_true) <= 1e-4 and rel_l2(fu, f_true) <= 1e-4


def test_polar_ordered_subsets_match_oracle():
    """Ordered subsets on the polar scan: the views k and K-1-k are mirror
    images (phi -> -phi with the offsets reversed), so each pair folds onto a
    block of B rows, as for the point-source scans."""
    import torch
    from oracle import ossart as OO
    banner("polar ordered subsets tgs")
    g, A, _, p = _problem("tgs")
    _, _, S, _ = _systems(A, p)
    nsub = g.K // 2
    B = native.Subsets(S, nsub)
    sol = native.OsSolver([S], [B], native.SartOptions(lam=0.5, max_iter=10))
    f = [S.new_image()]
    h = [torch.full((11,), -1.0, dtype=torch.float64, device="cuda")]
    st, it = sol.solve(f, h)
    assert it == [10]
    Sp = OSp.fold(A.astype(np.float64))
    p1, p2 = OSp.fold_p(p.astype(np.float64))
    _, folded = OO.mirror_paired_views(g.K, g.B)
    f1, f2, res = OO.os_sart_split(Sp, p1, p2, 0.5, 10, folded)
    assert rel_l2(to_np(native.recombine(f[0])), OSp.recombine(f1, f2)) <= 1e-5
    assert_res_close(to_np(h[0]), res)
