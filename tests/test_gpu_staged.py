"""Staged SART kernels (ss_sart_opts.staged) against the FP64 oracle.

Bars as for the unstaged kernels: the recombined FP32 image within 1e-5
relative L2 of the FP64 oracle after 20 iterations and the residual history
within 1e-5 relative (+1e-6 absolute, the FP32 floor); batched solves bitwise
equal to solo solves with the same options; graph replay, plain launches and
repeated solves bitwise equal.  The staged forms sum in another order than
the unstaged kernels, so they are compared with the oracle, not bitwise
with the unstaged results.  Cases cover several bands and tiles, ragged
last bands and tiles, empty rows and columns, 16-bit weights, the unsplit
system, tiles whose rows overflow the LDS budget (global fallback), early
exit and the non-negativity projection."""
import numpy as np
import pytest

from gpu_util import assert_res_close, banner, device, problem, random_problem, rel_l2, to_np
from oracle import sart as OS
from oracle import split as OSp
from paper_1902_10559_amd import native

pytestmark = pytest.mark.gpu

BOTH = dict(staged=3, band_width=1024, tile_cols=64)


def _fold(pr, wdtype="f32"):
    import torch
    Ad = device(pr.A)
    pd = torch.from_numpy(np.ascontiguousarray(pr.p, np.float32)).cuda()
    return Ad, pd, native.fold(Ad, pd, wdtype)


def _solve(systems, iters, f=None, **kw):
    import torch
    opts = native.SartOptions(lam=kw.pop("lam", 0.5), max_iter=iters, **kw)
    sol = native.Solver(systems, opts)
    if f is None:
        f = [S.new_image() for S in systems]
    h = [torch.full((iters + 1,), -1.0, dtype=torch.float64, device="cuda") for _ in systems]
    status, it = sol.solve(f, h)
    return f, h, status, it


def _check_split(pr, S, f, h, iters, tol=1e-5):
    img = to_np(native.recombine(f))
    f_ref, res_ref = OS.sart_full(pr.A, pr.p, 0.5, iters)
    err = rel_l2(img, f_ref) if np.linalg.norm(f_ref) > 0 else float(np.linalg.norm(img))
    assert err <= tol, err
    assert_res_close(to_np(h), res_ref)
    return err


@pytest.mark.parametrize("staged", [1, 2, 3])
@pytest.mark.parametrize("rpw,cpw,unroll", [(4, 8, 4), (2, 4, 8), (8, 16, 8)])
def test_staged_split_sart_cfg1_matches_oracle(staged, rpw, cpw, unroll):
    # cfg1: n = 2048 columns -> two bands of 1024, 32 tiles of 64 columns
    banner(f"staged={staged} cfg1 rpw={rpw} cpw={cpw} unroll={unroll}")
    pr = problem(1)
    _, _, S = _fold(pr)
    f, h, status, it = _solve([S], 20, rows_per_wave=rpw, cols_per_wave=cpw, unroll=unroll, **dict(BOTH, staged=staged))
    assert status == 0 and it == [20]
    _check_split(pr, S, f[0], h[0], 20)


@pytest.mark.parametrize("band,tile,entries,unroll", [(1024, 64, 1024, 4), (4096, 1024, 65536, 8),
                                                    (2048, 256, 4096, 4), (4096, 512, 16384, 8)])
def test_staged_split_sart_cfg2_matches_oracle(band, tile, entries, unroll):
    # cfg2: 32768 columns; several work tiles per band, ragged last tiles
    banner(f"staged cfg2 band={band} tile={tile} entries={entries} unroll={unroll}")
    pr = problem(2)
    _, _, S = _fold(pr)
    f, h, status, it = _solve([S], 20, staged=3, band_width=band, tile_cols=tile, tile_entries=entries,
                              unroll=unroll)
    _check_split(pr, S, f[0], h[0], 20)


@pytest.mark.parametrize("entries", [1024, 4096])
def test_staged_segments_spanning_many_windows_match_oracle(entries):
    # dense rows: a row's segment in a band of 1024 columns holds up to 1024
    # entries (256 chunks, four windows of 64 chunks), so segments run across
    # windows and tiles hold a few segments each
    banner(f"staged long segments entries={entries}")
    pr = random_problem(61, 120, 4096, 0.9)
    _, _, S = _fold(pr)
    f, h, status, it = _solve([S], 20, staged=1, band_width=1024, tile_entries=entries)
    _check_split(pr, S, f[0], h[0], 20)


def test_staged_random_ragged_systems_match_oracle():
    # empty rows and columns, a last band of a few columns, tiny systems
    for seed, M, N, d in [(31, 800, 2100, 0.01), (32, 1002, 514, 0.05), (33, 66, 130, 0.3), (34, 2, 2, 1.0)]:
        banner(f"staged random M={M} N={N}")
        pr = random_problem(seed, M, N, d)
        _, _, S = _fold(pr)
        f, h, status, it = _solve([S], 20, **BOTH)
        _check_split(pr, S, f[0], h[0], 20)


def test_staged_tiles_that_overflow_fall_back_to_global_gathers():
    # 20000 x 600 at density 0.2: a tile of 256 columns touches more than
    # 4096 distinct rows, so its back projection gathers from global memory
    banner("staged overflow fallback")
    pr = random_problem(41, 20000, 600, 0.2)
    _, _, S = _fold(pr)
    f, h, status, it = _solve([S], 20, staged=3, band_width=1024, tile_cols=256)
    _check_split(pr, S, f[0], h[0], 20)


@pytest.mark.parametrize("wdtype", ["bf16", "f16"])
def test_staged_16bit_weights_match_oracle_on_rounded_values(wdtype):
    import dataclasses
    banner(f"staged {wdtype}")
    pr = problem(3)
    _, _, S = _fold(pr, wdtype)
    f, h, status, it = _solve([S], 20, **BOTH)
    # the oracle on the same rounded values (and the FP32-derived sums)
    R = OSp.fold(pr.A, "fp32")
    R = dataclasses.replace(R, v1=OSp.round_storage(R.v1, wdtype), v2=OSp.round_storage(R.v2, wdtype))
    p1, p2 = OSp.fold_p(pr.p)
    g1, g2, res = OS.sart_split(R, p1, p2, 0.5, 20)
    assert rel_l2(to_np(native.recombine(f[0])), OSp.recombine(g1, g2)) <= 1e-5
    assert_res_close(to_np(h[0]), res)


def test_staged_unsplit_matches_oracle():
    import torch
    banner("staged unsplit")
    pr = problem(1)
    Ad = device(pr.A)
    pd = torch.from_numpy(pr.p).cuda()
    U = native.unsplit(Ad, pd)
    f, h, status, it = _solve([U], 20, staged=3, band_width=1024, tile_cols=128)
    f_ref, res_ref = OS.sart_full(pr.A, pr.p, 0.5, 20)
    assert rel_l2(to_np(f[0]), f_ref) <= 1e-5
    assert_res_close(to_np(h[0]), res_ref)


def test_staged_batched_equals_solo_bitwise_and_runs_repeat():
    banner("staged batched vs solo")
    probs = [problem(1), random_problem(51, 1002, 514, 0.05), random_problem(52, 800, 2100, 0.01),
             random_problem(53, 130, 98, 0.1)]
    systems = [_fold(pr)[2] for pr in probs]
    fb, hb, _, _ = _solve(systems, 15, **BOTH)
    for k, S in enumerate(systems):
        fs, hs, _, _ = _solve([S], 15, **BOTH)
        assert np.array_equal(to_np(fb[k]).view(np.uint32), to_np(fs[0]).view(np.uint32))
        assert np.array_equal(to_np(hb[k]), to_np(hs[0]))
    for k, pr in enumerate(probs):
        _check_split(pr, systems[k], fb[k], hb[k], 15)


def test_staged_graph_and_plain_launches_agree_bitwise():
    banner("staged graph vs plain")
    pr = problem(1)
    _, _, S = _fold(pr)
    a, ha, _, _ = _solve([S], 25, use_graph=True, **BOTH)
    b, hb, _, _ = _solve([S], 25, use_graph=False, **BOTH)
    c, hc, _, _ = _solve([S], 25, use_graph=True, **BOTH)
    assert np.array_equal(to_np(a[0]).view(np.uint32), to_np(b[0]).view(np.uint32))
    assert np.array_equal(to_np(a[0]).view(np.uint32), to_np(c[0]).view(np.uint32))
    assert np.array_equal(to_np(ha[0]), to_np(hb[0]))


@pytest.mark.parametrize("kstar", [38, 37])
def test_staged_early_exit_at_tolerance(kstar):
    banner(f"staged early exit k*={kstar}")
    pr = problem(1)
    _, _, S = _fold(pr)
    _, res_ref = OS.sart_full(pr.A, pr.p, 0.5, 60)
    tol = 0.5 * (res_ref[kstar] + res_ref[kstar - 1])
    f, h, status, it = _solve([S], 60, tol=tol, check_every=4, **BOTH)
    assert it == [kstar]
    img = to_np(native.recombine(f[0]))
    f_ref, _ = OS.sart_full(pr.A, pr.p, 0.5, kstar)
    assert rel_l2(img, f_ref) <= 1e-5
    assert_res_close(to_np(h[0])[: kstar + 1], res_ref[: kstar + 1])


def test_staged_nonneg_matches_clamped_oracle():
    banner("staged nonneg")
    pr = problem(1)
    _, _, S = _fold(pr)
    f, h, status, it = _solve([S], 20, nonneg=True, **BOTH)
    f_ref, res_ref = OS.sart_full(pr.A, pr.p, 0.5, 20, nonneg=True)
    img = to_np(native.recombine(f[0]))
    assert img.min() >= 0.0
    assert rel_l2(img, f_ref) <= 1e-5
    assert_res_close(to_np(h[0]), res_ref)


def test_staged_phase_timer_reports_three_launches():
    banner("staged phase timer")
    pr = problem(2)
    _, _, S = _fold(pr)
    sol = native.Solver([S], native.SartOptions(lam=0.5, max_iter=10, staged=3, band_width=4096, tile_cols=1024))
    ms = sol.time_phases([S.new_image()], reps=5)
    assert all(t > 0 for t in ms), ms
    sol0 = native.Solver([S], native.SartOptions(lam=0.5, max_iter=10))
    ms0 = sol0.time_phases([S.new_image()], reps=5)
    assert ms0[0] > 0 and ms0[1] == 0 and ms0[2] > 0
