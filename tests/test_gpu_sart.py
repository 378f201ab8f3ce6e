"""GPU SART (ss_sart_solve) against the FP64 oracle.

Bars: the recombined FP32 image within 1e-5 relative L2 of the FP64 oracle
after 20 iterations, the residual history within 1e-5 relative; batched
solves bitwise equal to solo solves; graph replay bitwise equal to plain
launches; resumed runs bitwise equal to one long run."""
import numpy as np
import pytest

from gpu_util import assert_res_close, banner, device, problem, random_problem, rel_l2, to_np
from oracle import sart as OS
from oracle import split as OSp
from paper_1902_10559_amd import native

pytestmark = pytest.mark.gpu


def _split_system(pr, wdtype="f32"):
    import torch
    Ad = device(pr.A)
    pd = torch.from_numpy(pr.p).cuda()
    return Ad, pd, native.fold(Ad, pd, wdtype)


def _solve(systems, iters, f=None, hist=True, **kw):
    import torch
    opts = native.SartOptions(lam=kw.pop("lam", 0.5), max_iter=iters, **kw)
    sol = native.Solver(systems, opts)
    if f is None:
        f = [S.new_image() for S in systems]
    h = [torch.full((iters + 1,), -1.0, dtype=torch.float64, device="cuda") for _ in systems] if hist else None
    status, it = sol.solve(f, h)
    return f, h, status, it


@pytest.mark.parametrize("cfg,iters", [(1, 20), (2, 20)])
def test_split_sart_matches_fp64_oracle(cfg, iters):
    banner(f"split SART cfg{cfg} {iters} iterations")
    pr = problem(cfg)
    _, _, S = _split_system(pr)
    f, h, status, it = _solve([S], iters)
    assert status == 0 and it == [iters]
    img = to_np(native.recombine(f[0]))
    f_ref, res_ref = OS.sart_full(pr.A, pr.p, 0.5, iters)
    assert rel_l2(img, f_ref) <= 1e-5
    assert_res_close(to_np(h[0]), res_ref)
    # the halves themselves against the oracle's split iteration
    Sref = OSp.fold(pr.A)
    p1, p2 = OSp.fold_p(pr.p)
    g1, g2, res_s = OS.sart_split(Sref, p1, p2, 0.5, iters)
    f12 = to_np(f[0])
    assert rel_l2(f12[:, 0], g1) <= 1e-5 and rel_l2(f12[:, 1], g2) <= 1e-5


def test_split_sart_cfg2_100_iterations_matches_oracle():
    # the single-slice workload at full size and iteration count: default
    # options, and the launch configuration bench.py times for it (the fold
    # writing the interleaved order for 32 lanes per row and 8 per column,
    # persistent grid)
    import torch
    banner("split SART cfg2 100 iterations")
    pr = problem(2)
    Ad, pd, S = _split_system(pr)
    f_ref, res_ref = OS.sart_full(pr.A, pr.p, 0.5, 100)
    S_il = native.fold(Ad, pd, row_lanes=32, col_lanes=8)
    bench_shape = dict(rows_per_wave=2, cols_per_wave=8, xcd_remap=1, unroll=8, persistent=1, chunked=12)
    for sys_, kw in ((S, {}), (S_il, bench_shape)):
        f, h, status, it = _solve([sys_], 100, **kw)
        err = rel_l2(to_np(native.recombine(f[0])), f_ref)
        banner(f"cfg2 100 iterations {kw} rel L2 {err:.3e}")
        assert err <= 1e-4
        assert_res_close(to_np(h[0]), res_ref)


def test_unsplit_sart_matches_fp64_oracle():
    import torch
    banner("unsplit SART cfg1")
    pr = problem(1)
    Ad = device(pr.A)
    pd = torch.from_numpy(pr.p).cuda()
    U = native.unsplit(Ad, pd)
    f, h, status, it = _solve([U], 20)
    f_ref, res_ref = OS.sart_full(pr.A, pr.p, 0.5, 20)
    assert rel_l2(to_np(f[0]), f_ref) <= 1e-5
    assert_res_close(to_np(h[0]), res_ref)


def test_random_ragged_systems_match_oracle():
    banner("split SART random ragged")
    for seed, M, N in [(11, 1002, 514), (12, 66, 130), (13, 2, 2)]:
        pr = random_problem(seed, M, N, 0.05 if M > 100 else 0.3)
        _, _, S = _split_system(pr)
        f, h, status, it = _solve([S], 20)
        f_ref, res_ref = OS.sart_full(pr.A, pr.p, 0.5, 20)
        if np.linalg.norm(f_ref) > 0:
            assert rel_l2(to_np(native.recombine(f[0])), f_ref) <= 1e-5
        assert_res_close(to_np(h[0]), res_ref)


def test_batched_solve_equals_solo_solves_bitwise():
    # same launch shape on both sides: the summation order is then identical
    banner("batched vs solo")
    probs = [problem(1), random_problem(21, 1002, 514, 0.05), random_problem(22, 130, 98, 0.1)]
    systems = [_split_system(pr)[2] for pr in probs]
    shape = dict(rows_per_wave=2, cols_per_wave=4)
    fb, hb, _, itb = _solve(systems, 15, **shape)
    for k, S in enumerate(systems):
        fs, hs, _, its = _solve([S], 15, **shape)
        assert np.array_equal(to_np(fb[k]).view(np.uint32), to_np(fs[0]).view(np.uint32))
        assert np.array_equal(to_np(hb[k]), to_np(hs[0]))


def test_graph_replay_and_plain_launches_agree_bitwise_and_runs_repeat():
    banner("graph vs plain, determinism")
    pr = problem(1)
    _, _, S = _split_system(pr)
    a, ha, _, _ = _solve([S], 25, use_graph=True)
    b, hb, _, _ = _solve([S], 25, use_graph=False)
    c, hc, _, _ = _solve([S], 25, use_graph=True)
    assert np.array_equal(to_np(a[0]).view(np.uint32), to_np(b[0]).view(np.uint32))
    assert np.array_equal(to_np(a[0]).view(np.uint32), to_np(c[0]).view(np.uint32))
    assert np.array_equal(to_np(ha[0]), to_np(hb[0]))


def test_resume_from_a_warm_start_equals_one_long_run():
    banner("warm-start resume")
    pr = problem(1)
    _, _, S = _split_system(pr)
    a, _, _, _ = _solve([S], 20)
    b, _, _, _ = _solve([S], 10)
    b, _, _, _ = _solve([S], 10, f=b)
    assert np.array_equal(to_np(a[0]).view(np.uint32), to_np(b[0]).view(np.uint32))


@pytest.mark.parametrize("kstar", [38, 37])
def test_early_exit_at_tolerance(kstar):
    # an odd stop index leaves f^k in the workspace buffer: checks the copy back
    banner(f"early exit k*={kstar}")
    pr = problem(1)
    _, _, S = _split_system(pr)
    f_ref, res_ref = OS.sart_full(pr.A, pr.p, 0.5, 60)
    tol = float(np.sqrt(res_ref[kstar - 1] * res_ref[kstar]))
    f, h, status, it = _solve([S], 60, tol=tol, check_every=7)
    assert status == 0 and it == [kstar]
    hist = to_np(h[0])
    assert hist[kstar] <= tol < hist[kstar - 1]
    assert np.all(hist[kstar + 1:] == -1.0)       # nothing written after the stop
    fr, _ = OS.sart_full(pr.A, pr.p, 0.5, kstar)
    assert rel_l2(to_np(native.recombine(f[0])), fr) <= 1e-5
    # unreachable tolerance: warning status, capped count
    f, h, status, it = _solve([S], 12, tol=1e-9, check_every=5)
    assert status == 1 and it == [12]


SHAPES = [(1, 1, 0, 4, 0, 0), (2, 4, 1, 8, 0, 3), (4, 8, 0, 4, 1, 1), (8, 16, 1, 8, 1, 2),
          (1, 2, 1, 8, 0, 3), (8, 1, 0, 4, 1, 3), (8, 8, 1, 8, 0, 12), (1, 16, 0, 4, 1, 6),
          (4, 1, 1, 8, 1, 9), (2, 2, 0, 4, 0, 15)]


@pytest.mark.parametrize("rpw,cpw,xcd,u,pers,ch", SHAPES)
def test_launch_shapes_agree_with_oracle(rpw, cpw, xcd, u, pers, ch):
    """Every launch shape, unroll depth, grid mode and stream form (entry-wise,
    chunked or interleaved, per kernel) on cfg1 and on ragged random systems (lines that
    start mid-chunk, empty lines, a 2 x 2 system)."""
    banner(f"launch shape rpw={rpw} cpw={cpw} xcd={xcd} u={u} pers={pers} chunked={ch}")
    shape = dict(rows_per_wave=rpw, cols_per_wave=cpw, xcd_remap=xcd, unroll=u, persistent=pers, chunked=ch)
    pr = problem(1)
    _, _, S = _split_system(pr)
    f, h, _, _ = _solve([S], 20, **shape)
    f_ref, res_ref = OS.sart_full(pr.A, pr.p, 0.5, 20)
    assert rel_l2(to_np(native.recombine(f[0])), f_ref) <= 1e-5
    assert_res_close(to_np(h[0]), res_ref)
    for seed, M, N in [(11, 1002, 514), (13, 2, 2)]:
        pr = random_problem(seed, M, N, 0.05 if M > 100 else 0.3)
        _, _, S = _split_system(pr)
        f, h, _, _ = _solve([S], 20, **shape)
        f_ref, res_ref = OS.sart_full(pr.A, pr.p, 0.5, 20)
        if np.linalg.norm(f_ref) > 0:
            assert rel_l2(to_np(native.recombine(f[0])), f_ref) <= 1e-5
        assert_res_close(to_np(h[0]), res_ref)


def test_stream_forms_agree():
    """Entry-wise and chunked streams visit the same entries in a different
    per-lane order: the images agree to FP32 rounding."""
    banner("stream forms")
    pr = problem(1)
    _, _, S = _split_system(pr)
    f0, _, _, _ = _solve([S], 20, chunked=0)
    f3, _, _, _ = _solve([S], 20, chunked=3)
    a, b = to_np(f0[0]), to_np(f3[0])
    assert rel_l2(b, a) <= 1e-6


@pytest.mark.parametrize("rpw,cpw,u", [(8, 8, 8), (1, 16, 4), (4, 2, 8)])
def test_interleaved_streams_are_bitwise_entrywise(rpw, cpw, u):
    """The interleaved copy gives every lane the entries g, g + L, g + 2L, ...
    of its line in that order, as the entry-wise form does: images and
    residual histories are bitwise equal, on the folded pair (FP32 and BF16
    values) and on the unsplit A, ragged random systems included."""
    banner(f"interleaved vs entry-wise rpw={rpw} cpw={cpw} u={u}")
    shape = dict(rows_per_wave=rpw, cols_per_wave=cpw, unroll=u)
    pr = problem(1)
    Ad, pd, S = _split_system(pr)
    cases = [S, native.unsplit(Ad, pd), _split_system(pr, "bf16")[2],
             _split_system(random_problem(11, 1002, 514, 0.05))[2]]
    for sys_ in cases:
        f0, h0, _, _ = _solve([sys_], 20, chunked=0, **shape)
        f1, h1, _, _ = _solve([sys_], 20, chunked=12, **shape)
        assert np.array_equal(to_np(f0[0]).view(np.uint32), to_np(f1[0]).view(np.uint32))
        assert np.array_equal(to_np(h0[0]), to_np(h1[0]))


@pytest.mark.parametrize("rl,cl,u", [(8, 8, 8), (64, 4, 4), (16, 32, 8)])
def test_stored_interleaved_lines_solve_bitwise_as_entrywise(rl, cl, u):
    """A pair folded straight into the interleaved order is read in place
    (no copies) and gives the entry-wise results bitwise, with the launch
    shape its line order fixes; the autotuner keeps that shape."""
    import torch
    banner(f"stored interleaved lines rl={rl} cl={cl} u={u}")
    shape = dict(rows_per_wave=64 // rl, cols_per_wave=64 // cl, unroll=u)
    for pr in [problem(1), random_problem(11, 1002, 514, 0.05)]:
        Ad = device(pr.A)
        pd = torch.from_numpy(np.ascontiguousarray(pr.p, dtype=np.float32)).cuda()
        S0 = native.fold(Ad, pd)
        S1 = native.fold(Ad, pd, row_lanes=rl, col_lanes=cl)
        f0, h0, _, _ = _solve([S0], 20, chunked=0, **shape)
        f1, h1, _, _ = _solve([S1], 20, chunked=0, **shape)
        assert np.array_equal(to_np(f0[0]).view(np.uint32), to_np(f1[0]).view(np.uint32))
        assert np.array_equal(to_np(h0[0]), to_np(h1[0]))
    sol = native.Solver([S1], native.SartOptions(lam=0.5, max_iter=20))
    o = sol.autotune([S1.new_image()])
    assert o.rows_per_wave == 64 // rl and o.cols_per_wave == 64 // cl


def test_interleaved_form_with_nonnegativity_and_early_exit():
    """The projection onto f >= 0 and the stop at a tolerance behave as in
    the entry-wise form: same stop index, bitwise equal images and
    histories."""
    banner("interleaved: nonneg + early exit")
    pr = problem(1)
    _, _, S = _split_system(pr)
    shape = dict(rows_per_wave=4, cols_per_wave=8, unroll=4)
    f0, h0, s0, it0 = _solve([S], 60, chunked=0, nonneg=1, tol=0.08, check_every=7, **shape)
    f1, h1, s1, it1 = _solve([S], 60, chunked=12, nonneg=1, tol=0.08, check_every=7, **shape)
    assert s0 == s1 == 0 and it0 == it1 and it0[0] < 60
    assert np.array_equal(to_np(f0[0]).view(np.uint32), to_np(f1[0]).view(np.uint32))
    assert np.array_equal(to_np(h0[0]), to_np(h1[0]))
    assert to_np(native.recombine(f1[0])).min() >= 0.0


def test_interleaved_form_rejects_single_16bit_values():
    banner("interleaved form: 16-bit unsplit rejected")
    pr = problem(1)
    Ad, pd, _ = _split_system(pr)
    U16 = native.unsplit(Ad, pd, "bf16")
    with pytest.raises(native.SSError) as e:
        _solve([U16], 2, chunked=4)
    assert e.value.code == -1


def test_misaligned_stream_arrays_are_rejected():
    import torch
    banner("alignment check")
    pr = problem(1)
    _, _, S = _split_system(pr)
    buf = torch.empty(S.col_idx.numel() + 8, dtype=torch.int32, device="cuda")
    buf[1:1 + S.col_idx.numel()].copy_(S.col_idx)
    import dataclasses
    bad = dataclasses.replace(S, col_idx=buf[1:1 + S.col_idx.numel()])
    with pytest.raises(native.SSError) as e:
        _solve([bad], 2)
    assert e.value.code == -1 and "aligned" in str(e.value)


def test_autotune_and_kernel_timing_run():
    banner("autotune")
    pr = problem(1)
    _, _, S = _split_system(pr)
    sol = native.Solver([S], native.SartOptions(max_iter=20))
    scratch = [S.new_image()]
    opts = sol.autotune(scratch)
    assert opts.rows_per_wave in (1, 2, 4, 8) and opts.cols_per_wave in (1, 2, 4, 8, 16)
    fp, bp = sol.time_kernels(scratch, reps=5)
    assert fp > 0 and bp > 0
    f = [S.new_image()]
    sol.solve(f)
    f_ref, _ = OS.sart_full(pr.A, pr.p, 0.5, 20)
    assert rel_l2(to_np(native.recombine(f[0])), f_ref) <= 1e-5


def test_iterations_to_1e3_match_the_oracle():
    """The 64 x 64 slice reaches rel_res 1e-3: the GPU's first k with
    rel_res(f^k) <= 1e-3 matches the FP64 oracle's to within 2 iterations
    (the residual falls by ~1e-3 relative per iteration there, so FP32
    rounding can move the crossing by at most a step or two)."""
    banner("iterations to 1e-3")
    pr = problem(1)
    _, _, S = _split_system(pr)
    _, res_ref = OS.sart_full(pr.A, pr.p, 0.5, 2000)
    k_ref = int(np.argmax(res_ref <= 1e-3))
    assert res_ref[k_ref] <= 1e-3 and k_ref > 1000
    f, h, status, it = _solve([S], 5000, tol=1e-3, check_every=50)
    assert status == 0 and abs(it[0] - k_ref) <= 2


@pytest.mark.parametrize("cfg", [1, 2])
def test_nonnegative_sart_matches_the_oracle(cfg):
    """The fused projection onto f >= 0 (the pair map of eq. (5) on the
    split, a clamp on the unsplit A) against the clamped FP64 oracle."""
    banner(f"nonneg SART cfg{cfg}")
    pr = problem(cfg)
    Ad, pd, S = _split_system(pr)
    f_ref, res_ref = OS.sart_full(pr.A, pr.p, 0.5, 20, nonneg=True)
    f_free, _ = OS.sart_full(pr.A, pr.p, 0.5, 20)
    assert f_free.min() < 0.0                      # the constraint binds
    f, h, _, _ = _solve([S], 20, nonneg=True)
    img = to_np(native.recombine(f[0]))
    assert img.min() >= 0.0 and rel_l2(img, f_ref) <= 1e-5
    assert_res_close(to_np(h[0]), res_ref)
    U = native.unsplit(Ad, pd)
    fu, hu, _, _ = _solve([U], 20, nonneg=True)
    assert rel_l2(to_np(fu[0]), f_ref) <= 1e-5
    assert_res_close(to_np(hu[0]), res_ref)
