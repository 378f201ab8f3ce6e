"""The batched workload at full size: 256 slices of 1024 x nz voxels (nz in
{32, 48, ..., 128}), 24 sources, 2048 bins, each slice with its own system,
both halves of every slice solved in the same launches (graph replay).

Parity on sampled outputs: two sampled slices (the deepest and the
shallowest) carry projections made by the oracle, and their recombined images
from the full batched solve are checked against the FP64 oracle: in the
staged launch configuration bench.py times (bands of 4096 voxels, work tiles
of 2048 entries with one window per batch, back-projection tiles of 512
columns with 8 per wavefront) at the bench's 100 iterations, with BF16
weights against the oracle
on the same rounded values, and in the unstaged interleaved configuration
(the fold writing the interleaved line order for 8 lanes, 8 rows and 8
columns per wavefront, 8 entries per lane and pass, XCD-ordered blocks); a
small batch is checked bitwise against solo solves of the same slices."""
import dataclasses

import numpy as np
import pytest

from gpu_util import assert_res_close, banner, rel_l2, to_np
from oracle import geometry as G
from oracle import sart as OS
from oracle import split as OSp
from paper_1902_10559_amd import inputs, native, workloads

pytestmark = pytest.mark.gpu

ITERS = 20


def _oracle_problem(s):
    nz = int(inputs.cfg4_depths()[s])
    g = inputs.geometry_cfg4_slice(s, nz)
    A = G.to_fp32(G.system_matrix(g))
    f_true = G.image_to_snake(inputs.phantom_for(4, s, g))
    p = (A.astype(np.float64) @ f_true).astype(np.float32)
    return A, p


@pytest.fixture(scope="module")
def sampled():
    depths = inputs.cfg4_depths()
    picks = [int(np.argmax(depths)), int(np.argmin(depths))]
    return {s: _oracle_problem(s) for s in picks}


# the staged kernels in the shape bench.py times on this workload
BENCH_STAGED = dict(staged=3, band_width=4096, tile_cols=512, tile_entries=2048, cols_per_wave=8, unroll=4)


@pytest.fixture(scope="module")
def batch(sampled):
    banner("batched: building 256 slices (ascending fold)")
    sl = workloads.batched_slices(256, p_override={s: v[1] for s, v in sampled.items()}, progress=banner)
    return sl


def _solve(systems, iters, **kw):
    import torch
    sol = native.Solver(systems, native.SartOptions(lam=0.5, max_iter=iters, zero_start=True, use_graph=True, **kw))
    f = [S.new_image() for S in systems]
    hist = [torch.zeros(iters + 1, dtype=torch.float64, device="cuda") for _ in systems]
    status, it = sol.solve(f, hist)
    assert status == 0 and it == [iters] * len(systems)
    return f, hist


def test_full_batch_staged_at_bench_length_matches_oracle(batch, sampled):
    iters = 100
    banner(f"batched: staged bench configuration, {iters} iterations")
    f, hist = _solve([x.S for x in batch], iters, **BENCH_STAGED)
    for s, (A, p) in sampled.items():
        f_ref, res_ref = OS.sart_full(A, p, 0.5, iters)
        err = rel_l2(to_np(native.recombine(f[s])), f_ref)
        banner(f"slice {s} (nz={batch[s].geom.nz}) rel L2 {err:.2e} after {iters}")
        assert err <= 1e-5
        assert_res_close(to_np(hist[s]), res_ref)


def test_full_batch_bf16_staged_matches_oracle_on_rounded_values(batch, sampled):
    banner("batched: BF16 weights, staged configuration")
    low = [native.fold(x.A, x.p, "bf16", nnz_half=x.S.nnz) for x in batch]
    f, hist = _solve(low, ITERS, **BENCH_STAGED)
    for s, (A, p) in sampled.items():
        R = OSp.fold(A, "fp32")
        R = dataclasses.replace(R, v1=OSp.round_storage(R.v1, "bf16"), v2=OSp.round_storage(R.v2, "bf16"))
        p1, p2 = OSp.fold_p(p)
        g1, g2, res = OS.sart_split(R, p1, p2, 0.5, ITERS)
        err = rel_l2(to_np(native.recombine(f[s])), OSp.recombine(g1, g2))
        banner(f"slice {s} bf16 rel L2 {err:.2e} against the oracle on the rounded values")
        assert err <= 1e-5
        assert_res_close(to_np(hist[s]), res)


def test_full_batch_sampled_slices_match_oracle(sampled):
    import torch
    banner("batched: building 256 slices")
    sl = workloads.batched_slices(256, p_override={s: v[1] for s, v in sampled.items()},
                                  progress=banner)
    systems = [x.S for x in sl]
    total = sum(x.A.nnz for x in sl)
    banner(f"batched: nnz total {total}")
    for S in systems:
        S.row_lanes = S.col_lanes = 8
    native.FoldBatch([x.A for x in sl], [x.p for x in sl], systems)()
    opts = native.SartOptions(max_iter=ITERS, zero_start=True, rows_per_wave=8, cols_per_wave=8, xcd_remap=1,
                              unroll=8, chunked=12)
    sol = native.Solver(systems, opts)
    f = [S.new_image() for S in systems]
    hist = [torch.zeros(ITERS + 1, dtype=torch.float64, device="cuda") for _ in systems]
    status, iters = sol.solve(f, hist)
    assert status == 0 and iters == [ITERS] * len(systems)
    for s, (A, p) in sampled.items():
        # the library's matrix for this slice equals the oracle's
        assert np.array_equal(to_np(sl[s].A.col_idx), A.indices)
        assert np.array_equal(to_np(sl[s].A.val).view(np.uint32), A.data.view(np.uint32))
        f_ref, res_ref = OS.sart_full(A, p, 0.5, ITERS)
        err = rel_l2(to_np(native.recombine(f[s])), f_ref)
        banner(f"slice {s} (nz={sl[s].geom.nz}) rel L2 {err:.2e}")
        assert err <= 1e-5
        assert_res_close(to_np(hist[s]), res_ref)
    # every slice's residual falls (noise-free data)
    for h in hist:
        hh = to_np(h)
        assert hh[0] == pytest.approx(1.0) and hh[-1] < hh[0]


def test_small_batch_equals_solo_solves_bitwise():
    banner("batched: 6 slices vs solo")
    sl = workloads.batched_slices(6)
    systems = [x.S for x in sl]
    shape = dict(rows_per_wave=4, cols_per_wave=8, xcd_remap=1)
    fb = [S.new_image() for S in systems]
    native.Solver(systems, native.SartOptions(max_iter=7, **shape)).solve(fb)
    for k, S in enumerate(systems):
        fs = [S.new_image()]
        native.Solver([S], native.SartOptions(max_iter=7, **shape)).solve(fs)
        assert np.array_equal(to_np(fb[k]).view(np.uint32), to_np(fs[0]).view(np.uint32))


def test_batch_in_stored_interleaved_order_equals_ascending_batch():
    """The batch folded straight into the interleaved line order (one
    ss_fold_batch) and solved in place gives, bitwise, what the ascending
    batch gives with the entry-wise form at the same shape."""
    import torch
    banner("batched: stored interleaved order vs ascending")
    sl = workloads.batched_slices(6)
    systems = [x.S for x in sl]
    shape = dict(rows_per_wave=8, cols_per_wave=16, xcd_remap=1, unroll=8)
    f0 = [S.new_image() for S in systems]
    h0 = [torch.full((8,), -1.0, dtype=torch.float64, device="cuda") for _ in systems]
    native.Solver(systems, native.SartOptions(max_iter=7, chunked=0, **shape)).solve(f0, h0)
    for S in systems:
        S.row_lanes, S.col_lanes = 8, 4
    native.FoldBatch([x.A for x in sl], [x.p for x in sl], systems)()
    f1 = [S.new_image() for S in systems]
    h1 = [torch.full((8,), -1.0, dtype=torch.float64, device="cuda") for _ in systems]
    native.Solver(systems, native.SartOptions(max_iter=7, **shape)).solve(f1, h1)
    for a, b, ha, hb in zip(f0, f1, h0, h1):
        assert np.array_equal(to_np(a).view(np.uint32), to_np(b).view(np.uint32))
        assert np.array_equal(to_np(ha), to_np(hb))
    for S in systems:
        S.row_lanes = S.col_lanes = 0
