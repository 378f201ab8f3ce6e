"""Split-SART benchmark on one MI355X.

One step is the whole hot path over one batch of input already resident in
HBM: fold A and p into the split pair (systems (3), (4) of the paper), run
100 SART iterations on both halves, recombine by Theorem 1, eq. (5).  Building
A (host Siddon) and synthesising p happen before the timed region.

Workloads:
  batched (default)  256 slices of 1024 x nz voxels, nz in {32, 48, ..., 128},
                   each with its own geometry, 24 sources, 2048 bins,
                   noise-free, 100 iterations; all slices and both halves in
                   the same launches.  Its 11 GB per iteration stream from
                   HBM: the workload the HBM roofline is taken on.
  slice            a 512 x 128 voxel slice (N = 65536), 24 sources over +-20
                   degrees, 1024-bin detector (M = 24576), 40 random ellipses,
                   1 % noise, 100 iterations, FP32 weights.  Its 32 MB per
                   iteration stay in the 256 MB Infinity Cache, so its kernels
                   are bound by latency, not by HBM.
The same step on the unsplit A is timed beside it.  Extras: ordered-subset
SART against SART to a residual of 1e-2, the direct path (normal equations by
Cholesky, Theorem 2) on Table 1's three sizes, time to a residual of 1e-3,
and the CPU oracle's rate.  ``--direct-only``, ``--polar-only``, ``--conv-only`` and
``--subsets-only`` print just that report.

Output: one JSON line on stdout (progress on stderr).  ``value`` is
original-system nonzeros processed per second: iterations x nnz(A) / time.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "split-SART nnz/s & HBM GB/s vs unsplit; time to residual 1e-3 on 1 MI355X"
PEAK_HBM_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--iters", type=int, default=100, help="SART iterations per step")
    ap.add_argument("--workload", choices=["slice", "batched"], default="batched")
    ap.add_argument("--wdtype", choices=["f32", "bf16", "f16"], default="f32",
                    help="storage type of the split pair's weights")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-subsets", action="store_true", help="skip the ordered-subset comparison")
    ap.add_argument("--no-direct", action="store_true",
                    help="skip the direct (normal-equation) path at Table 1's sizes")
    ap.add_argument("--no-polar", action="store_true",
                    help="skip the polar-grid SART comparison")
    ap.add_argument("--direct-only", action="store_true",
                    help="only the direct path's report (one JSON line), for profiling it")
    ap.add_argument("--conv-only", action="store_true",
                    help="only the learned initialiser's per-layer convolution report (one JSON line)")
    ap.add_argument("--polar-only", action="store_true",
                    help="only the polar-grid report (one JSON line), for profiling it")
    ap.add_argument("--subsets-only", action="store_true",
                    help="only the ordered-subset comparison on the workload (one JSON line)")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the timed steps (for profiler runs)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the plain vs learned-start comparison on the 256x256 workload")
    ap.add_argument("--no-ttr", action="store_true",
                    help="skip the time-to-1e-3 runs on the workload")
    ap.add_argument("--no-dtypes", action="store_true",
                    help="skip the BF16/FP16-weight step records")
    ap.add_argument("--staged", default="", metavar="BITS,BAND,TILE,ENTRIES,CPW,UNROLL",
                    help="fixed staged-kernel configuration instead of the timed choice "
                         "(BITS 0 keeps the unstaged kernels of --shape or the autotuner)")
    ap.add_argument("--shape", default="", metavar="RPW,CPW,XCD,UNROLL,PERSISTENT,CHUNKED",
                    help="fixed launch shape instead of the autotuner's choice")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of this many MiB, so that "
                         "hardware byte counters can be scaled against a known size")
    return ap.parse_args()


def bytes_per_iteration(nnz, m, n, nv, sv):
    """Algorithmic HBM bytes of one SART iteration, per kernel.

    Forward projection: per pattern entry a 4-byte index and nv values of sv
    bytes; per row the offset (8), p (4 nv), 1/W (4) and the z write (4 nv);
    the image once (4 nv n).  Back projection: per entry index and values; per
    column the offset (8), 1/V (4), the image read and the new image write
    (8 nv); z once (4 nv m)."""
    per_entry = 4 + nv * sv
    fp = nnz * per_entry + m * (8 + 4 * nv + 4 + 4 * nv) + n * 4 * nv
    bp = nnz * per_entry + n * (8 + 4 + 8 * nv) + m * 4 * nv
    return fp, bp


def source_hash():
    """Hash of the solver's device code (device.h, lines.h, staged.h and the
    kernel section of sart.hip): traffic counted for other kernel code is not
    reported."""
    csrc = os.path.join(ROOT, "paper_1902_10559_amd", "csrc")
    h = hashlib.sha256(open(os.path.join(csrc, "device.h"), "rb").read())
    h.update(open(os.path.join(csrc, "lines.h"), "rb").read())
    h.update(open(os.path.join(csrc, "staged.h"), "rb").read())
    text = open(os.path.join(csrc, "sart.hip")).read()
    a, b = text.index("// ---- device code begin"), text.index("// ---- device code end")
    h.update(text[a:b].encode())
    return h.hexdigest()[:16]


SV = {"f32": 4, "bf16": 2, "f16": 2}


def setup(args, dev):
    """Device-resident inputs of the workload: a list of slices with A, p and
    the folded system."""
    from paper_1902_10559_amd import inputs, workloads
    if args.workload == "slice":
        sl = [workloads.single_slice(2, dev, args.wdtype, keep_host=True)]
        desc = ("512x128 slice (N=65536), K=24 sources over +-20 deg, 1024 bins (M=24576), "
                "40 ellipses, 1% noise")
    else:
        sl = workloads.batched_slices(256, dev, args.wdtype, progress=log)
        desc = ("256 slices of 1024 x nz voxels (nz in {32,...,128}), K=24 sources over +-20 deg, "
                "2048 bins (M=49152 per slice), 10 ellipses per slice, noise-free")
    lam = inputs.WORKLOADS[2 if args.workload == "slice" else 4].lam
    return sl, desc, lam


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(both halves and all slices run on one device); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1902_10559_amd import native

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.direct_only:
        print(json.dumps({"direct_normal_equations": direct_report(dev)}), flush=True)
        return
    if args.conv_only:
        print(json.dumps({"conv_layers": conv_report(dev)}), flush=True)
        return
    if args.polar_only:
        print(json.dumps({"polar_grid": polar_report(dev, 0.5)}), flush=True)
        return
    log(f"setting up workload {args.workload}")
    slices, desc, lam = setup(args, dev)
    systems = [x.S for x in slices]
    nnz_full = sum(x.A.nnz for x in slices)
    nnz_half = sum(S.nnz for S in systems)
    iters = args.iters
    # eq. (2) and the arrays of every matrix, checked as one batch
    out_validate = validation_report(slices)
    log(f"validation: {out_validate}")
    opts, lanes = choose_config(args, slices, systems, lam, iters)
    for S in systems:
        S.row_lanes, S.col_lanes = lanes
    sol = native.Solver(systems, opts)
    scratch = [S.new_image() for S in systems]
    f12 = [S.new_image() for S in systems]
    f_out = [torch.empty(2 * S.n, dtype=torch.float32, device=dev) for S in systems]
    log(f"slices={len(slices)} nnz={nnz_full} nnz_half={nnz_half} config {config_of(opts)} lanes {lanes}")
    fold_all, recombine_all = step_parts(slices, systems, f12, f_out)

    def split_step():
        fold_all()
        sol.solve(f12, want_iters=False)
        recombine_all()

    if args.subsets_only:
        ascending_order(slices, systems)
        print(json.dumps({"ordered_subsets": subsets_report(slices, systems, opts, dev, lam)}), flush=True)
        return

    ms, wall = timed(split_step, args.steps, args.warmup)
    value = iters * nnz_full / (ms * 1e-3)
    log(f"split step {ms:.3f} ms ({wall:.3f} s wall for {args.steps} steps)")
    out = {
        "metric": METRIC, "value": value, "unit": "nnz/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.wdtype if args.wdtype == "f32" else f"{args.wdtype} weights, f32 arithmetic",
        "data": "synthetic",
        "config": dict({"workload": f"{desc}; fold + {iters} split-SART iterations (lambda={lam}) "
                                    f"+ recombination per step",
                        "slices": len(slices), "nnz": int(nnz_full), "nnz_half": int(nnz_half),
                        "iterations": iters}, **config_of(opts)),
    }
    if args.no_extras:
        print(json.dumps(out), flush=True)
        return
    out["validate"] = out_validate

    # per-launch durations, stamped by the kernels' own dispatches on the
    # solver's stream, in the alternating forward/back sequence
    kern = kernel_report(sol, systems, scratch, opts, 2, SV[args.wdtype])
    out["roofline"] = roofline_of(kern, args)
    out["kernels"] = kern
    out["bytes_per_iteration"] = kern["bytes_per_iteration"]
    out["kernel_gbs_per_iteration"] = kern["gbs_per_iteration"]
    out["step_gbs"] = iters * kern["bytes_per_iteration"] / (ms * 1e-3) / 1e9

    # the unsplit A (same FP32 arithmetic, one value per entry), with the
    # same kind of kernels
    unsplit = [native.unsplit(x.A, x.p) for x in slices]
    uopts = unsplit_config(unsplit, opts, lam, iters)
    usol = native.Solver(unsplit, uopts)
    uscratch = [U.new_image() for U in unsplit]
    fu = [U.new_image() for U in unsplit]
    ums, _ = timed(lambda: usol.solve(fu, want_iters=False), args.steps, args.warmup)
    ukern = kernel_report(usol, unsplit, uscratch, uopts, 1, 4)
    out["unsplit"] = {"ms_per_step": ums, "value": iters * nnz_full / (ums * 1e-3),
                      "kernels": ukern, "bytes_per_iteration": ukern["bytes_per_iteration"],
                      "kernel_gbs_per_iteration": ukern["gbs_per_iteration"], "config": config_of(uopts)}
    out["split_vs_unsplit"] = ums / ms
    log(f"unsplit step {ums:.3f} ms; split/unsplit speedup {ums / ms:.2f}")

    # 16-bit weights: the same step with BF16 and FP16 storage of the pair
    low = {}
    if not args.no_dtypes and args.wdtype == "f32":
        for wd in ("bf16", "f16"):
            low[wd] = dtype_systems(slices, wd)
        out["weights_16bit"] = {wd: dtype_record(args, slices, low[wd], opts, lanes, wd, iters, nnz_full, timed)
                                for wd in low}
        log(f"16-bit weights: {out['weights_16bit']}")

    # time to relative residuals 1e-2 and 1e-3 on the workload itself
    # (capped at 10000 and 20000 iterations): split vs unsplit FP32, and
    # 16-bit weights
    ttr = {}
    ascending_order(slices, systems)
    if not args.no_ttr:
        ttr["workload"] = workload_time_to_tol(slices, systems, unsplit, low, opts, uopts, lanes, lam, dev)
        log(f"time to tolerance on the workload: {ttr['workload']}")
    for wd in list(low):
        del low[wd]
    del usol, uscratch, fu, unsplit
    torch.cuda.empty_cache()

    # ordered subsets (mirror-paired views) against SART, to rel_res 1e-2
    if not args.no_subsets:
        ascending_order(slices, systems)
        out["ordered_subsets"] = subsets_report(slices, systems, opts, dev, lam)
        log(f"ordered subsets: {out['ordered_subsets']}")

    # the direct path (Theorem 2) at Table 1's sizes: full system vs split pair
    if not args.no_direct:
        out["direct_normal_equations"] = direct_report(dev)
        log(f"direct path: {out['direct_normal_equations']}")

    # the polar grid of the closing example (Fig. 4) at 32768 voxels
    if not args.no_polar:
        out["polar_grid"] = polar_report(dev, lam)
        log(f"polar grid: {out['polar_grid']}")

    # plain vs learned-initialised SART on the 256 x 256 workload
    if not args.no_learned:
        out["learned"] = learned_report(dev)
        log(f"learned: {out['learned']}")

    ttr["64x64_slice_0.5pct_noise"] = small_slice_time_to_tol(dev, lam)
    out["time_to_1e-3"] = ttr
    log(f"time to 1e-3 (64x64): {ttr['64x64_slice_0.5pct_noise']}")

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, slices, iters, lam)
        log(f"cpu baseline {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


def timed(step, k, w):
    """Mean event time of k steps after w untimed ones, and the wall time."""
    import torch
    for _ in range(w):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(k):
        step()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / k, time.perf_counter() - t0


def step_parts(slices, systems, f12, f_out):
    """The fold of all slices and the recombination of all images: one launch
    per phase for a batch."""
    from paper_1902_10559_amd import native
    if len(slices) > 1:
        return (native.FoldBatch([x.A for x in slices], [x.p for x in slices], systems),
                native.RecombineBatch(f12, f_out))

    def fold_all():
        native.fold_into(slices[0].A, slices[0].p, systems[0])

    def recombine_all():
        native.recombine(f12[0], f_out[0])
    return fold_all, recombine_all


def config_of(o):
    """The launch configuration fields of a SartOptions, for the report."""
    return {"rows_per_wave": o.rows_per_wave, "cols_per_wave": o.cols_per_wave, "xcd_remap": o.xcd_remap,
            "unroll": o.unroll, "persistent": o.persistent, "chunked": o.chunked, "staged": o.staged,
            "band_width": o.band_width, "tile_cols": o.tile_cols, "tile_entries": o.tile_entries}


def lanes_of(o):
    """The line orders the step's fold writes for these options: the
    interleaved order for an unstaged kernel reading it in place, ascending
    for the staged ones."""
    rl = 64 // o.rows_per_wave if (o.chunked & 4) and not (o.staged & 1) else 0
    cl = 64 // o.cols_per_wave if (o.chunked & 8) and not (o.staged & 2) else 0
    return rl, cl


def validation_report(slices, reps=3):
    """ss_fold_size_batch on every matrix of the workload (eq. (2) bitwise,
    offsets, order, range, finiteness, CSR = CSC, the fold's size): best of
    `reps` event times."""
    import torch
    from paper_1902_10559_amd import native
    chk = native.FoldCheckBatch([x.A for x in slices], [x.p for x in slices])
    sizes = chk()
    best = 1e30
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        chk()
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    ok = all(S is None or k == S.nnz for k, S in zip(sizes, [x.S for x in slices]))
    return {"validate_ms": best, "matrices": len(slices), "sizes_match_fold": bool(ok)}


def choose_config(args, slices, systems, lam, iters):
    """The step's kernels: the autotuned unstaged launch shape (or --shape),
    a small search of the staged forms (or --staged), then whole steps timed
    for unstaged, staged and mixed forward/back choices; the fastest wins.
    Returns the options and the line orders the fold must write."""
    import dataclasses
    from paper_1902_10559_amd import native
    scratch = [S.new_image() for S in systems]
    base = native.SartOptions(lam=lam, max_iter=iters, use_graph=True, zero_start=True)
    for S in systems:
        S.row_lanes = S.col_lanes = 0
    if args.shape:
        (base.rows_per_wave, base.cols_per_wave, base.xcd_remap, base.unroll,
         base.persistent, base.chunked) = map(int, args.shape.split(","))
    else:
        sol = native.Solver(systems, base)
        sol.autotune(scratch)
        sol = pick_line_order(args, slices, systems, sol, scratch)
        base = sol.opts
    if args.staged:
        bits, band, tile, entries, cpw, unroll = map(int, args.staged.split(","))
        if bits == 0:
            return base, lanes_of(base)
        o = dataclasses.replace(base, staged=bits, band_width=band, tile_cols=tile, unroll=unroll,
                                tile_entries=entries if bits & 1 else 0,
                                cols_per_wave=cpw if bits & 2 else base.cols_per_wave)
        return o, lanes_of(o)
    fp, bp = staged_search(systems, base, scratch)
    # `unroll` sets the band kernel's batches only (the staged back
    # projection's chunks per pass follow its columns per wavefront)
    cands = [base,
             dataclasses.replace(base, staged=3, unroll=fp[2], band_width=fp[0], tile_entries=fp[1],
                                 cols_per_wave=bp[1], tile_cols=bp[0]),
             dataclasses.replace(base, staged=1, unroll=fp[2], band_width=fp[0], tile_entries=fp[1]),
             dataclasses.replace(base, staged=2, cols_per_wave=bp[1], tile_cols=bp[0])]
    best, best_ms = base, 1e30
    for o in cands:
        lanes = lanes_of(o)
        for S in systems:
            S.row_lanes, S.col_lanes = lanes
        f12 = [S.new_image() for S in systems]
        f_out = [S.new_image().view(-1) for S in systems]
        fold_all, recombine_all = step_parts(slices, systems, f12, f_out)
        slv = native.Solver(systems, o)

        def step():
            fold_all()
            slv.solve(f12, want_iters=False)
            recombine_all()
        ms, _ = timed(step, 3, 1)
        log(f"step candidate {config_of(o)}: {ms:.2f} ms")
        if ms < best_ms:
            best, best_ms = o, ms
        del slv, f12, f_out, fold_all, recombine_all
    for S in systems:
        S.row_lanes = S.col_lanes = 0
    return best, lanes_of(best)


def staged_search(systems, base, scratch):
    """Per-kernel times of a few staged shapes (systems in ascending order):
    the forward band width, work-tile entries and windows in flight (unroll),
    the back-projection tile width and columns per wavefront.  Returns
    (band, entries, unroll), (tile, cpw)."""
    import dataclasses
    import statistics
    from paper_1902_10559_amd import native

    def phases(o):
        # the median of three timings of 10 launches each: one timing that
        # comes back wrong (a stamp of a launch that did not run as timed)
        # does not pick the shape
        slv = native.Solver(systems, o)
        runs = [slv.time_phases(scratch, reps=10) for _ in range(3)]
        return [statistics.median(r[k] for r in runs) for k in range(3)]
    # A time under half the first candidate's is a timing that did not see
    # the launches it stamps (it has come back, for one shape, on every one
    # of the three timings) and is not taken: the shapes here differ by
    # tens of percent at most.  Bands of 2048 voxels are not tried: timed
    # as whole steps they were slower every time (217 and 216 ms against
    # 207-208 ms), while their phase timing was the one that came back short.
    fp_best, bp_best = ((4096, 2048, 4), 1e30), ((512, 8), 1e30)
    fp_ref = bp_ref = None
    for band, entries, unroll in ((4096, 2048, 4), (4096, 4096, 4), (4096, 1024, 4), (4096, 2048, 8)):
        o = dataclasses.replace(base, staged=1, band_width=band, tile_entries=entries, unroll=unroll, chunked=0)
        ms = phases(o)
        t = ms[0] + ms[1]
        fp_ref = t if fp_ref is None else fp_ref
        if t < 0.5 * fp_ref:
            log(f"staged search: forward {band, entries, unroll} timed {t:.4f} ms, not taken")
            continue
        if t < fp_best[1]:
            fp_best = ((band, entries, unroll), t)
    for tile, cpw in ((512, 8), (1024, 8), (256, 8), (512, 16)):
        o = dataclasses.replace(base, staged=2, tile_cols=tile, cols_per_wave=cpw, unroll=8, chunked=0)
        ms = phases(o)
        bp_ref = ms[2] if bp_ref is None else bp_ref
        if ms[2] < 0.5 * bp_ref:
            log(f"staged search: back {tile, cpw} timed {ms[2]:.4f} ms, not taken")
            continue
        if ms[2] < bp_best[1]:
            bp_best = ((tile, cpw), ms[2])
    log(f"staged search: forward {fp_best}, back {bp_best}")
    return fp_best[0], bp_best[0]


def unsplit_config(unsplit, opts, lam, iters):
    """The unsplit baseline's options: the split step's kinds of kernels
    (staged or not), with its own autotuned unstaged shape."""
    import dataclasses
    from paper_1902_10559_amd import native
    uopts = native.SartOptions(lam=lam, max_iter=iters, use_graph=True, zero_start=True)
    usol = native.Solver(unsplit, uopts)
    usol.autotune([U.new_image() for U in unsplit])
    uopts = usol.opts
    if opts.staged:
        uopts = dataclasses.replace(uopts, staged=opts.staged, band_width=opts.band_width,
                                    tile_cols=opts.tile_cols, tile_entries=opts.tile_entries,
                                    cols_per_wave=opts.cols_per_wave if opts.staged & 2 else uopts.cols_per_wave,
                                    unroll=opts.unroll)
    return uopts


def kernel_report(slv, systems, scratch, o, nv, sv):
    """Per-launch times of one iteration and the algorithmic bytes of each
    launch (the byte model of the kernels the options select); per launch
    the median of three timings of 50 iterations."""
    import statistics
    runs = [slv.time_phases(scratch, reps=50) for _ in range(3)]
    ms = [statistics.median(r[k] for r in runs) for k in range(3)]
    info = slv.staged_info(scratch) if o.staged else [0, 0, 0, 0, 0]
    nnz = sum(S.nnz for S in systems)
    m = sum(S.m for S in systems)
    n = sum(S.n for S in systems)
    ntiles_bp = sum((S.n + (o.tile_cols or 1024) - 1) // (o.tile_cols or 1024) for S in systems)
    fp_u, bp_u = bytes_per_iteration(nnz, m, n, nv, sv)
    rep = {"ms": {}, "bytes": {}}
    if o.staged & 1:
        segs = info[0]
        rep["ms"]["band_fp"], rep["ms"]["band_fin"] = ms[0], ms[1]
        # per entry its 16-bit index and values; per segment its sum; one
        # start bit per chunk of 4; the image once; 32 bytes per tile
        rep["bytes"]["band_fp"] = (nnz * (2 + nv * sv) + segs * 4 * nv + nnz // 32 + n * 4 * nv
                                   + 32 * info[1])
        # per row its slot range, p, 1/W and z; per segment its slot and sum
        rep["bytes"]["band_fin"] = m * (4 + 4 * nv + 4 + 4 * nv) + segs * (4 + 4 * nv)
        rep["segments"], rep["band_tiles"] = segs, info[1]
    else:
        rep["ms"]["sart_fp"] = ms[0]
        rep["bytes"]["sart_fp"] = fp_u
    if o.staged & 2:
        rep["ms"]["tile_bp"] = ms[2]
        rep["bytes"]["tile_bp"] = nnz * (2 + nv * sv) + n * (8 + 4 + 8 * nv) + m * 4 * nv + 16 * ntiles_bp
        rep["bp_tiles"], rep["bp_tiles_staged"], rep["bp_staged_rows"] = info[2], info[3], info[4]
    else:
        rep["ms"]["sart_bp"] = ms[2]
        rep["bytes"]["sart_bp"] = bp_u
    tot_b = sum(rep["bytes"].values())
    tot_ms = sum(rep["ms"].values())
    rep["bytes_per_iteration"] = tot_b
    rep["ms_per_iteration"] = tot_ms
    rep["gbs_per_iteration"] = tot_b / (tot_ms * 1e-3) / 1e9
    rep["gbs"] = {k: rep["bytes"][k] / (rep["ms"][k] * 1e-3) / 1e9 for k in rep["ms"] if rep["ms"][k] > 0}
    return rep


def roofline_of(kern, args):
    """The dominant launch (the longest) of an iteration against the HBM peak,
    with the hardware byte count when a matching profile is on file."""
    dom = max(kern["ms"], key=lambda k: kern["ms"][k])
    achieved = kern["bytes"][dom] / (kern["ms"][dom] * 1e-3) / 1e9
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"traffic_{args.workload}_{args.wdtype}.json")
    if os.path.exists(tfile):
        t = json.load(open(tfile))
        if t.get("source_hash") == source_hash() and dom in t.get("kernels", {}):
            traffic = t["kernels"][dom]["bytes_per_launch"]
    return {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": traffic, "algorithmic_bytes_per_launch": kern["bytes"][dom],
            "launch_ms": kern["ms"][dom]}


def dtype_systems(slices, wdtype):
    """The workload's split pairs with 16-bit weight storage (fold of every
    slice's A)."""
    from paper_1902_10559_amd import native
    out = []
    for x in slices:
        out.append(native.fold(x.A, x.p, wdtype, nnz_half=x.S.nnz))
    return out


def dtype_record(args, slices, systems, opts, lanes, wdtype, iters, nnz_full, timed_fn):
    """The step (fold + iterations + recombination) with 16-bit weights under
    the FP32 step's kernels, its per-launch times, GB/s and roofline."""
    import argparse
    import dataclasses
    import torch
    from paper_1902_10559_amd import native
    o = dataclasses.replace(opts)
    for S in systems:
        S.row_lanes, S.col_lanes = lanes
    f12 = [S.new_image() for S in systems]
    f_out = [torch.empty(2 * S.n, dtype=torch.float32, device=S.p.device) for S in systems]
    fold_all, recombine_all = step_parts([dataclasses.replace(x, S=S) for x, S in zip(slices, systems)],
                                         systems, f12, f_out)
    slv = native.Solver(systems, o)

    def step():
        fold_all()
        slv.solve(f12, want_iters=False)
        recombine_all()
    ms, _ = timed_fn(step, 5, 2)
    kern = kernel_report(slv, systems, [S.new_image() for S in systems], o, 2, SV[wdtype])
    for S in systems:
        S.row_lanes = S.col_lanes = 0
    # back to ascending order for the solves that follow
    native.FoldBatch([x.A for x in slices], [x.p for x in slices], systems)()
    return {"ms_per_step": ms, "value": iters * nnz_full / (ms * 1e-3), "kernels": kern,
            "roofline": roofline_of(kern, argparse.Namespace(**dict(vars(args), wdtype=wdtype)))}


def workload_time_to_tol(slices, systems, unsplit, low, opts, uopts, lanes, lam, dev, caps=((1e-2, 10000), (1e-3, 20000))):
    """workload_time_to_tol_one for each (tolerance, iteration cap)."""
    return {f"{tol:g}": workload_time_to_tol_one(slices, systems, unsplit, low, opts, uopts, lanes, lam, dev, tol, cap)
            for tol, cap in caps}


def workload_time_to_tol_one(slices, systems, unsplit, low, opts, uopts, lanes, lam, dev, tol, cap):
    """Iterations and time for every slice of the workload to reach rel_res
    <= tol from f0 = 0, each slice stopping on its own (the solve ends when
    all have, or at the cap): split vs unsplit in FP32 (the same k* per
    slice up to FP32 rounding, since by Theorem 1 the split iterates are the
    full ones), and split with BF16 / FP16 weights.  Events around the whole
    solve; host checks every 200 iterations."""
    import dataclasses
    import numpy as np
    import torch
    from paper_1902_10559_amd import native
    res = {"tol": tol, "cap": cap, "slices": len(slices)}
    ks = {}
    runs = [("split_f32", systems, opts), ("unsplit_f32", unsplit, uopts)]
    runs += [(f"split_{wd}", low[wd], opts) for wd in low]
    for name, syss, o in runs:
        for S in syss:
            S.row_lanes = S.col_lanes = 0
        oo = dataclasses.replace(o, max_iter=cap, tol=tol, check_every=200, zero_start=True)
        slv = native.Solver(syss, oo)
        imgs = [S.new_image() for S in syss]
        hist = [torch.empty(cap + 1, dtype=torch.float64, device=dev) for _ in syss]
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        st, it = slv.solve(imgs, hist)
        e1.record()
        torch.cuda.synchronize()
        it = np.array(it)
        reached = it < cap
        res[name] = {"median_iters": float(np.median(it)), "max_iters": int(it.max()),
                     "reached": int(reached.sum()), "all_reached": bool(reached.all()),
                     "seconds": e0.elapsed_time(e1) * 1e-3}
        if not reached.all():
            res[name]["not_reached"] = f"{int((~reached).sum())} slice(s) above {tol:g} after {cap} iterations"
        ks[name] = it
        log(f"time to {tol:g}: {name} {res[name]}")
        del slv, imgs, hist
    if "unsplit_f32" in ks:
        d = np.abs(ks["split_f32"] - ks["unsplit_f32"])
        res["split_vs_unsplit"] = {"same_kstar": int((d == 0).sum()), "max_kstar_difference": int(d.max()),
                                   "time_ratio": res["unsplit_f32"]["seconds"] / res["split_f32"]["seconds"]}
    return res


def learned_report(dev, train_items=4096, test_items=64, epochs=2):
    """Plain vs learned-initialised split SART on the 256 x 256 workload:
    training pairs (5 -> 200 split-SART iterations) generated and the network
    trained inside this run, then iterations and seconds to 1e-2 and 1e-3 on
    held-out phantoms from f0 = 0 and from the judged learned start."""
    from paper_1902_10559_amd import learned, unet
    t0 = time.perf_counter()
    sc = learned.scan(dev)
    X, Y = learned.make_pairs(sc, list(range(train_items)))
    t_data = time.perf_counter() - t0
    net = unet.UNet(sc.geom.nz, sc.geom.nx, seed=0)
    t1 = time.perf_counter()
    losses = learned.train(net, X, Y, epochs=epochs)
    t_train = time.perf_counter() - t1
    del X, Y
    rep = learned.evaluate(net, sc, list(range(10 ** 6, 10 ** 6 + test_items)))
    return {"workload": "256x256 slices, K=16 sources over +-20 deg, 512 bins, noise-free",
            "train_items": train_items, "epochs": epochs, "params": net.nparams,
            "data_seconds": t_data, "train_seconds": t_train, "final_loss": losses[-1], **rep}


def time_to_tol(slv, img, dev, tol=1e-3, cap=20000):
    """Iterations to rel_res <= tol from f0 = 0, then the time of exactly
    that many iterations (a second run with max_iter = k*, so that the graph
    chunks of the first run do not overshoot), by events on the stream."""
    import torch
    o = slv.opts
    saved = (o.max_iter, o.tol, o.check_every, o.zero_start)
    o.max_iter, o.tol, o.check_every, o.zero_start = cap, tol, 50, True
    hist = [torch.empty(cap + 1, dtype=torch.float64, device=dev) for _ in img]
    st, it = slv.solve(img, hist)
    k = it[0]
    rec = {"iterations": k, "reached": bool(st == 0), "final_rel_res": float(hist[0][k].item()), "cap": cap}
    o.max_iter, o.tol = k, 0.0
    slv.solve(img, want_iters=False)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    slv.solve(img, want_iters=False)
    e1.record()
    torch.cuda.synchronize()
    rec["seconds"] = e0.elapsed_time(e1) * 1e-3
    rec["us_per_iteration"] = rec["seconds"] * 1e6 / max(k, 1)
    o.max_iter, o.tol, o.check_every, o.zero_start = saved
    return rec


def pick_line_order(args, slices, systems, sol, scratch):
    """The step folds A on every pass, so it can write the lines in the
    solver's interleaved order at no cost (ss_system row_lanes/col_lanes),
    where the autotuner charges a copy per solve.  Times the tuned shape
    with both kernels reading that stored order against the tuned choice
    (kernel times, the fold's own time included) and keeps the faster;
    returns the solver to use (its opts updated in place)."""
    import dataclasses
    import torch
    from paper_1902_10559_amd import native
    opts = sol.opts
    if opts.chunked & 12 == 12:
        return sol

    def cost(o, rl, cl):
        for S in systems:
            S.row_lanes, S.col_lanes = rl, cl
        if len(slices) > 1:
            fold = native.FoldBatch([x.A for x in slices], [x.p for x in slices], systems)
        else:
            def fold():
                native.fold_into(slices[0].A, slices[0].p, systems[0])
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fold()
        torch.cuda.synchronize()
        e0.record()
        fold()
        e1.record()
        torch.cuda.synchronize()
        slv = native.Solver(systems, o)
        fp, bp = slv.time_kernels(scratch, reps=20)
        return args.iters * (fp + bp) + e0.elapsed_time(e1), slv

    tuned = dataclasses.replace(opts)
    stored = dataclasses.replace(opts, chunked=12)
    t_tuned, _ = cost(tuned, 64 // opts.rows_per_wave if opts.chunked & 4 else 0,
                      64 // opts.cols_per_wave if opts.chunked & 8 else 0)
    t_stored, _ = cost(stored, 64 // opts.rows_per_wave, 64 // opts.cols_per_wave)
    log(f"line order: tuned (chunked={opts.chunked}) {t_tuned:.1f} ms, "
        f"both interleaved {t_stored:.1f} ms per {args.iters} iterations + fold")
    if t_stored < t_tuned:
        opts.chunked = 12
    for S in systems:
        S.row_lanes = S.col_lanes = 0
    return native.Solver(systems, opts)


def ascending_order(slices, systems):
    """Folds the systems again, in ascending line order: the ordered-subset
    build needs each column's rows ascending.  Always refolds: the arrays
    may hold the order of the last configuration the search tried, whatever
    the order fields say."""
    from paper_1902_10559_amd import native
    for S in systems:
        S.row_lanes = S.col_lanes = 0
    if len(slices) > 1:
        native.FoldBatch([x.A for x in slices], [x.p for x in slices], systems)()
    else:
        native.fold_into(slices[0].A, slices[0].p, systems[0])


def os_forms(chunked):
    """Stream forms for the ordered-subset kernels: the forward projection
    keeps its form (interleaved included), the back projection, which has
    no interleaved form (it reads the subset-major copy), takes chunks where
    the SART one is chunked or interleaved."""
    return (chunked & 5) | (2 if chunked & 10 else 0)


def subsets_report(slices, systems, opts, dev, lam, tol=1e-2, cap=5000):
    """Whole-batch time to rel_res <= tol from f0 = 0: SART iterations
    against ordered-subset SART passes with S = K/2 mirror-paired views
    (every system stops on its own; the solve ends when all have)."""
    import numpy as np
    import torch
    from paper_1902_10559_amd import native
    S_count = slices[0].geom.K // 2
    subsets = [native.Subsets(S, S_count) for S in systems]
    import dataclasses
    rep = {"subsets": S_count, "tol": tol, "cap": cap}
    for name, every in (("sart", 0), ("os_sart", 1), ("os_sart_residual_every_4", 4)):
        if name == "sart":   # the step's kernels (staged where chosen)
            o = dataclasses.replace(opts, lam=lam, max_iter=cap, tol=tol, check_every=25, zero_start=True)
        else:
            # the subset back projection picks its own lanes per column (1/S
            # of each column per launch); 8 rows per wavefront and 8 entries
            # per lane and pass were the fastest ordered-subset shape on the
            # batch (3.85 ms per pass with the interleaved forward form,
            # against 3.96 with 4 entries)
            o = native.SartOptions(lam=lam, max_iter=cap, tol=tol, check_every=24, zero_start=True,
                                   rows_per_wave=8, cols_per_wave=0, xcd_remap=opts.xcd_remap, unroll=8,
                                   chunked=os_forms(opts.chunked), residual_every=every)
        slv = native.Solver(systems, o) if name == "sart" else native.OsSolver(systems, subsets, o)
        imgs = [S.new_image() for S in systems]
        slv.solve(imgs)                     # warm-up (graph capture)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        st, it = slv.solve(imgs)
        e1.record()
        torch.cuda.synchronize()
        rep[name] = {"median_steps": float(np.median(it)), "max_steps": int(max(it)), "reached": bool(st == 0),
                     "seconds": e0.elapsed_time(e1) * 1e-3}
    rep["speedup"] = rep["sart"]["seconds"] / rep["os_sart"]["seconds"]
    rep["speedup_residual_every_4"] = rep["sart"]["seconds"] / rep["os_sart_residual_every_4"]["seconds"]
    return rep


def polar_report(dev, lam, iters=100, reps=5):
    """The polar grid (128 rings x 256 sectors, N = 32768; 256 parallel views
    x 256 offsets, M = 65536; noise-free): 100 split-SART iterations against
    100 on the unsplit A, each autotuned and graph-replayed (best of `reps`),
    their kernels' algorithmic GB/s, and the fold."""
    import torch
    from paper_1902_10559_amd import native, workloads
    case = workloads.polar_case(8, dev)
    rep = {"M": case.A.M, "N": case.A.N, "nnz": case.A.nnz, "nnz_half": case.S.nnz, "iterations": iters}

    def best_of(fn):
        fn()
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    for name, S in (("split", case.S), ("unsplit", native.unsplit(case.A, case.p))):
        sol = native.Solver([S], native.SartOptions(lam=lam, max_iter=iters, use_graph=True))
        scratch = [S.new_image()]
        sol.autotune(scratch)
        f = [S.new_image()]
        ms = best_of(lambda: sol.solve(f, want_iters=False))
        fp, bp = sol.time_kernels(scratch, reps=50)
        a, b = bytes_per_iteration(S.nnz, S.m, S.n, S.nvals, 4)
        rep[name] = {"ms_per_iteration": ms / iters, "nnz_per_s": iters * case.A.nnz / (ms * 1e-3),
                     "fp_ms": fp, "bp_ms": bp, "kernel_gbs": (a + b) / ((fp + bp) * 1e-3) / 1e9}
    rep["split_vs_unsplit"] = rep["unsplit"]["ms_per_iteration"] / rep["split"]["ms_per_iteration"]
    rep["fold_ms"] = best_of(lambda: native.fold_into(case.A, case.p, case.S))
    return rep


FP64_PEAK_TFLOPS = 78.6   # MI355X dense FP64 (matrix cores and vector units alike)
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix cores

# each layer's input map in the network's buffers
CONV_INPUT = {"e1a": "x16", "e1b": "e1a", "e2a": "p1", "e2b": "e2a", "e3a": "p2", "e3b": "e3a", "ba": "p3",
              "bb": "ba", "bc": "bb", "bd": "bc", "be": "bd", "d3a": "c3", "d3b": "d3a", "d2a": "c2",
              "d2b": "d2a", "d1a": "c1", "d1b": "d1a", "out": "d1"}


def conv_report(dev, N=16, H=256, W=256, reps=20):
    """The learned initialiser's convolutions at the training shape (N
    images of H x W): per layer the forward, weight-gradient and
    input-gradient launches timed with events (best of `reps`), each
    2*9*C*O*N*h*w flop, against the BF16 matrix-core peak; and a whole
    training step (forward, backward, Adam, weight preparation)."""
    import torch
    from paper_1902_10559_amd import native, unet
    net = unet.UNet(H, W, device=dev, seed=0)
    g = torch.Generator(device="cpu").manual_seed(5)
    x32 = torch.rand(N, H, W, 1, generator=g).to(dev)
    tgt = (x32 + 0.05 * torch.randn(N, H, W, 1, generator=g).to(dev)).contiguous()
    x16 = torch.empty(x32.numel(), dtype=torch.int16, device=dev)
    native.nn_to_bf16(x32, x16)
    net.train_step(x32, x16, tgt, N, 1e-4)   # buffers, and every map filled
    B = net._bufs[N]

    def best(fn):
        fn()
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            t.append(e0.elapsed_time(e1))
        return min(t)
    layers, total_flop, total_ms = [], 0.0, 0.0
    for name, C, O, relu in unet.LAYERS:
        L = net.layers[name]
        lvl = unet.LEVEL[name]
        h, w = H >> lvl, W >> lvl
        xin = B[CONV_INPUT[name]]
        y = torch.empty(N * h * w * O, dtype=torch.float32 if name == "out" else torch.int16, device=dev)
        gy = torch.zeros(N * h * w * O, dtype=torch.int16, device=dev)
        gin = torch.empty(N * h * w * C, dtype=torch.float32, device=dev)
        flop = 2.0 * 9 * C * O * N * h * w
        t_f = best(lambda: native.nn_conv3x3(xin, N, h, w, C, L.wf, L.b, O, relu, y, name == "out"))
        t_w = best(lambda: native.nn_conv3x3_wgrad(xin, gy, N, h, w, C, O, L.gw, L.gb, ws=B["ws"]))
        t_d = best(lambda: native.nn_conv3x3(gy, N, h, w, O, L.wb, None, C, False, gin, True))
        rec = {"layer": name, "C": C, "O": O, "h": h, "w": w, "gflop": flop / 1e9}
        for k, t in (("forward", t_f), ("wgrad", t_w), ("dgrad", t_d)):
            rec[k] = {"ms": t, "tflops": flop / t / 1e9, "frac_bf16_peak": flop / t / 1e9 / BF16_PEAK_TFLOPS}
        layers.append(rec)
        total_flop += 3 * flop
        total_ms += t_f + t_w + t_d
    step = best(lambda: net.train_step(x32, x16, tgt, N, 1e-4))
    return {"shape": f"{N} x {H} x {W}", "layers": layers,
            "conv_total": {"gflop": total_flop / 1e9, "ms": total_ms, "tflops": total_flop / total_ms / 1e9},
            "train_step": {"ms": step, "tflops_conv": total_flop / step / 1e9}}


def direct_report(dev, sizes=(32, 64, 128), reps=3):
    """ss_normal_solve on the n x n slices of Table 1's shapes (M = 2304
    (n/32)^2 rays, N = n^2 voxels): the unsplit system against the split pair
    (both halves factored together), best of `reps` after a warm-up.  The
    Cholesky flop count is N^3/3 unsplit and 2 (N/2)^3/3 split; `tflops` is
    that count over the whole solve's time (formation and substitutions
    included), against the FP64 peak."""
    import numpy as np
    import torch
    from paper_1902_10559_amd import native, workloads
    rep = {}
    for n in sizes:
        case = workloads.table1_case(n, dev)
        N = case.A.N
        f_true = torch.from_numpy(workloads.phantom_snake(case.geom, 6, 0)).to(dev).double()
        row = {"M": case.A.M, "N": N, "nnz": case.A.nnz}
        for name, S, flops in (("unsplit", native.unsplit(case.A, case.p), N ** 3 / 3),
                               ("split", case.S, 2 * (N // 2) ** 3 / 3)):
            f = native.normal_solve(S)
            best = 1e30
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                native.normal_solve(S, f)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t0)
            err = float(torch.linalg.norm(f - f_true) / torch.linalg.norm(f_true))
            row[name] = {"ms": best * 1e3, "rel_err_vs_phantom": err,
                         "tflops": flops / best / 1e12, "frac_fp64_peak": flops / best / 1e12 / FP64_PEAK_TFLOPS}
        row["speedup"] = row["unsplit"]["ms"] / row["split"]["ms"]
        rep[f"{n}x{n}"] = row
        del case
    return rep


def small_slice_time_to_tol(dev, lam):
    """The 64 x 64 slice (K=10, 128 bins, 0.5% noise), which reaches 1e-3:
    split vs unsplit SART in FP32, and split SART with BF16 and FP16 weights."""
    from paper_1902_10559_amd import native, workloads
    res = {}
    for name, wdtype, split in (("split_f32", "f32", True), ("unsplit_f32", "f32", False),
                                ("split_bf16", "bf16", True), ("split_f16", "f16", True)):
        sl = workloads.single_slice(1, dev, wdtype)
        S = sl.S if split else native.unsplit(sl.A, sl.p, wdtype)
        slv = native.Solver([S], native.SartOptions(lam=lam, use_graph=True))
        slv.autotune([S.new_image()])
        res[name] = time_to_tol(slv, [S.new_image()], dev)
    return res


def cpu_baseline(args, slices, iters, lam):
    """The FP64 oracle on the host cores: fold + split SART + recombination
    on the same A and p, one thread, as many whole steps as fit in ~15 s
    (slice workload), or a sample of slices of the batched workload."""
    import scipy.sparse as sp
    from threadpoolctl import threadpool_limits

    from oracle import sart as OS
    from oracle import split as OSp
    from paper_1902_10559_amd import native

    if args.workload == "slice":
        sample = [slices[0]]
        what = "the whole workload"
    else:
        sample = [slices[0], slices[len(slices) // 2]]
        what = f"slices 0 and {len(slices) // 2} of {len(slices)}"
    mats = []
    for x in sample:
        hm = x.host or native.build_system(x.geom)
        mats.append((sp.csr_matrix((hm.val, hm.col_idx, hm.row_ptr), shape=(hm.M, hm.N)),
                     x.p.cpu().numpy()))
    nnz = sum(A.nnz for A, _ in mats)
    steps, t0 = 0, time.perf_counter()
    with threadpool_limits(1):
        while True:
            for A, p in mats:
                Sp = OSp.fold(A, "fp64")
                p1, p2 = OSp.fold_p(p)
                f1, f2, _ = OS.sart_split(Sp, p1, p2, lam, iters)
                OSp.recombine(f1, f2)
            steps += 1
            el = time.perf_counter() - t0
            if el > 15.0 or steps >= 20:
                break
    return {"value": steps * iters * nnz / el, "unit": "nnz/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} pass(es) over {what} (FP64 fold + {iters} split-SART iterations + "
                      f"recombination, numpy/scipy CSR, one thread), {el:.1f} s; the host offers "
                      f"{len(os.sched_getaffinity(0))} cores"}


if __name__ == "__main__":
    main()
