"""Split-SART benchmark on one MI355X.

One step is the whole hot path on one batch of input already resident in
HBM: fold A and p into the split pair (systems (3), (4) of the paper), run
100 SART iterations on both halves, recombine by Theorem 1, eq. (5).  Building
A (host Siddon) and synthesising p happen before the timed region.

Workload (default): a 512 x 128 voxel slice (N = 65536), 24 sources over +-20
degrees, 1024-bin detector (M = 24576), 40 random ellipses, 1 % noise, 100
iterations, FP32 values.  The same step on the unsplit A is timed beside it.

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

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "split-SART nnz/s & HBM GB/s vs unsplit; time to residual 1e-3 on 1 MI355X"
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_cfg2.json")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--iters", type=int, default=100, help="SART iterations per step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the timed steps (for profiler runs)")
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
    h = hashlib.sha256()
    for f in ("device.h", "sart.hip"):
        h.update(open(os.path.join(ROOT, "paper_1902_10559_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the two halves and all slices run on one device); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1902_10559_amd import inputs, native

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    wl = inputs.WORKLOADS[2]
    g = inputs.geometry_cfg2()
    log("building A (host Siddon)")
    hm = native.build_system(g)
    A = native.to_device(hm, dev)
    snake = native.snake_order(g.nx, g.nz)
    img = inputs.phantom_for(2, 0, g)
    f_true = np.zeros(g.N, np.float32)
    f_true[snake.ravel()] = img.ravel()
    q = native.project(A, torch.from_numpy(f_true).to(dev)).cpu().numpy()
    active = np.diff(hm.row_ptr) > 0
    p_host = inputs.add_noise(q, inputs.noise_draws(2, 0, g.M), active, wl.noise)
    p = torch.from_numpy(p_host).to(dev)
    nnz_half = native.fold_size(A, p)
    S = native.fold(A, p, "f32", nnz_half)
    U = native.unsplit(A, p)
    m, n = S.m, S.n
    iters = args.iters
    opts = native.SartOptions(lam=wl.lam, max_iter=iters, use_graph=True, zero_start=True)
    sol = native.Solver([S], opts)
    scratch = [S.new_image()]
    sol.autotune(scratch)
    f12 = [S.new_image()]
    f_out = torch.empty(g.N, dtype=torch.float32, device=dev)
    uopts = native.SartOptions(lam=wl.lam, max_iter=iters, use_graph=True, zero_start=True)
    usol = native.Solver([U], uopts)
    usol.autotune([U.new_image()])
    fu = [U.new_image()]
    log(f"M={g.M} N={g.N} nnz={hm.nnz} nnz_half={nnz_half} "
        f"split shape rpw={opts.rows_per_wave} cpw={opts.cols_per_wave} xcd={opts.xcd_remap}; "
        f"unsplit rpw={uopts.rows_per_wave} cpw={uopts.cols_per_wave} xcd={uopts.xcd_remap}")

    def split_step():
        native.fold_into(A, p, S)
        sol.solve(f12, want_iters=False)
        native.recombine(f12[0], f_out)

    def unsplit_step():
        usol.solve(fu, want_iters=False)

    def timed(step, k, w):
        for _ in range(w):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(k):
            step()
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return e0.elapsed_time(e1) / k, wall

    ms, wall = timed(split_step, args.steps, args.warmup)
    value = args.steps * iters * hm.nnz / (ms * 1e-3 * args.steps)
    log(f"split step {ms:.3f} ms ({wall:.3f} s wall for {args.steps} steps)")
    out = {
        "metric": METRIC, "value": value, "unit": "nnz/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "512x128 slice (N=65536), K=24 sources over +-20 deg, "
                               "1024 bins (M=24576), 40 ellipses, 1% noise; fold + 100 "
                               "split-SART iterations (lambda=0.5) + recombination per step",
                   "M": g.M, "N": g.N, "nnz": int(hm.nnz), "nnz_half": int(nnz_half),
                   "iterations": iters, "rows_per_wave": opts.rows_per_wave,
                   "cols_per_wave": opts.cols_per_wave, "xcd_remap": opts.xcd_remap},
    }
    if args.no_extras:
        print(json.dumps(out), flush=True)
        return

    # per-kernel durations (HIP events on the solver's stream) -> roofline
    fp_ms, bp_ms = sol.time_kernels(scratch, reps=100)
    fp_b, bp_b = bytes_per_iteration(nnz_half, m, n, 2, 4)
    dom = ("sart_fp", fp_ms, fp_b) if fp_ms >= bp_ms else ("sart_bp", bp_ms, bp_b)
    achieved = dom[2] / (dom[1] * 1e-3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        t = json.load(open(TRAFFIC_FILE))
        if t.get("source_hash") == source_hash() and dom[0] in t.get("kernels", {}):
            traffic = t["kernels"][dom[0]]["bytes_per_launch"]
    out["roofline"] = {"bound": "hbm", "kernel": dom[0], "achieved": achieved,
                       "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                       "traffic": traffic, "algorithmic_bytes_per_launch": dom[2],
                       "launch_ms": dom[1], "fp_ms": fp_ms, "bp_ms": bp_ms}
    it_s = (fp_b + bp_b) / ((fp_ms + bp_ms) * 1e-3) / 1e9
    out["iteration_gbs"] = it_s

    ums, _ = timed(unsplit_step, args.steps, args.warmup)
    ufp, ubp = usol.time_kernels([U.new_image()], reps=100)
    uf_b, ub_b = bytes_per_iteration(hm.nnz, g.M, g.N, 1, 4)
    out["unsplit"] = {"ms_per_step": ums, "value": iters * hm.nnz / (ums * 1e-3),
                      "fp_ms": ufp, "bp_ms": ubp,
                      "iteration_gbs": (uf_b + ub_b) / ((ufp + ubp) * 1e-3) / 1e9,
                      "bytes_per_iteration": uf_b + ub_b}
    out["split_vs_unsplit"] = ums / ms
    out["bytes_per_iteration"] = fp_b + bp_b
    log(f"unsplit step {ums:.3f} ms; split/unsplit speedup {ums / ms:.2f}")

    # time to relative residual 1e-3 (capped at 20000 iterations)
    ttr = {}
    for name, slv, img in (("split", sol, f12), ("unsplit", usol, fu)):
        o = slv.opts
        saved = (o.max_iter, o.tol, o.check_every)
        o.max_iter, o.tol, o.check_every = 20000, 1e-3, 100
        hist = torch.empty(20001, dtype=torch.float64, device=dev)
        if name == "split":
            native.fold_into(A, p, S)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, it = slv.solve(img, [hist])
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        h = hist[: it[0] + 1].cpu().numpy()
        ttr[name] = {"iterations": it[0], "seconds": secs, "reached": bool(st == 0),
                     "final_rel_res": float(h[-1])}
        o.max_iter, o.tol, o.check_every = saved
    out["time_to_1e-3"] = ttr
    log(f"time to 1e-3: {ttr}")

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, hm, p_host, iters)
        log(f"cpu baseline {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


def cpu_baseline(g, hm, p_host, iters):
    """The FP64 oracle on the host cores: fold + split SART + recombination
    on the same A and p, as many whole steps as fit in ~15 s (at least one)."""
    import scipy.sparse as sp
    from threadpoolctl import threadpool_limits

    from oracle import sart as OS
    from oracle import split as OSp
    A = sp.csr_matrix((hm.val, hm.col_idx, hm.row_ptr), shape=(hm.M, hm.N))
    steps, t0 = 0, time.perf_counter()
    with threadpool_limits(1):
        while True:
            Sp = OSp.fold(A, "fp64")
            p1, p2 = OSp.fold_p(p_host)
            f1, f2, _ = OS.sart_split(Sp, p1, p2, 0.5, iters)
            OSp.recombine(f1, f2)
            steps += 1
            el = time.perf_counter() - t0
            if el > 15.0 or steps >= 20:
                break
    return {"value": steps * iters * hm.nnz / el, "unit": "nnz/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{steps} whole step(s) of the same workload (FP64 fold + {iters} "
                      f"split-SART iterations + recombination, numpy/scipy CSR, one thread); "
                      f"{el:.1f} s; host has {len(os.sched_getaffinity(0))} cores available"}


if __name__ == "__main__":
    main()
