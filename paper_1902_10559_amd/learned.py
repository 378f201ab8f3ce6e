"""Learned SART initialiser on the 256 x 256 slice workload (K = 16 sources
over +-20 degrees, 512 bins): training pairs made by split SART itself
(input: the 5-iteration image, target: the 200-iteration image, both
recombined by eq. (5)), training of ``unet.UNet`` with the library's kernels,
and the residual-judged warm start.

SART stays the arbiter: a learned start is used only when its relative
residual ||p - A f|| / ||p|| is strictly below that of the 5-iteration image
it was computed from; otherwise the solve continues from that image.

Run ``python -m paper_1902_10559_amd.learned`` for the full experiment (data
generation, training, evaluation); it prints one JSON report.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import dataclasses
import json
import os
import sys
import time

import numpy as np

from . import inputs, native, unet, workloads

CFG = 5


@dataclasses.dataclass
class Scan:
    geom: inputs.Geometry
    A: native.DeviceMatrix
    S: native.System          # folded pair; p is replaced per phantom


def scan(device="cuda") -> Scan:
    import torch
    g = inputs.geometry_cfg5()
    A = native.to_device(native.build_system(g), device)
    S = native.fold(A, torch.zeros(A.M, dtype=torch.float32, device=device))
    return Scan(g, A, S)


def _phantoms(g, items):
    with cf.ThreadPoolExecutor(min(8, max(1, len(os.sched_getaffinity(0))))) as ex:
        return list(ex.map(lambda it: workloads.phantom_snake(g, CFG, it), items))


def folded_projections(sc: Scan, items):
    """p(1), p(2) (interleaved) of the noise-free projections of phantoms."""
    import torch
    out = []
    for f in _phantoms(sc.geom, items):
        q = native.project(sc.A, torch.from_numpy(f).to(sc.A.val.device))
        out.append(native.fold_rhs(q))
    return out


def systems_for(sc: Scan, p12s):
    return [dataclasses.replace(sc.S, p=p) for p in p12s]


def solve(systems, images, iters, zero_start, tol=0.0, check_every=50, res=None, shape=None):
    opts = native.SartOptions(lam=inputs.WORKLOADS[CFG].lam, max_iter=iters, tol=tol,
                              check_every=check_every, zero_start=zero_start)
    if shape:
        opts.rows_per_wave, opts.cols_per_wave, opts.xcd_remap = shape
    sol = native.Solver(systems, opts)
    return sol.solve(images, res)


def recombined_images(sc: Scan, f12s):
    """(B, nz, nx, 1) FP32 images of the recombined iterates."""
    import torch
    g = sc.geom
    B = len(f12s)
    snake = torch.empty((B, g.N), dtype=torch.float32, device=f12s[0].device)
    for b, f in enumerate(f12s):
        native.recombine(f, snake[b])
    img = torch.empty((B, g.nz, g.nx, 1), dtype=torch.float32, device=snake.device)
    native.nn_snake_image(snake, B, g.nx, g.nz, True, img)
    return img


def images_to_f12(sc: Scan, img):
    """Images (B, nz, nx, 1) -> split starts (interleaved halves)."""
    import torch
    g = sc.geom
    B = img.shape[0]
    snake = torch.empty((B, g.N), dtype=torch.float32, device=img.device)
    native.nn_snake_image(img, B, g.nx, g.nz, False, snake)
    return [native.image_fold(snake[b]) for b in range(B)]


def make_pairs(sc: Scan, items, iters_in=5, iters_out=200, batch=256, log=None):
    """Training pairs for phantoms `items`: (X, Y) images (n, nz, nx, 1) FP32."""
    import torch
    g = sc.geom
    n = len(items)
    X = torch.empty((n, g.nz, g.nx, 1), dtype=torch.float32, device=sc.A.val.device)
    Y = torch.empty_like(X)
    for s in range(0, n, batch):
        chunk = items[s:s + batch]
        systems = systems_for(sc, folded_projections(sc, chunk))
        f = [sc.S.new_image() for _ in chunk]
        solve(systems, f, iters_in, zero_start=True)
        X[s:s + len(chunk)] = recombined_images(sc, f)
        solve(systems, f, iters_out - iters_in, zero_start=False)
        Y[s:s + len(chunk)] = recombined_images(sc, f)
        if log:
            log(f"pairs {s + len(chunk)}/{n}")
    return X, Y


def train(net: unet.UNet, X, Y, epochs=2, batch=16, lr=1e-3, seed=0, log=None):
    """Minibatches are contiguous slices of the (already random) pairs, in a
    seeded random order each epoch."""
    import torch
    n = X.shape[0] // batch * batch
    X16 = torch.empty(X.numel(), dtype=torch.int16, device=X.device)
    native.nn_to_bf16(X, X16)
    per = X[0].numel()
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        for j, bi in enumerate(rng.permutation(n // batch)):
            s = bi * batch
            loss = net.train_step(X[s:s + batch], X16[s * per:(s + batch) * per], Y[s:s + batch], batch, lr)
            if j % 25 == 0:
                hist.append(loss.item())
        if log:
            log(f"epoch {ep + 1}: loss {hist[-1]:.4e}")
    return hist


def learned_starts(net: unet.UNet, sc: Scan, systems, f5, res5):
    """The network's starts from the 5-iteration iterates f5, each kept only
    if its relative residual is below res5 (that of f5); returns (starts,
    accepted flags, residuals of the learned starts)."""
    import torch
    img = recombined_images(sc, f5)
    B = img.shape[0]
    x16 = torch.empty(img.numel(), dtype=torch.int16, device=img.device)
    native.nn_to_bf16(img, x16)
    outs = []
    for b in range(B):   # batch 1 through the network
        per = img[b].numel()
        out = net.forward(img[b:b + 1], x16[b * per:(b + 1) * per], 1)
        outs.append(out.clone())
    cand = images_to_f12(sc, torch.stack(outs).view(B, *img.shape[1:]))
    hist = [torch.empty(1, dtype=torch.float64, device=img.device) for _ in range(B)]
    solve(systems, cand, 0, zero_start=False, res=hist)   # residual only, no update
    res_l = [h.item() for h in hist]
    starts, acc = [], []
    for b in range(B):
        ok = res_l[b] < res5[b]
        acc.append(ok)
        starts.append(cand[b] if ok else f5[b].clone())
    return starts, acc, res_l


def evaluate(net: unet.UNet, sc: Scan, items, tols=(1e-2, 1e-3), cap=20000, log=None):
    """Iterations to each tolerance from f0 = 0 (plain) and from the judged
    learned start (5 iterations + network, counted), on held-out phantoms."""
    import torch
    p12s = folded_projections(sc, items)
    systems = systems_for(sc, p12s)
    B = len(items)
    f5 = [sc.S.new_image() for _ in range(B)]
    h5 = [torch.empty(6, dtype=torch.float64, device=sc.A.val.device) for _ in range(B)]
    solve(systems, f5, 5, zero_start=True, res=h5)
    res5 = [h[5].item() for h in h5]
    starts, acc, res_l = learned_starts(net, sc, systems, f5, res5)
    report = {"phantoms": B, "accepted": int(sum(acc)), "res_after_5": float(np.median(res5)),
              "res_learned_start": float(np.median(res_l)), "tolerances": {}}
    for tol in tols:
        f = [sc.S.new_image() for _ in range(B)]
        t0 = time.perf_counter()
        _, it_plain = solve(systems, f, cap, zero_start=True, tol=tol, check_every=50)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        f = [s.clone() for s in starts]
        t0 = time.perf_counter()
        _, it_l = solve(systems, f, cap, zero_start=False, tol=tol, check_every=50)
        torch.cuda.synchronize()
        t_l = time.perf_counter() - t0
        it_learned = [5 + k for k in it_l]
        report["tolerances"][f"{tol:g}"] = {
            "plain_median_iters": float(np.median(it_plain)),
            "learned_median_iters": float(np.median(it_learned)),
            "plain_reached": int(sum(k < cap for k in it_plain)),
            "learned_reached": int(sum(k < cap for k in it_l)),
            "iteration_saving": float(1.0 - np.median(it_learned) / max(np.median(it_plain), 1)),
            "plain_seconds_batch": t_plain, "learned_seconds_batch": t_l}
        if log:
            log(f"tol {tol:g}: plain {np.median(it_plain)} learned {np.median(it_learned)}")
    return report


def save(net: unet.UNet, path: str, meta: dict):
    """Weights and Adam state as .npz plus a JSON header."""
    np.savez(path, params=net.params.cpu().numpy(), m=net.m.cpu().numpy(), v=net.v.cpu().numpy(),
             step=np.int64(net.step_count))
    with open(path + ".json", "w") as fh:
        json.dump(meta, fh, indent=1)


def load(net: unet.UNet, path: str):
    d = np.load(path, allow_pickle=False)
    net.load_params(d["params"])
    net.m.copy_(__import__("torch").from_numpy(d["m"]))
    net.v.copy_(__import__("torch").from_numpy(d["v"]))
    net.step_count = int(d["step"])


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-items", type=int, default=20000)
    ap.add_argument("--test-items", type=int, default=64)
    ap.add_argument("--epochs", type=int, default=2)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--cap", type=int, default=20000)
    ap.add_argument("--save", default="")
    args = ap.parse_args(argv)

    def log(*a):
        print("[learned]", *a, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    sc = scan()
    log(f"scan M={sc.A.M} N={sc.A.N} nnz={sc.A.nnz}")
    X, Y = make_pairs(sc, list(range(args.train_items)), log=log)
    t_data = time.perf_counter() - t0
    net = unet.UNet(sc.geom.nz, sc.geom.nx, seed=0)
    base = evaluate(net, sc, list(range(10 ** 6, 10 ** 6 + args.test_items)), cap=args.cap, log=log)
    t1 = time.perf_counter()
    tail = train(net, X, Y, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
    t_train = time.perf_counter() - t1
    rep = evaluate(net, sc, list(range(10 ** 6, 10 ** 6 + args.test_items)), cap=args.cap, log=log)
    out = {"workload": "256x256 slice, K=16 over +-20 deg, 512 bins; pairs: 5 -> 200 split-SART iterations",
           "train_items": args.train_items, "epochs": args.epochs, "batch": args.batch, "lr": args.lr,
           "params": net.nparams, "data_seconds": t_data, "train_seconds": t_train,
           "final_losses": tail[-5:], "untrained": base, "trained": rep}
    if args.save:
        save(net, args.save, out)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
