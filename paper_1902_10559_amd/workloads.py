"""Device-resident workloads built through the library: the system matrix
from the host Siddon builder, synthetic projections from the library's own
forward projector, and the fold into the split pair.  Nothing here computes
on tensors itself; it only sequences library calls over the seeded inputs of
``inputs``."""
from __future__ import annotations

import concurrent.futures as cf
import dataclasses
import os

import numpy as np

from . import inputs, native


@dataclasses.dataclass
class Slice:
    geom: inputs.Geometry
    host: native.HostMatrix | None
    A: native.DeviceMatrix
    p: "torch.Tensor"
    S: native.System | None = None


def phantom_snake(g: inputs.Geometry, cfg: int, item: int) -> np.ndarray:
    """The seeded phantom of (cfg, item) as a vector in vertical-snake order,
    using the library's numbering (ss_snake_order)."""
    snake = native.snake_order(g.nx, g.nz)
    img = inputs.phantom_for(cfg, item, g)
    f = np.zeros(g.N, np.float32)
    f[snake.ravel()] = img.ravel()
    return f


def projections(A: native.DeviceMatrix, g: inputs.Geometry, f_true: np.ndarray, cfg: int,
                item: int, noise: float, device) -> "torch.Tensor":
    """p = A f_true by ss_project, plus the workload's seeded noise on the
    rays that cross the grid (none for a noise-free workload)."""
    import torch
    q = native.project(A, torch.from_numpy(f_true).to(device))
    if noise == 0.0:
        return q
    qh = q.cpu().numpy()
    active = np.diff(A.row_ptr.cpu().numpy()) > 0
    ph = inputs.add_noise(qh, inputs.noise_draws(cfg, item, g.M), active, noise)
    return torch.from_numpy(ph).to(device)


def single_slice(cfg: int, device="cuda", wdtype: str = "f32", keep_host: bool = False) -> Slice:
    g = inputs.geometry_for(cfg)
    hm = native.build_system(g)
    A = native.to_device(hm, device)
    wl = inputs.WORKLOADS[cfg]
    p = projections(A, g, phantom_snake(g, cfg, 0), cfg, 0, wl.noise, device)
    S = native.fold(A, p, wdtype)
    return Slice(g, hm if keep_host else None, A, p, S)


def batched_slices(n_slices: int = 256, device="cuda", wdtype: str = "f32",
                   p_override: dict | None = None, fold: bool = True,
                   progress=None) -> list[Slice]:
    """The batched workload: slice s has depth nz_s from ``cfg4_depths``, its
    own geometry (source height 650 + 0.5 s mm) and its own phantom; noise
    free.  Host matrices are built on a thread pool (the builder releases the
    interpreter lock) and uploaded one at a time.  ``p_override[s]`` replaces
    the projections of slice s (a float32 host array)."""
    import torch
    depths = inputs.cfg4_depths()[:n_slices]
    geoms = [inputs.geometry_cfg4_slice(s, int(depths[s])) for s in range(n_slices)]
    cores = max(1, len(os.sched_getaffinity(0)))
    workers = min(4, cores)
    per = max(1, cores // workers)
    out: list[Slice] = []
    with cf.ThreadPoolExecutor(workers) as ex:
        futs = [ex.submit(native.build_system, g, per) for g in geoms]
        for s, (g, fu) in enumerate(zip(geoms, futs)):
            hm = fu.result()
            A = native.to_device(hm, device)
            if p_override and s in p_override:
                p = torch.from_numpy(np.ascontiguousarray(p_override[s], np.float32)).to(device)
            else:
                p = projections(A, g, phantom_snake(g, 4, s), 4, s, 0.0, device)
            S = native.fold(A, p, wdtype) if fold else None
            out.append(Slice(g, None, A, p, S))
            futs[s] = None
            if progress and (s + 1) % 32 == 0:
                progress(f"built {s + 1}/{n_slices} slices")
    return out


def table1_case(n: int, device="cuda") -> Slice:
    """The direct path's workload at one of Table 1's sizes (n = 32, 64,
    128): the n x n slice of ``geometry_normal``, its seeded phantom and
    noise-free projections, and the fold."""
    g = inputs.geometry_normal(n)
    hm = native.build_system(g)
    A = native.to_device(hm, device)
    f = phantom_snake(g, 6, 0)
    p = projections(A, g, f, 6, 0, 0.0, device)
    return Slice(g, None, A, p, native.fold(A, p))


def polar_case(cfg: int, device="cuda") -> Slice:
    """A polar-grid workload (cfg 7: the closing example's 72 voxels; cfg 8:
    128 rings x 256 sectors): the library's polar matrix, noise-free
    projections of the seeded polar phantom, and the fold."""
    g = inputs.geometry_tgs() if cfg == 7 else inputs.geometry_polar_large()
    hm = native.build_polar_system(g)
    A = native.to_device(hm, device)
    f = inputs.polar_phantom(cfg, 0, g).astype(np.float32)
    p = projections(A, g, f, cfg, 0, inputs.WORKLOADS[cfg].noise, device)
    return Slice(g, None, A, p, native.fold(A, p))
