"""Seeded synthetic inputs: scan geometries, ellipse phantoms and noise draws.

This module feeds both the reconstruction library and the FP64 checker. It
holds none of the reconstruction arithmetic: no voxel numbering, no ray
tracing, no fold, no solver. It only states the five workloads (grid size,
source and detector positions, phantom recipe, noise level, iteration count)
and draws the random numbers they need.

Conventions shared by every workload:

* The slice is a 2D grid of ``nx`` x ``nz`` square voxels of side ``pitch``
  (mm), centred on the OZ axis in x (x in [-nx*pitch/2, nx*pitch/2]) with its
  bottom face at z = 0.  A 2D image is an array ``img[r, c]`` with row r = 0 at
  the top (largest z) and column c = 0 at the most negative x.
* Sources sit in positions pairwise symmetric about OZ (Section 2 of the
  paper); the detector is a flat row of bins at ``det_z`` below the grid.
  Every mirrored coordinate is built as the exact negation of its partner, so
  ``src_x[K-1-k] == -src_x[k]`` and ``bin_x[B-1-b] == -bin_x[b]`` hold bitwise.
* Random streams: ``numpy.random.default_rng(SeedSequence([cfg, item,
  stream]))`` with stream 0 = phantom, 1 = noise, 2 = per-slice layout.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

STREAM_PHANTOM = 0
STREAM_NOISE = 1
STREAM_LAYOUT = 2


def rng_for(cfg: int, item: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([cfg, item, stream]))


@dataclasses.dataclass(frozen=True)
class Geometry:
    """One 2D slice and its scan: grid, K point sources, B detector bins."""

    nx: int
    nz: int
    pitch: float
    src_x: np.ndarray  # (K,) ascending, exact mirror pairs
    src_z: np.ndarray  # (K,)
    bin_x: np.ndarray  # (B,) ascending, exact mirror pairs
    det_z: float

    @property
    def K(self) -> int:
        return int(self.src_x.shape[0])

    @property
    def B(self) -> int:
        return int(self.bin_x.shape[0])

    @property
    def M(self) -> int:
        return self.K * self.B

    @property
    def N(self) -> int:
        return self.nx * self.nz


def mirrored(positive_half) -> np.ndarray:
    """Ascending array whose second half is ``positive_half`` and whose first
    half is its exact negation, reversed."""
    pos = np.asarray(positive_half, dtype=np.float64)
    return np.concatenate([-pos[::-1], pos])


def detector_bins(B: int, bin_pitch: float = 1.0) -> np.ndarray:
    """Centres of B flat-detector bins of width ``bin_pitch`` centred on OZ."""
    assert B % 2 == 0
    return mirrored((np.arange(B // 2) + 0.5) * bin_pitch)


def angular_sources(K: int, half_angle_deg: float, height: float,
                    det_z: float) -> tuple[np.ndarray, np.ndarray]:
    """K sources at ``height`` above the detector plane, at angles evenly
    spaced over [-half_angle, +half_angle] (endpoints included), seen from the
    origin of the detector: x = height * tan(theta)."""
    assert K % 2 == 0
    k = np.arange(K // 2)
    theta = np.deg2rad(half_angle_deg * (2 * k + 1) / (K - 1))
    src_x = mirrored(height * np.tan(theta))
    src_z = np.full(K, det_z + height)
    return src_x, src_z


def geometry_cfg1() -> Geometry:
    """64x64 slice, 1 mm voxels, 10 sources at z=600 mm, x=+-{20..180} mm,
    128-bin detector at z=-50 mm (M=1280, N=4096)."""
    src_x = mirrored([20.0, 60.0, 100.0, 140.0, 180.0])
    return Geometry(nx=64, nz=64, pitch=1.0, src_x=src_x,
                    src_z=np.full(10, 600.0), bin_x=detector_bins(128),
                    det_z=-50.0)


def geometry_cfg2() -> Geometry:
    """512x128 wide shallow slice, 24 sources over +-20 deg, 1024 bins
    (M=24576, N=65536)."""
    src_x, src_z = angular_sources(24, 20.0, 650.0, -50.0)
    return Geometry(nx=512, nz=128, pitch=1.0, src_x=src_x, src_z=src_z,
                    bin_x=detector_bins(1024), det_z=-50.0)


def geometry_cfg4_slice(s: int, nz: int) -> Geometry:
    """Slice s of the batched workload: 1024 x nz voxels, 24 sources over
    +-20 deg at height 650 + 0.5*s mm above the detector, 2048 bins."""
    src_x, src_z = angular_sources(24, 20.0, 650.0 + 0.5 * s, -50.0)
    return Geometry(nx=1024, nz=nz, pitch=1.0, src_x=src_x, src_z=src_z,
                    bin_x=detector_bins(2048), det_z=-50.0)


def cfg4_depths(n_slices: int = 256) -> np.ndarray:
    """Per-slice depth nz drawn uniformly from {32, 48, ..., 128}."""
    rng = rng_for(4, 0, STREAM_LAYOUT)
    return rng.choice(np.arange(32, 129, 16), size=n_slices).astype(np.int64)


def geometry_cfg5() -> Geometry:
    """256x256 slice, 16 sources over +-20 deg, 512 bins (M=8192, N=65536)."""
    src_x, src_z = angular_sources(16, 20.0, 650.0, -50.0)
    return Geometry(nx=256, nz=256, pitch=1.0, src_x=src_x, src_z=src_z,
                    bin_x=detector_bins(512), det_z=-50.0)


def geometry_normal(n: int) -> Geometry:
    """The shape of the paper's Table 1 experiment (Example 2): an n x n
    slice (n = 32, 64, 128) seen from K = 24 n/32 sources over +-30 degrees
    and B = 96 n/32 bins, so that A has M = 2304 (n/32)^2 rays for
    N = n^2 voxels (the paper: 2280, 9120, 36480) and full column rank;
    sources 100 n/32 mm above a detector plane 50 n/32 mm below the slice,
    0.7 mm bins."""
    s = n // 32
    assert n == 32 * s and s >= 1
    src_x, src_z = angular_sources(24 * s, 30.0, 100.0 * s, -50.0 * s)
    return Geometry(nx=n, nz=n, pitch=1.0, src_x=src_x, src_z=src_z,
                    bin_x=detector_bins(96 * s, 0.7), det_z=-50.0 * s)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    cfg: int
    n_ellipses: int
    noise: float  # relative noise level eta (0 = noise-free)
    iters: int
    lam: float = 0.5


WORKLOADS = {
    1: Workload("cfg1: 64x64 slice, K=10, 128 bins", 1, 10, 0.005, 20),
    2: Workload("cfg2: 512x128 slice, K=24 over +-20 deg, 1024 bins", 2, 40, 0.01, 100),
    3: Workload("cfg3: cfg1 geometry, bf16/fp16 weights", 3, 10, 0.005, 100),
    4: Workload("cfg4: 256 slices 1024 x nz, K=24, 2048 bins", 4, 10, 0.0, 100),
    5: Workload("cfg5: 256x256 slice, K=16, 512 bins", 5, 10, 0.0, 200),
    6: Workload("cfg6: Table 1 shapes, n x n slices, normal equations", 6, 10, 0.0, 0),
    7: Workload("cfg7: polar grid 3 rings x 24 sectors (72 voxels), 12 views x 24 offsets", 7, 4, 0.0, 20),
    8: Workload("cfg8: polar grid 128 rings x 256 sectors, 256 views x 256 offsets", 8, 10, 0.0, 100),
}


def geometry_for(cfg: int) -> Geometry:
    if cfg in (1, 3):
        return geometry_cfg1()
    if cfg == 2:
        return geometry_cfg2()
    if cfg == 5:
        return geometry_cfg5()
    raise ValueError("cfg4 has one geometry per slice: use geometry_cfg4_slice")


# ------------------------------------------------------- polar geometry
@dataclasses.dataclass(frozen=True)
class PolarGeometry:
    """A polar voxel grid (``rings`` x ``sectors`` voxels of a disk of
    ``radius`` mm, sector boundaries including OZ) and a parallel-beam scan
    (view angles ``phi`` in (-pi/2, pi/2), lateral offsets ``offset`` mm,
    both mirror-exact); ray i = k*B + b."""
    rings: int
    sectors: int
    radius: float
    phi: np.ndarray
    offset: np.ndarray

    @property
    def K(self) -> int:
        return int(self.phi.shape[0])

    @property
    def B(self) -> int:
        return int(self.offset.shape[0])

    @property
    def M(self) -> int:
        return self.K * self.B

    @property
    def N(self) -> int:
        return self.rings * self.sectors


def parallel_views(K: int) -> np.ndarray:
    """K view angles evenly spread over the half-turn (-pi/2, pi/2), mirror
    exact: (k + 1/2) pi / K - pi/2."""
    assert K % 2 == 0
    return mirrored((np.arange(K // 2) + 0.5) * (math.pi / K))


def geometry_tgs() -> PolarGeometry:
    """The closing example's size: 72 voxels (3 rings x 24 sectors) of a
    300 mm-radius container, 12 views x 24 offsets 25 mm apart (288 rays)."""
    return PolarGeometry(3, 24, 300.0, parallel_views(12), detector_bins(24, 25.0))


def geometry_polar_large() -> PolarGeometry:
    """128 rings x 256 sectors (N = 32768) of a 300 mm disk, 256 views x
    256 offsets 2.34375 mm apart (M = 65536)."""
    return PolarGeometry(128, 256, 300.0, parallel_views(256), detector_bins(256, 600.0 / 256))


def polar_voxel_centres(g: PolarGeometry) -> tuple[np.ndarray, np.ndarray]:
    """(x, z) of every voxel's centre (mid radius, mid angle) in index order
    j = r*(S/2) + h on the side x < 0, N-1-j for its mirror."""
    S2 = g.sectors // 2
    r = np.repeat(np.arange(g.rings), S2)
    h = np.tile(np.arange(S2), g.rings)
    rho = (r + 0.5) * g.radius / g.rings
    ang = (h + 0.5) * (2.0 * math.pi / g.sectors)
    x_left, z = -rho * np.sin(ang), rho * np.cos(ang)
    x = np.concatenate([x_left, -x_left[::-1]])
    zz = np.concatenate([z, z[::-1]])
    return x, zz


def polar_phantom(cfg: int, item: int, g: PolarGeometry) -> np.ndarray:
    """Seeded ellipses inside the disk (centres within 0.6 R, semi-axes in
    [0.1, 0.4] R, densities in [0.1, 1]) sampled at the voxel centres, as a
    vector in the polar numbering."""
    rng = rng_for(cfg, item, STREAM_PHANTOM)
    n = WORKLOADS[cfg].n_ellipses
    R = g.radius
    rad = 0.6 * R * np.sqrt(rng.uniform(0.0, 1.0, n))
    th = rng.uniform(0.0, 2.0 * math.pi, n)
    e = Ellipses(rad * np.sin(th), rad * np.cos(th), rng.uniform(0.1, 0.4, n) * R,
                 rng.uniform(0.1, 0.4, n) * R, rng.uniform(0.0, math.pi, n), rng.uniform(0.1, 1.0, n))
    x, z = polar_voxel_centres(g)
    f = np.zeros(g.N)
    for k in range(n):
        dx, dz = x - e.cx[k], z - e.cz[k]
        cs, sn = math.cos(e.phi[k]), math.sin(e.phi[k])
        u = (dx * cs + dz * sn) / e.a[k]
        v = (-dx * sn + dz * cs) / e.b[k]
        f += np.where(u * u + v * v <= 1.0, e.rho[k], 0.0)
    return f


# ----------------------------------------------------------------- phantoms
@dataclasses.dataclass(frozen=True)
class Ellipses:
    cx: np.ndarray
    cz: np.ndarray
    a: np.ndarray      # semi-axis along the rotated x direction (mm)
    b: np.ndarray      # semi-axis along the rotated z direction (mm)
    phi: np.ndarray    # rotation (rad)
    rho: np.ndarray    # additive density


def draw_ellipses(rng: np.random.Generator, g: Geometry, count: int) -> Ellipses:
    """``count`` ellipses with centres uniform over the slice, full axis
    lengths uniform in [4, 20] mm (semi-axes in [2, 10]), rotation uniform in
    [0, pi) and density uniform in [0.1, 1]."""
    half_w = 0.5 * g.nx * g.pitch
    height = g.nz * g.pitch
    cx = rng.uniform(-half_w, half_w, count)
    cz = rng.uniform(0.0, height, count)
    a = rng.uniform(2.0, 10.0, count)
    b = rng.uniform(2.0, 10.0, count)
    phi = rng.uniform(0.0, math.pi, count)
    rho = rng.uniform(0.1, 1.0, count)
    return Ellipses(cx, cz, a, b, phi, rho)


def phantom_image(g: Geometry, e: Ellipses) -> np.ndarray:
    """Sum of ellipse densities sampled at voxel centres, as ``img[r, c]``
    (row 0 on top), float64."""
    c = np.arange(g.nx)
    r = np.arange(g.nz)
    x = (c - g.nx / 2 + 0.5) * g.pitch
    z = (g.nz - r - 0.5) * g.pitch
    X, Z = np.meshgrid(x, z)  # (nz, nx)
    img = np.zeros((g.nz, g.nx))
    for k in range(e.cx.shape[0]):
        dx = X - e.cx[k]
        dz = Z - e.cz[k]
        cs, sn = math.cos(e.phi[k]), math.sin(e.phi[k])
        u = (dx * cs + dz * sn) / e.a[k]
        v = (-dx * sn + dz * cs) / e.b[k]
        img += np.where(u * u + v * v <= 1.0, e.rho[k], 0.0)
    return img


def phantom_for(cfg: int, item: int, g: Geometry) -> np.ndarray:
    wl = WORKLOADS[cfg]
    rng = rng_for(cfg, item, STREAM_PHANTOM)
    return phantom_image(g, draw_ellipses(rng, g, wl.n_ellipses))


# -------------------------------------------------------------------- noise
def noise_draws(cfg: int, item: int, M: int) -> np.ndarray:
    """Standard-normal draws, one per ray."""
    return rng_for(cfg, item, STREAM_NOISE).standard_normal(M)


def add_noise(q: np.ndarray, e: np.ndarray, active: np.ndarray,
              eta: float) -> np.ndarray:
    """Noisy projections ``q + s * e`` on the rays flagged ``active`` (rays
    that cross the grid), scaled so the noise norm is ``eta * ||q||``; rays
    that miss the grid keep q (= 0).  Returned as float32, the precision
    the reconstruction consumes."""
    q = np.asarray(q, dtype=np.float64)
    en = np.where(active, e, 0.0)
    nrm = float(np.linalg.norm(en))
    if eta == 0.0 or nrm == 0.0:
        return q.astype(np.float32)
    s = eta * float(np.linalg.norm(q)) / nrm
    return (q + s * en).astype(np.float32)
