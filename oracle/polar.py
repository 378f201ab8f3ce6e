"""System matrix A of eq. (1) for a polar voxel grid scanned by parallel
beams (oracle): the second symmetric geometry of the paper's closing
example (tomographic gamma scanning of a cylindrical container, Fig. 4).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* Grid (a reading: Fig. 4 is not part of the text): a disk of radius R (mm)
  centred on the origin of the slice plane, cut into ``rings`` rings of equal
  width and ``sectors`` (even) sectors of equal angle whose boundaries
  include the symmetry axis OZ.  On either side of OZ a voxel is (ring r,
  counted from the centre; sector h, counted from +z by the angle
  atan2(|x|, z) in [0, pi]).
* Numbering (Fig. 4b as read here): the voxel (r, h) with x < 0 has index
  j = r*(S/2) + h and its mirror (x > 0) has N-1-j, so that eq. (2)'s
  pairing j <-> N-1-j is the mirror about OZ (N = rings * sectors).
* Scan: parallel beams.  View angles phi_k with phi[K-1-k] = -phi[k] and
  lateral offsets t_b with t[B-1-b] = -t[b] (both bitwise); ray i = k*B + b
  is the line {t_b n_k + u d_k} with n = (cos phi, sin phi) and
  d = (sin phi, -cos phi) (phi = 0: rays along -z), so ray M-1-i is the
  mirror of ray i.
* Weights: w_ij = length (mm) of ray i inside voxel j.  The ray's crossings
  with the ring circles and with the S/2 lines through the centre that carry
  the sector boundaries, sorted along the ray and clipped to the disk, cut
  the chord into segments that each lie in one voxel; a segment's voxel is
  that of its midpoint.  A line can cross one annular sector twice (the
  inner circle is concave; never more, since a line meets an annulus in at
  most two pieces and a wedge is convex), and the voxel then gets the sum of
  the two lengths.  Segments <= 1e-9 mm are dropped.
* Eq. (2) holds bitwise: cos and sin are taken of |phi| (sin carrying phi's
  sign), the boundary line of a mirrored sector has the exactly negated x
  direction, so a ray and its mirror have the same crossing parameters, and
  the voxel of a midpoint is found through |x|.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

MIN_SEGMENT_MM = 1e-9


def voxel_index(r, h, left, rings: int, sectors: int):
    """Index of voxel (ring r, sector h from +z) on the side x < 0 (left) or
    x > 0."""
    half = r * (sectors // 2) + h
    return half if left else rings * sectors - 1 - half


def boundary_lines(sectors: int):
    """Directions e_s (s = 0 .. S/2-1) of the full lines through the centre at
    angles 2 pi s / S from +z (each carries two sector boundaries).  The line
    S/2 - s is the mirror of line s, and its direction is built as the exact
    x-negation of line s's."""
    S2 = sectors // 2
    e = [None] * S2
    for s in range(S2):
        if s == 0:
            e[s] = (0.0, 1.0)
        elif 2 * s == S2:
            e[s] = (1.0, 0.0)
        elif 2 * s < S2:
            a = 2.0 * math.pi * s / sectors
            e[s] = (math.sin(a), math.cos(a))
    for s in range(S2):
        if e[s] is None:
            ex, ez = e[S2 - s]
            e[s] = (-ex, ez)
    return e


def ray_line(phi: float, t: float):
    """(px, pz, dx, dz): a point of the ray and its direction."""
    c = math.cos(abs(phi))
    s = math.copysign(math.sin(abs(phi)), phi)
    return t * c, t * s, s, -c


def polar_ray(g, phi: float, t: float):
    """Voxel indices (ascending) and FP64 lengths of one ray of the scan
    ``g`` (an object with rings, sectors, radius)."""
    px, pz, dx, dz = ray_line(phi, t)
    a = dx * dx + dz * dz
    b = 2.0 * (px * dx + pz * dz)
    pp = px * px + pz * pz
    R = g.radius
    disc = b * b - 4.0 * a * (pp - R * R)
    if not disc > 0.0:
        return np.zeros(0, np.int64), np.zeros(0)
    q = math.sqrt(disc)
    u0, u1 = (-b - q) / (2.0 * a), (-b + q) / (2.0 * a)
    # ring circles r = 1 .. rings-1
    rho = np.arange(1, g.rings) * R / g.rings
    dr = b * b - 4.0 * a * (pp - rho * rho)
    qr = np.sqrt(dr[dr > 0.0])
    ring_cuts = np.concatenate([(-b - qr) / (2.0 * a), (-b + qr) / (2.0 * a)])
    # sector-boundary lines through the centre
    e = np.array(boundary_lines(g.sectors))
    den = dx * e[:, 1] - dz * e[:, 0]
    nz_ = den != 0.0
    line_cuts = -(px * e[nz_, 1] - pz * e[nz_, 0]) / den[nz_]
    u = np.sort(np.concatenate([[u0, u1], ring_cuts, line_cuts]))
    u = u[(u >= u0) & (u <= u1)]
    length = (u[1:] - u[:-1]) * math.sqrt(a)
    mid = 0.5 * (u[:-1] + u[1:])
    keep = length > MIN_SEGMENT_MM
    length, mid = length[keep], mid[keep]
    mx, mz = px + mid * dx, pz + mid * dz
    ring = np.floor(np.sqrt(mx * mx + mz * mz) * g.rings / R).astype(np.int64)
    inside = ring < g.rings
    length, mx, mz, ring = length[inside], mx[inside], mz[inside], ring[inside]
    assert np.all(mx != 0.0), "segment midpoint on the symmetry axis"
    width = 2.0 * math.pi / g.sectors
    ang = np.array([math.atan2(abs(x), z) for x, z in zip(mx.tolist(), mz.tolist())])
    h = np.minimum(np.floor(ang / width).astype(np.int64), g.sectors // 2 - 1)
    half = ring * (g.sectors // 2) + h
    j = np.where(mx < 0.0, half, g.rings * g.sectors - 1 - half)
    # a line meets an annular sector in at most two pieces: sum them
    cols, inv = np.unique(j, return_inverse=True)
    w = np.zeros(cols.shape[0])
    np.add.at(w, inv, length)
    return cols, w


def system_matrix(g) -> sp.csr_matrix:
    """A (M x N) as FP64 CSR with ascending columns, for a scan ``g`` with
    rings, sectors, radius, phi (K) and offset (B)."""
    assert g.sectors % 2 == 0 and g.K % 2 == 0 and g.B % 2 == 0
    assert np.array_equal(g.phi[::-1], -g.phi), "views not mirror-exact"
    assert np.array_equal(g.offset[::-1], -g.offset), "offsets not mirror-exact"
    indptr = [0]
    cols, vals = [], []
    for k in range(g.K):
        for b in range(g.B):
            j, w = polar_ray(g, float(g.phi[k]), float(g.offset[b]))
            cols.append(j)
            vals.append(w)
            indptr.append(indptr[-1] + j.shape[0])
    A = sp.csr_matrix((np.concatenate(vals), np.concatenate(cols), np.array(indptr)), shape=(g.M, g.N))
    assert A.has_canonical_format
    return A


def voxel_area(g, j: int) -> float:
    """Area (mm^2) of voxel j: half the ring's annulus area over S/2 sectors."""
    half = j if j < g.N // 2 else g.N - 1 - j
    r = half // (g.sectors // 2)
    r0, r1 = r * g.radius / g.rings, (r + 1) * g.radius / g.rings
    return math.pi * (r1 * r1 - r0 * r0) / g.sectors
