"""Pins for the polar-grid oracle (the closing example's geometry, Fig. 4):
eq. (2) bitwise, chord lengths against the closed form 2 sqrt(R^2 - t^2),
voxel areas from a dense parallel sweep, brute-force sampling along rays,
and the numbering's mirror pairing."""
import math

import numpy as np
import pytest

from oracle import geometry as G
from oracle import polar as P
from paper_1902_10559_amd import inputs


def _scan(rings=3, sectors=24, K=12, B=16, radius=300.0, offsets=None, phi=None):
    if phi is None:
        phi = inputs.parallel_views(K)
    if offsets is None:
        offsets = inputs.detector_bins(B, 2.0 * radius / B * 0.98)
    return inputs.PolarGeometry(rings, sectors, radius, np.asarray(phi), np.asarray(offsets))


def test_tgs_matrix_is_mirror_symmetric_and_complete():
    g = inputs.geometry_tgs()
    A = P.system_matrix(g)
    assert A.shape == (g.M, 72)
    assert G.is_symmetric(G.to_fp32(A))
    assert G.is_symmetric(A)
    # every voxel is crossed by some ray
    assert np.all(np.asarray((A != 0).sum(axis=0)).ravel() > 0)


def test_row_sums_are_chord_lengths():
    g = _scan(rings=5, sectors=12, K=8, B=40)
    A = P.system_matrix(g)
    rows = np.asarray(A.sum(axis=1)).ravel()
    R = g.radius
    for k in range(g.K):
        for b in range(g.B):
            t = g.offset[b]
            want = 2.0 * math.sqrt(R * R - t * t) if abs(t) < R else 0.0
            assert abs(rows[k * g.B + b] - want) <= 1e-9 * R


@pytest.mark.parametrize("phi0", [0.1234, 0.7, 1.3])
def test_dense_sweep_gives_voxel_areas(phi0):
    """One view of 6000 parallel rays of spacing delta covering the disk:
    sum_i w_ij * delta tends to the area of voxel j (error O(delta))."""
    B = 6000
    R = 100.0
    delta = 2.0 * R / B
    offsets = inputs.detector_bins(B, delta)
    g = inputs.PolarGeometry(4, 16, R, np.array([-phi0, phi0]), offsets)
    A = P.system_matrix(g)
    sweep = np.asarray(A[:B].sum(axis=0)).ravel() * delta
    area = np.array([P.voxel_area(g, j) for j in range(g.N)])
    assert np.allclose(sweep, area, rtol=2e-3, atol=0)
    assert abs(area.sum() - math.pi * R * R) < 1e-9 * R * R


def _brute(g, phi, t, steps=400000):
    """Lengths by sampling the chord at many points and classifying each
    point with full-circle polar coordinates (independent of the oracle's
    crossing logic)."""
    c, s = math.cos(phi), math.sin(phi)
    px, pz, dx, dz = t * c, t * s, s, -c
    R = g.radius
    if abs(t) >= R:
        return {}
    half = math.sqrt(R * R - t * t)
    u = (np.arange(steps) + 0.5) / steps * 2 * half - half
    x, z = px + u * dx, pz + u * dz
    ring = np.floor(np.hypot(x, z) * g.rings / R).astype(int)
    ang = np.mod(np.arctan2(x, z), 2 * math.pi)          # from +z towards +x
    sec = np.floor(ang / (2 * math.pi / g.sectors)).astype(int)   # 0..S-1 around the circle
    S2 = g.sectors // 2
    out = {}
    for r_, s_ in zip(ring, sec):
        if s_ < S2:      # x > 0: sector h = s_
            j = g.N - 1 - (r_ * S2 + s_)
        else:            # x < 0: angle from +z is 2 pi - ang
            j = r_ * S2 + (g.sectors - 1 - s_)
        out[j] = out.get(j, 0) + 1
    seg = 2 * half / steps
    return {j: n * seg for j, n in out.items()}


def test_lengths_match_brute_force_sampling():
    g = _scan(rings=3, sectors=24, K=4, B=6)
    for k in range(g.K):
        for b in range(g.B):
            j, w = P.polar_ray(g, float(g.phi[k]), float(g.offset[b]))
            got = {}
            for jj, ww in zip(j.tolist(), w.tolist()):
                got[jj] = got.get(jj, 0.0) + ww
            want = _brute(g, float(g.phi[k]), float(g.offset[b]))
            assert set(k_ for k_, v in want.items() if v > 0.05) <= set(got)
            for jj in set(got) | set(want):
                assert abs(got.get(jj, 0.0) - want.get(jj, 0.0)) <= 0.02, (k, b, jj)


def test_ray_reentering_an_annular_sector_sums_both_pieces():
    """A chord passing near the centre crosses the inner disk: the ring-1
    sector it leaves and re-enters on the same side gets both pieces."""
    g = inputs.PolarGeometry(2, 2, 10.0, np.array([-math.pi / 2, math.pi / 2]), np.array([-1.0, 1.0]))
    # S = 2: one sector per side.  Ray (phi = pi/2, t = 1): the horizontal
    # line z = 1 (direction (1, -cos)) crosses the outer ring on the left,
    # the inner disk, and the outer ring on the right.
    A = P.system_matrix(g).toarray()
    R, r1, t = 10.0, 5.0, 1.0
    outer = math.sqrt(R * R - t * t) - math.sqrt(r1 * r1 - t * t)
    inner = math.sqrt(r1 * r1 - t * t)
    i = 1 * g.B + 1   # phi = pi/2, t = 1
    row = A[i]
    # left side x < 0: ring 0 -> j = 0, ring 1 -> j = 1; right: ring 1 -> N-1-1 = 2, ring 0 -> 3
    assert np.allclose(row, [inner, outer, outer, inner], atol=1e-12)


def test_numbering_pairs_mirrors():
    g = _scan(rings=3, sectors=8)
    for r in range(3):
        for h in range(4):
            j = P.voxel_index(r, h, True, 3, 8)
            assert P.voxel_index(r, h, False, 3, 8) == g.N - 1 - j
    js = sorted(P.voxel_index(r, h, left, 3, 8) for r in range(3) for h in range(4) for left in (True, False))
    assert js == list(range(24))
