"""Oracle pins for the voxel numbering and the Siddon system matrix.

The Siddon walk is checked against brute force (each voxel clipped against
the ray on its own), against the closed-form chord length of the ray inside
the grid box, against axis-parallel rays with known answers, and against the
plane-crossing count; eq. (2) is checked bitwise on generated matrices."""
import numpy as np
import pytest

from oracle import geometry as G
from paper_1902_10559_amd import inputs


def _clip(sx, sz, ex, ez, x0, x1, z0, z1):
    """Length of segment (sx,sz)-(ex,ez) inside the box [x0,x1]x[z0,z1]
    (Liang-Barsky parametric clipping)."""
    dx, dz = ex - sx, ez - sz
    t0, t1 = 0.0, 1.0
    for p, q in ((-dx, sx - x0), (dx, x1 - sx), (-dz, sz - z0), (dz, z1 - sz)):
        if p == 0.0:
            if q < 0.0:
                return 0.0
            continue
        t = q / p
        if p < 0.0:
            t0 = max(t0, t)
        else:
            t1 = min(t1, t)
    return max(0.0, t1 - t0) * np.hypot(dx, dz)


def _brute_row(g, sx, sz, ex, ez):
    row = np.zeros(g.N)
    H = g.nz * g.pitch
    for c in range(g.nx):
        x0 = (c - g.nx // 2) * g.pitch
        for r in range(g.nz):
            z1 = H - r * g.pitch
            w = _clip(sx, sz, ex, ez, x0, x0 + g.pitch, z1 - g.pitch, z1)
            if w > G.MIN_SEGMENT_MM:
                row[G.snake_index(c, r, g.nz)] = w
    return row


def _small_geometry(nx=8, nz=6, pitch=1.5):
    return inputs.Geometry(nx=nx, nz=nz, pitch=pitch,
                           src_x=inputs.mirrored([3.0, 17.5]),
                           src_z=np.full(4, 40.0),
                           bin_x=inputs.mirrored([0.25, 2.0, 5.5, 9.75, 20.0]),
                           det_z=-4.0)


def test_snake_numbering_is_a_bijection_with_mirror_pairing():
    for nx, nz in [(2, 1), (4, 3), (8, 6), (64, 64), (10, 7)]:
        c, r = np.meshgrid(np.arange(nx), np.arange(nz), indexing="ij")
        j = G.snake_index(c, r, nz)
        assert np.array_equal(np.sort(j.ravel()), np.arange(nx * nz))
        jm = G.snake_index(nx - 1 - c, r, nz)
        assert np.array_equal(jm, nx * nz - 1 - j)
        cc, rr = G.snake_to_2d(j, nz)
        assert np.array_equal(cc, c) and np.array_equal(rr, r)
        # vertical snake: consecutive indices are vertical neighbours inside
        # a column and horizontal neighbours across a column boundary
        cs, rs = G.snake_to_2d(np.arange(nx * nz), nz)
        step = np.abs(np.diff(cs)) + np.abs(np.diff(rs))
        assert np.all(step == 1)


def test_snake_with_odd_nx_breaks_the_mirror_pairing():
    nx, nz = 5, 3
    c, r = np.meshgrid(np.arange(nx), np.arange(nz), indexing="ij")
    j = G.snake_index(c, r, nz)
    assert not np.array_equal(G.snake_index(nx - 1 - c, r, nz), nx * nz - 1 - j)


def test_siddon_equals_brute_force_voxel_clipping():
    g = _small_geometry()
    rng = np.random.default_rng(7)
    rays = list(zip(*G.ray_endpoints(g)))
    # random rays, including ones entering through the sides or missing
    for _ in range(60):
        rays.append((rng.uniform(-20, 20), rng.uniform(-5, 30),
                     rng.uniform(-20, 20), rng.uniform(-5, 30)))
    for sx, sz, ex, ez in rays:
        j, w = G.siddon_ray(g, sx, sz, ex, ez)
        got = np.zeros(g.N)
        got[j] = w
        want = _brute_row(g, sx, sz, ex, ez)
        assert np.array_equal(got != 0, want != 0)
        assert np.max(np.abs(got - want)) < 1e-12


def test_siddon_row_sum_is_the_clipped_chord_length():
    g = inputs.geometry_cfg1()
    sx, sz, ex, ez = G.ray_endpoints(g)
    H = g.nz * g.pitch
    half = g.nx * g.pitch / 2
    for i in range(0, g.M, 7):
        j, w = G.siddon_ray(g, sx[i], sz[i], ex[i], ez[i])
        chord = _clip(sx[i], sz[i], ex[i], ez[i], -half, half, 0.0, H)
        assert abs(w.sum() - chord) < 1e-12


def test_axis_parallel_rays_give_pitch_weights():
    g = _small_geometry()
    # vertical ray down the middle of column 5
    x = (5 - g.nx // 2 + 0.5) * g.pitch
    j, w = G.siddon_ray(g, x, 50.0, x, -10.0)
    assert np.allclose(w, g.pitch, atol=1e-12) and len(j) == g.nz
    assert set(G.snake_to_2d(j, g.nz)[0]) == {5}
    # horizontal ray through row 2
    z = g.nz * g.pitch - 2.5 * g.pitch
    j, w = G.siddon_ray(g, -30.0, z, 30.0, z)
    assert np.allclose(w, g.pitch, atol=1e-12) and len(j) == g.nx
    assert set(G.snake_to_2d(j, g.nz)[1]) == {2}


def test_entries_per_ray_is_one_plus_interior_plane_crossings():
    g = inputs.geometry_cfg1()
    sx, sz, ex, ez = G.ray_endpoints(g)
    H = g.nz * g.pitch
    half = g.nx * g.pitch / 2
    X = (np.arange(g.nx + 1) - g.nx // 2) * g.pitch
    Z = np.arange(g.nz + 1) * g.pitch
    checked = 0
    for i in range(3, g.M, 11):
        j, w = G.siddon_ray(g, sx[i], sz[i], ex[i], ez[i])
        if len(j) == 0:
            continue
        # entry and exit points of the ray in the grid box, by clipping
        dx, dz = ex[i] - sx[i], ez[i] - sz[i]
        tx = sorted([(-half - sx[i]) / dx, (half - sx[i]) / dx])
        tz = sorted([(0.0 - sz[i]) / dz, (H - sz[i]) / dz])
        t0, t1 = max(0.0, tx[0], tz[0]), min(1.0, tx[1], tz[1])
        xa, xb = sorted([sx[i] + t0 * dx, sx[i] + t1 * dx])
        za, zb = sorted([sz[i] + t0 * dz, sz[i] + t1 * dz])
        crossings = np.sum((X > xa) & (X < xb)) + np.sum((Z > za) & (Z < zb))
        # a ray through a grid corner crosses two planes at once
        xs_at_z = sx[i] + (Z[(Z > za) & (Z < zb)] - sz[i]) / dz * dx
        corners = np.sum(np.abs(xs_at_z / g.pitch - np.round(xs_at_z / g.pitch)) < 1e-9)
        assert len(j) == 1 + crossings - corners
        checked += 1
    assert checked > 50


@pytest.mark.parametrize("g", [_small_geometry(), inputs.geometry_cfg1()],
                         ids=["small", "cfg1"])
def test_generated_matrix_satisfies_eq2_bitwise(g):
    A = G.system_matrix(g)
    assert A.shape == (g.M, g.N)
    assert G.is_symmetric(A)
    assert G.is_symmetric(G.to_fp32(A))
    D = A.toarray()
    assert np.array_equal(D, D[::-1, ::-1])
    # a single perturbed weight is detected
    B = G.to_fp32(A)
    k = B.indptr[g.M // 3] + 1
    B.data[k] = np.nextafter(B.data[k], np.float32(np.inf))
    assert not G.is_symmetric(B)


def test_cfg1_matrix_shape_and_statistics():
    g = inputs.geometry_cfg1()
    A = G.system_matrix(g)
    assert (g.M, g.N) == (1280, 4096)
    lens = np.diff(A.indptr)
    W = G.row_sums(A)
    assert np.all(np.diff(A.indices[A.indptr[5]:A.indptr[6]]) > 0)
    # every stored weight is a positive length no longer than a voxel diagonal
    assert A.data.min() > 0 and A.data.max() <= np.sqrt(2) * g.pitch + 1e-12
    assert np.array_equal(lens > 0, W > 0)
