"""System matrix A of eq. (1) for a symmetric tomosynthesis scan (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* Voxel numbering -- Section 2 ("vertical snake", Fig. 1; the figure itself is
  not part of the text, so the reading below is stated): voxel columns are
  counted left to right (c = 0 at the most negative x), rows top to bottom
  (r = 0 at the top), and the index runs down even columns and up odd ones:
  ``j = c*nz + (r if c is even else nz-1-r)`` (0-based).  With nx even the
  mirror of voxel (c, r) about OZ, (nx-1-c, r), gets index N-1-j, the
  0-based form of the pairing j <-> N-j+1 used by eq. (2).
* Ray numbering: sources sorted by x, bins sorted by x, ray i = k*B + b.  The
  mirror of ray (k, b) is (K-1-k, B-1-b), index M-1-i.
* Weights: w_ij is the length (mm) of ray i inside voxel j (one ray from the
  source to each bin centre), found by Siddon's method: the ray's crossings
  with every grid plane, sorted by the ray parameter alpha, cut the ray into
  segments that each lie in one voxel.  Segments of length <= 1e-9 mm (corner
  touches) are dropped.
* Eq. (2) then holds bitwise when every mirrored coordinate is the exact
  negation of its partner: all alpha values of a ray and of its mirror agree
  bitwise, and the voxel column of a segment midpoint is computed from |x| so
  that mirrored midpoints land in mirrored columns.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

MIN_SEGMENT_MM = 1e-9


def snake_index(c, r, nz: int):
    """Vertical-snake index of voxel (column c, row r)."""
    c = np.asarray(c, dtype=np.int64)
    r = np.asarray(r, dtype=np.int64)
    return c * nz + np.where(c % 2 == 0, r, nz - 1 - r)


def snake_to_2d(j, nz: int):
    """Inverse of ``snake_index``: (c, r) of snake index j."""
    j = np.asarray(j, dtype=np.int64)
    c = j // nz
    s = j % nz
    r = np.where(c % 2 == 0, s, nz - 1 - s)
    return c, r


def image_to_snake(img: np.ndarray) -> np.ndarray:
    """2D image img[r, c] -> vector f in snake order."""
    nz, nx = img.shape
    j = np.arange(nx * nz)
    c, r = snake_to_2d(j, nz)
    return img[r, c]


def snake_to_image(f: np.ndarray, nx: int, nz: int) -> np.ndarray:
    j = np.arange(nx * nz)
    c, r = snake_to_2d(j, nz)
    img = np.zeros((nz, nx), dtype=np.asarray(f).dtype)
    img[r, c] = f
    return img


def ray_endpoints(g):
    """(sx, sz, dx_end, dz_end) for every ray, in ray order i = k*B + b."""
    K, B = g.K, g.B
    sx = np.repeat(g.src_x, B)
    sz = np.repeat(g.src_z, B)
    ex = np.tile(g.bin_x, K)
    ez = np.full(K * B, g.det_z)
    return sx, sz, ex, ez


def _column_of(x, nx: int, pitch: float):
    # computed from |x| so that x and -x give mirrored columns bitwise
    half = nx // 2
    return np.where(x >= 0, half + np.floor(x / pitch),
                    half - 1 - np.floor(-x / pitch)).astype(np.int64)


def siddon_ray(g, sx, sz, ex, ez):
    """Snake indices and FP64 intersection lengths of the ray from the source
    (sx, sz) to the detector point (ex, ez) through the grid of ``g``.
    Returns (cols, lengths) in order along the ray."""
    nx, nz, pitch = g.nx, g.nz, g.pitch
    X = (np.arange(nx + 1) - nx // 2) * pitch   # x-planes, X[nx-k] == -X[k]
    Z = np.arange(nz + 1) * pitch               # z-planes, bottom face z = 0
    dx = ex - sx
    dz = ez - sz
    d = np.sqrt(dx * dx + dz * dz)
    # parameter range of the ray inside the grid box (entry/exit)
    lo, hi = 0.0, 1.0
    if dx != 0.0:
        a0, a1 = (X[0] - sx) / dx, (X[-1] - sx) / dx
        lo, hi = max(lo, min(a0, a1)), min(hi, max(a0, a1))
    elif not (X[0] < sx < X[-1]):
        return np.zeros(0, np.int64), np.zeros(0)
    if dz != 0.0:
        a0, a1 = (Z[0] - sz) / dz, (Z[-1] - sz) / dz
        lo, hi = max(lo, min(a0, a1)), min(hi, max(a0, a1))
    elif not (Z[0] < sz < Z[-1]):
        return np.zeros(0, np.int64), np.zeros(0)
    if not lo < hi:
        return np.zeros(0, np.int64), np.zeros(0)
    parts = [np.array([lo, hi])]
    if dx != 0.0:
        ax = (X - sx) / dx
        parts.append(ax[(ax > lo) & (ax < hi)])
    if dz != 0.0:
        az = (Z - sz) / dz
        parts.append(az[(az > lo) & (az < hi)])
    alpha = np.sort(np.concatenate(parts))
    length = d * np.diff(alpha)
    mid = 0.5 * (alpha[:-1] + alpha[1:])
    keep = length > MIN_SEGMENT_MM
    length, mid = length[keep], mid[keep]
    xm = sx + mid * dx
    zm = sz + mid * dz
    c = _column_of(xm, nx, pitch)
    r = np.floor((Z[-1] - zm) / pitch).astype(np.int64)
    assert np.all((c >= 0) & (c < nx) & (r >= 0) & (r < nz))
    return snake_index(c, r, nz), length


def system_matrix(g) -> sp.csr_matrix:
    """A (M x N) as FP64 CSR with ascending column indices per row."""
    assert g.nx % 2 == 0, "vertical-snake mirror pairing needs nx even"
    assert g.K % 2 == 0 and g.B % 2 == 0
    assert np.array_equal(g.src_x[::-1], -g.src_x), "sources not mirror-exact"
    assert np.array_equal(g.src_z[::-1], g.src_z)
    assert np.array_equal(g.bin_x[::-1], -g.bin_x), "bins not mirror-exact"
    sx, sz, ex, ez = ray_endpoints(g)
    M, N = g.M, g.N
    rows, cols, vals = [], [], []
    for i in range(M):
        j, w = siddon_ray(g, sx[i], sz[i], ex[i], ez[i])
        order = np.argsort(j)
        j, w = j[order], w[order]
        assert np.all(np.diff(j) > 0), "a ray entered one voxel twice"
        rows.append(np.full(j.shape[0], i, np.int64))
        cols.append(j)
        vals.append(w)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    A = sp.csr_matrix((vals, (rows, cols)), shape=(M, N))
    A.sort_indices()
    assert A.has_canonical_format
    return A


def to_fp32(A: sp.csr_matrix) -> sp.csr_matrix:
    """Weights rounded to FP32: the matrix the reconstruction consumes."""
    B = sp.csr_matrix((A.data.astype(np.float32), A.indices.copy(),
                       A.indptr.copy()), shape=A.shape)
    return B


def is_symmetric(A: sp.csr_matrix) -> bool:
    """Eq. (2): w[i, j] == w[M-1-i, N-1-j] for every entry, bitwise (0-based
    indices), pattern included."""
    M, N = A.shape
    A = A.tocsr()
    for i in range(M):
        s, e = A.indptr[i], A.indptr[i + 1]
        t, u = A.indptr[M - 1 - i], A.indptr[M - i]
        if e - s != u - t:
            return False
        if not np.array_equal(A.indices[s:e], N - 1 - A.indices[t:u][::-1]):
            return False
        if not np.array_equal(A.data[s:e].view(np.uint8),
                              A.data[t:u][::-1].copy().view(np.uint8)):
            return False
    return True


def row_sums(A) -> np.ndarray:
    return np.asarray(A.astype(np.float64).sum(axis=1)).ravel()


def col_sums(A) -> np.ndarray:
    return np.asarray(A.astype(np.float64).sum(axis=0)).ravel()
