"""Sphere geometry on the lattice, FP64.

Conventions (the paper is silent on them; the readings are stated here):
* cell (i, j, k) has its centre at (i + 1/2, j + 1/2, k + 1/2);
* displacements between a point and a sphere centre use the minimum image of
  the periodic box, applied once on the cell-centre displacement;
* a point is inside a sphere of radius R when |d|^2 <= R^2, evaluated as
  ((dx*dx + dy*dy) + dz*dz) without fused multiply-add.

Functions:
* ``min_image``        -- periodic minimum-image displacement.
* ``solid_cells``      -- binary mapping of Sec. 2.2 (cell solid iff its centre
                          is inside the sphere).
* ``link_delta``       -- delta_q of Sec. 2.2.1: the fraction of the link x -> x+c_q
                          at which the sphere surface lies, x_b = x + delta_q c_q.
* ``eps_flat`` / ``eps_recursive`` -- the supersampled solid volume fraction of
                          Sec. 2.3.2: the share of an n^3 grid of sub-cell-centre
                          sample points that lie inside the sphere; the recursive
                          form classifies whole octree blocks of sample points at
                          once and returns exactly the same count.
* ``eps_edge`` / ``eps_distance`` -- the two other estimators Sec. 2.3.2 names:
                          the covered share of the cell's twelve edges, and a
                          value from the distance of the cell centre to the
                          surface (reading: 1/2 - s clamped to [0, 1], s the
                          signed distance in cells; parity unpinned as a design).
"""
import math

import numpy as np


def min_image(d, L):
    """Wrap a displacement component into [-L/2, L/2)."""
    d = np.asarray(d, dtype=np.float64)
    d = np.where(d >= 0.5 * L, d - L, d)
    d = np.where(d < -0.5 * L, d + L, d)
    return d


def centre_disp(idx, X, L):
    """Minimum-image displacement of cell centre(s) idx + 1/2 from coordinate X."""
    return min_image((np.asarray(idx, dtype=np.float64) + 0.5) - X, L)


def dist2(dx, dy, dz):
    return (dx * dx + dy * dy) + dz * dz


def bbox_range(Xa, R, L):
    """Cell indices (unwrapped, then wrapped) along one axis that can touch the sphere."""
    lo = int(math.floor(Xa - R - 1.0))
    hi = int(math.floor(Xa + R + 1.0))
    idx = np.arange(lo, hi + 1)
    return np.mod(idx, L)


def solid_cells(shape, X, R):
    """Boolean mask [z, y, x] of cells whose centre lies inside the sphere."""
    nz, ny, nx = shape
    mask = np.zeros(shape, dtype=bool)
    ix = bbox_range(X[0], R, nx)
    iy = bbox_range(X[1], R, ny)
    iz = bbox_range(X[2], R, nz)
    dx = centre_disp(ix, X[0], nx)
    dy = centre_disp(iy, X[1], ny)
    dz = centre_disp(iz, X[2], nz)
    d2 = dist2(dx[None, None, :], dy[None, :, None], dz[:, None, None])
    inside = d2 <= R * R
    mask[np.ix_(iz, iy, ix)] = inside
    return mask


def link_delta(d, c, R):
    """delta_q of Sec. 2.2.1: smallest root in (0, 1] of |d + delta c|^2 = R^2, where
    d is the minimum-image displacement of the fluid cell centre x from the sphere
    centre and c = c_q points into the sphere.  With a = c.c, b = d.c and
    e = |d|^2 - R^2 > 0 the smaller root is e / (-b + sqrt(b^2 - a e))."""
    d = np.asarray(d, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    a = c[..., 0] * c[..., 0] + c[..., 1] * c[..., 1] + c[..., 2] * c[..., 2]
    b = d[..., 0] * c[..., 0] + d[..., 1] * c[..., 1] + d[..., 2] * c[..., 2]
    e = dist2(d[..., 0], d[..., 1], d[..., 2]) - R * R
    return e / (-b + np.sqrt(b * b - a * e))


def sample_offsets(n):
    """Offsets of the n sub-cell centres from the cell centre along one axis."""
    a = np.arange(n, dtype=np.float64)
    return (a + 0.5) / n - 0.5


def eps_flat_counts(dcx, dcy, dcz, R, n):
    """Number of the n^3 sample points inside the sphere for cells with centre
    displacements (dcx, dcy, dcz) (equal-length 1-D arrays)."""
    o = sample_offsets(n)
    px = dcx[:, None] + o[None, :]
    py = dcy[:, None] + o[None, :]
    pz = dcz[:, None] + o[None, :]
    sq = (px[:, None, None, :] * px[:, None, None, :] + py[:, None, :, None] * py[:, None, :, None]) + \
        pz[:, :, None, None] * pz[:, :, None, None]
    return (sq <= R * R).reshape(len(dcx), -1).sum(axis=1).astype(np.int64)


def _count_block(px, py, pz, R2):
    """Recursive count over a block of sample points given per-axis coordinate arrays."""
    # farthest sample point along each axis, and nearest (0 if the block straddles 0)
    fx, fy, fz = (max(abs(p[0]), abs(p[-1])) for p in (px, py, pz))
    if dist2(fx, fy, fz) <= R2:
        return len(px) * len(py) * len(pz)
    nx_, ny_, nz_ = (0.0 if (p[0] <= 0.0 <= p[-1]) else min(abs(p[0]), abs(p[-1])) for p in (px, py, pz))
    if dist2(nx_, ny_, nz_) > R2:
        return 0
    if len(px) == 1:
        return 1 if dist2(px[0], py[0], pz[0]) <= R2 else 0
    h = len(px) // 2
    total = 0
    for sz in (pz[:h], pz[h:]):
        for sy in (py[:h], py[h:]):
            for sx in (px[:h], px[h:]):
                total += _count_block(sx, sy, sz, R2)
    return total


def eps_recursive_count(dcx, dcy, dcz, R, n):
    """Recursive (octree) form of the supersampling count for one cell; n must be
    a power of two.  Blocks whose farthest sample point is inside count whole,
    blocks whose nearest sample point is outside count zero, others split."""
    assert n & (n - 1) == 0
    o = sample_offsets(n)
    px = [float(v) for v in (dcx + o)]
    py = [float(v) for v in (dcy + o)]
    pz = [float(v) for v in (dcz + o)]
    return _count_block(px, py, pz, R * R)


def overlap_cells(shape, X, R, n, recursive=False, estimator=None):
    """All cells with a nonzero solid fraction for one sphere: supersampled
    (flat or recursive), or by ``estimator`` ('edge' / 'distance') as a count
    out of n^3.

    Returns (iz, iy, ix, eps) with eps = count / n^3 > 0."""
    nz, ny, nx = shape
    ix = bbox_range(X[0], R, nx)
    iy = bbox_range(X[1], R, ny)
    iz = bbox_range(X[2], R, nz)
    gz, gy, gx = np.meshgrid(iz, iy, ix, indexing="ij")
    gz, gy, gx = gz.ravel(), gy.ravel(), gx.ravel()
    dcx = centre_disp(gx, X[0], nx)
    dcy = centre_disp(gy, X[1], ny)
    dcz = centre_disp(gz, X[2], nz)
    if estimator in ("edge", "distance"):
        f = eps_edge if estimator == "edge" else eps_distance
        counts = np.array([eps_count(f(np.array([a, b, c]), R), n) for a, b, c in zip(dcx, dcy, dcz)],
                          dtype=np.int64)
    elif recursive:
        counts = np.array([eps_recursive_count(a, b, c, R, n) for a, b, c in zip(dcx, dcy, dcz)], dtype=np.int64)
    else:
        counts = eps_flat_counts(dcx, dcy, dcz, R, n)
    keep = counts > 0
    eps = counts[keep].astype(np.float64) / float(n ** 3)
    return gz[keep], gy[keep], gx[keep], eps


def eps_edge(d, R):
    """Edge-intersection estimate of eps_s (Sec. 2.3.2): the length of the
    cell's twelve edges inside the sphere over their total length 12.  d: the
    cell-centre displacement from the sphere centre.  Edges are taken axis by
    axis (x, y, z); for each, the two other coordinates at (-1/2, -1/2),
    (+1/2, -1/2), (-1/2, +1/2), (+1/2, +1/2) (first of the two varying fastest)."""
    R2 = R * R
    total = 0.0
    for a in range(3):
        b, c = [k for k in range(3) if k != a]
        for s2 in (-0.5, 0.5):
            for s1 in (-0.5, 0.5):
                yb = d[b] + s1
                zc = d[c] + s2
                h2 = R2 - (yb * yb + zc * zc)
                if h2 > 0.0:
                    h = math.sqrt(h2)
                    lo = max(d[a] - 0.5, -h)
                    hi = min(d[a] + 0.5, h)
                    total += max(0.0, hi - lo)
    return min(1.0, total / 12.0)  # hi - lo of a fully covered edge may round above 1


def eps_distance(d, R):
    """Distance estimate of eps_s (Sec. 2.3.2): 1/2 minus the signed distance
    s = |d| - R of the cell centre from the surface (in cells), clamped to
    [0, 1] -- 1/2 on the surface, 1 half a cell inside, 0 half a cell outside."""
    r = math.sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2])
    return min(1.0, max(0.0, 0.5 - (r - R)))


def eps_count(eps, n):
    """An estimate expressed as a count out of n^3 (nearest, ties to even), the
    form every estimator of the library stores."""
    return int(np.rint(eps * float(n) ** 3))
