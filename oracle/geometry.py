"""Oracle of the geometry workload (arXiv 2603.03935, Sec. III-B): each
segment's depth is back-projected to a point cloud, denoised with DBSCAN and
voxelised; segments are associated with map instances by exact voxel
overlap.

TEST INFRASTRUCTURE ONLY: the test suite and the benchmark's CPU-baseline leg
are the only callers; the HIP library never imports this module.

Plain numpy, written from the definitions.  Where floating point decides an
integer (which points are neighbours within eps, which voxel a point falls
in) the arithmetic is IEEE single precision in a fixed order with every
operation rounded on its own (numpy float32 has no fused multiply-add), the
precision of the GPU path; the float64 pins in the tests check that these
single-precision points agree with the exact formulas.

Readings (the paper gives the steps, not their definitions):
  G-BP   pixel (x, y) of a mask with depth z (finite, depth_min <= z <=
         depth_max; others are missing readings) and x, y multiples of the
         stride maps to the camera point ((x - cx) z / fx, (y - cy) z / fy, z)
         and the world point R p + t (pinhole model, camera-to-world pose).
         A segment's points are listed in row-major pixel order.
  G-DB   DBSCAN noise removal: a point is a core point when at least min_pts
         points of its segment (itself included) lie within distance eps
         (squared distance <= eps^2); the points kept are the core points and
         the points within eps of a core point (the border points); the rest
         are DBSCAN's noise.  Which cluster a border point joins does not
         matter for the filter, so the kept set is unique.
  G-VOX  voxel of a kept point: floor(p / v) per axis; a segment's voxel set
         is the set of distinct voxels of its kept points, listed in
         lexicographic (x, y, z) order.
  G-OV   overlap of a segment and a map instance: the number of voxels in
         both sets.
"""
from __future__ import annotations

import numpy as np

F = np.float32


def backproject(depth: np.ndarray, bits: np.ndarray, w: int, cam: dict, stride: int = 1):
    """G-BP -> (points float32 [n][3], offsets int64 [m+1])."""
    depth = np.asarray(depth, dtype=np.float32)
    h = depth.shape[0]
    m = bits.shape[0]
    fx, fy, cx, cy = F(cam["fx"]), F(cam["fy"]), F(cam["cx"]), F(cam["cy"])
    R = np.asarray(cam["R"], dtype=np.float32)
    t = np.asarray(cam["t"], dtype=np.float32)
    dmin, dmax = F(cam["depth_min"]), F(cam["depth_max"])
    pts, off = [], [0]
    cols = np.arange(w)
    for i in range(m):
        u8 = ((bits[i][:, cols // 64] >> (cols % 64).astype(np.uint64)) & np.uint64(1)).astype(bool)
        ys, xs = [], []
        for y in range(0, h, stride):
            for x in range(0, w, stride):
                if not u8[y, x]:
                    continue
                z = depth[y, x]
                if not np.isfinite(z) or z < dmin or z > dmax:
                    continue
                ys.append(y)
                xs.append(x)
        ys = np.array(ys, dtype=np.float32)
        xs = np.array(xs, dtype=np.float32)
        z = depth[ys.astype(np.int64), xs.astype(np.int64)] if len(ys) else np.zeros(0, np.float32)
        xc = ((xs - cx) * z) / fx
        yc = ((ys - cy) * z) / fy
        pc = (xc, yc, z)
        world = [((R[k, 0] * pc[0] + R[k, 1] * pc[1]) + R[k, 2] * pc[2]) + t[k] for k in range(3)]
        pts.append(np.stack(world, axis=1).astype(np.float32) if len(ys) else np.zeros((0, 3), np.float32))
        off.append(off[-1] + len(ys))
    return (np.concatenate(pts) if pts else np.zeros((0, 3), np.float32)), np.array(off, dtype=np.int64)


def _sqdist(p: np.ndarray, q: np.ndarray) -> np.ndarray:
    """[a][3] x [b][3] -> [a][b] squared distances, float32, fixed order."""
    dx = p[:, None, 0] - q[None, :, 0]
    dy = p[:, None, 1] - q[None, :, 1]
    dz = p[:, None, 2] - q[None, :, 2]
    return (dx * dx + dy * dy) + dz * dz


def dbscan_keep(points: np.ndarray, offsets: np.ndarray, eps: float, min_pts: int, chunk: int = 512):
    """G-DB -> keep uint8 [n] (1 = core or border point)."""
    points = np.asarray(points, dtype=np.float32)
    eps2 = F(eps) * F(eps)
    keep = np.zeros(len(points), dtype=np.uint8)
    for i in range(len(offsets) - 1):
        a, b = int(offsets[i]), int(offsets[i + 1])
        seg = points[a:b]
        n = b - a
        if n == 0:
            continue
        core = np.zeros(n, dtype=bool)
        for s in range(0, n, chunk):
            core[s:s + chunk] = (_sqdist(seg[s:s + chunk], seg) <= eps2).sum(axis=1) >= min_pts
        cs = seg[core]
        k = core.copy()
        if len(cs):
            for s in range(0, n, chunk):
                k[s:s + chunk] |= (_sqdist(seg[s:s + chunk], cs) <= eps2).any(axis=1)
        keep[a:b] = k
    return keep


def voxelize(points: np.ndarray, offsets: np.ndarray, keep, v: float):
    """G-VOX -> (voxels int32 [nv][3] sorted per segment, voffsets int64 [m+1])."""
    points = np.asarray(points, dtype=np.float32)
    vox, off = [], [0]
    for i in range(len(offsets) - 1):
        a, b = int(offsets[i]), int(offsets[i + 1])
        p = points[a:b] if keep is None else points[a:b][np.asarray(keep[a:b]).astype(bool)]
        c = np.floor(p / F(v)).astype(np.int64)
        u = np.unique(c, axis=0) if len(c) else np.zeros((0, 3), np.int64)
        vox.append(u.astype(np.int32))
        off.append(off[-1] + len(u))
    return np.concatenate(vox) if vox else np.zeros((0, 3), np.int32), np.array(off, dtype=np.int64)


def voxel_overlap(vox_a, off_a, vox_b, off_b, pairs) -> np.ndarray:
    """G-OV -> count [len(pairs)] of voxels shared by segment i of A and
    instance j of B for each pair (i, j)."""
    out = np.zeros(len(pairs), dtype=np.int64)
    for k, (i, j) in enumerate(pairs):
        sa = {tuple(x) for x in vox_a[off_a[i]:off_a[i + 1]].tolist()}
        sb = {tuple(x) for x in vox_b[off_b[j]:off_b[j + 1]].tolist()}
        out[k] = len(sa & sb)
    return out
