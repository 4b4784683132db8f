"""Pins of the geometry oracle (``oracle/geometry.py``) against what the
mathematics and independent libraries fix: the pinhole round trip in float64,
scikit-learn's DBSCAN, hand-built neighbourhoods, voxel grids with known
answers and set intersections computed another way.  Each pin takes the
oracle module as its argument so that planted mistakes can be run against
the same pins."""
from __future__ import annotations

import numpy as np

import disc_inputs as di


def _cam(rot=0.4, fx=500.0, fy=470.0):
    R = np.array([[np.cos(rot), 0.0, np.sin(rot)], [0.0, 1.0, 0.0], [-np.sin(rot), 0.0, np.cos(rot)]])
    return {"fx": fx, "fy": fy, "cx": 27.5, "cy": 19.0, "R": R, "t": np.array([0.5, -1.0, 2.0]),
            "depth_min": 0.2, "depth_max": 8.0}


def pin_bp_roundtrip(g, seed=61):
    """World points map back to their pixels and depths (float64 inverse of
    the pinhole model); counts and row-major order from an independent
    vectorised selection; stride and the depth range respected."""
    rng = np.random.default_rng(seed)
    h, w, stride = 41, 57, 2
    cam = _cam()
    depth = rng.uniform(0.5, 6.0, (h, w)).astype(np.float32)
    depth[rng.random((h, w)) < 0.1] = 0.0
    depth[4, 6] = 9.5  # beyond depth_max (on the stride grid)
    depth[6, 8] = np.nan
    u8 = (rng.random((3, h, w)) < 0.5).astype(np.uint8)
    u8[:2, 4, 6] = 1  # the out-of-range and the missing reading lie inside masks 0 and 1
    u8[:2, 6, 8] = 1
    u8[2] = 0
    pts, off = g.backproject(depth, di.pack_masks(u8), w, cam, stride)
    R, t = np.asarray(cam["R"]), np.asarray(cam["t"])
    for i in range(3):
        sel = u8[i].astype(bool) & np.isfinite(depth) & (depth >= 0.2) & (depth <= 8.0)
        grid = np.zeros((h, w), bool)
        grid[::stride, ::stride] = True
        ys, xs = np.nonzero(sel & grid)  # row-major
        p = pts[off[i]:off[i + 1]].astype(np.float64)
        assert len(p) == len(ys), f"mask {i}: point count"
        pc = (p - t) @ R  # R^T (p - t)
        assert np.allclose(pc[:, 2], depth[ys, xs], rtol=2e-6), "depth round trip"
        assert np.allclose(cam["fx"] * pc[:, 0] / pc[:, 2] + cam["cx"], xs, atol=2e-3), "column round trip"
        assert np.allclose(cam["fy"] * pc[:, 1] / pc[:, 2] + cam["cy"], ys, atol=2e-3), "row round trip"
    assert off[3] == off[2], "an empty mask has no points"


def pin_bp_plane(g):
    """Identity pose, constant depth: z is the depth exactly and neighbouring
    pixels are z / f apart."""
    h, w, z0 = 6, 9, 2.5
    cam = _cam(rot=0.0)
    cam["R"] = np.eye(3)
    cam["t"] = np.zeros(3)
    pts, off = g.backproject(np.full((h, w), z0, np.float32), di.pack_masks(np.ones((1, h, w), np.uint8)), w, cam, 1)
    assert off.tolist() == [0, h * w] and np.all(pts[:, 2] == np.float32(z0))
    grid = pts.reshape(h, w, 3).astype(np.float64)
    assert np.allclose(np.diff(grid[:, :, 0], axis=1), z0 / cam["fx"], rtol=1e-5)
    assert np.allclose(np.diff(grid[:, :, 1], axis=0), z0 / cam["fy"], rtol=1e-5)


def pin_dbscan_sklearn(g, seed=62):
    """Noise removal equals scikit-learn's DBSCAN (label -1 = removed) on
    random clusters with scattered outliers, per segment."""
    from sklearn.cluster import DBSCAN

    rng = np.random.default_rng(seed)
    segs = []
    for s in range(3):
        c = rng.uniform(-2, 2, (4, 3))
        blob = np.concatenate([c[k] + 0.05 * rng.standard_normal((60 + 20 * k, 3)) for k in range(4)])
        noise = rng.uniform(-3, 3, (25, 3))
        segs.append(np.concatenate([blob, noise]).astype(np.float32))
    pts = np.concatenate(segs)
    off = np.cumsum([0] + [len(x) for x in segs])
    eps, mp = 0.06, 5
    keep = g.dbscan_keep(pts, off, eps, mp)
    for s in range(3):
        lab = DBSCAN(eps=eps, min_samples=mp).fit(segs[s].astype(np.float64)).labels_
        assert np.array_equal(keep[off[s]:off[s + 1]].astype(bool), lab != -1), f"segment {s}"
    assert 0 < keep.sum() < len(keep)


def pin_dbscan_handmade(g):
    """A chain of points 0.8 eps apart with min_pts 3: inner points are core,
    the two ends border points (kept); an isolated point and a far pair are
    noise; segments do not see each other's points."""
    eps = 1.0
    chain = np.array([[0.8 * i, 0.0, 0.0] for i in range(6)], np.float32)
    lone = np.array([[50.0, 0.0, 0.0]], np.float32)
    pair = np.array([[0.0, 30.0, 0.0], [0.0, 30.9, 0.0]], np.float32)
    pts = np.concatenate([chain, lone, pair, chain[:2]])
    off = np.array([0, 6, 7, 9, 11])
    keep = g.dbscan_keep(pts, off, eps, 3)
    assert keep.tolist() == [1] * 6 + [0] + [0, 0] + [0, 0]
    keep1 = g.dbscan_keep(pts, off, eps, 1)
    assert keep1.all(), "min_pts 1: every point is core"


def pin_voxels_known(g):
    """Points at known voxel centres (negative coordinates included) with
    duplicates: the distinct voxels, in lexicographic order; keep flags
    exclude points."""
    v = 0.25
    cells = np.array([[1, 2, 3], [-1, 0, 0], [1, 2, 3], [0, -3, 5], [-1, 0, -1], [1, 1, 9]])
    pts = ((cells + 0.5) * v).astype(np.float32)
    keep = np.array([1, 1, 1, 1, 1, 0], np.uint8)
    vox, voff = g.voxelize(pts, np.array([0, 6]), keep, v)
    assert voff.tolist() == [0, 4]
    assert vox.tolist() == [[-1, 0, -1], [-1, 0, 0], [0, -3, 5], [1, 2, 3]]
    # a point just below a voxel boundary stays in the lower voxel
    vox2, _ = g.voxelize(np.array([[-1e-4, 0.2499, 0.0]], np.float32), np.array([0, 1]), None, v)
    assert vox2.tolist() == [[-1, 0, 0]]


def pin_overlap(g, seed=63):
    """Shared voxel counts equal row intersections computed with a
    structured-dtype view; identical sets give their size, disjoint 0."""
    rng = np.random.default_rng(seed)
    A = [np.unique(rng.integers(-4, 4, (n, 3)), axis=0).astype(np.int32) for n in (30, 50, 1)]
    B = [np.unique(rng.integers(-4, 4, (n, 3)), axis=0).astype(np.int32) for n in (40, 10)] + [A[0]]
    va, oa = np.concatenate(A), np.cumsum([0] + [len(x) for x in A])
    vb, ob = np.concatenate(B), np.cumsum([0] + [len(x) for x in B])
    pairs = [(i, j) for i in range(3) for j in range(3)]
    got = g.voxel_overlap(va, oa, vb, ob, pairs)
    dt = np.dtype([("x", np.int32), ("y", np.int32), ("z", np.int32)])
    for k, (i, j) in enumerate(pairs):
        want = len(np.intersect1d(np.ascontiguousarray(A[i]).view(dt), np.ascontiguousarray(B[j]).view(dt)))
        assert got[k] == want, f"pair {i},{j}"
    assert got[pairs.index((0, 2))] == len(A[0])
    far = g.voxel_overlap(va, oa, vb + 100, ob, [(0, 0)])
    assert far[0] == 0


ALL_GEOMETRY_PINS = [
    ("bp_roundtrip", pin_bp_roundtrip),
    ("bp_plane", pin_bp_plane),
    ("dbscan_sklearn", pin_dbscan_sklearn),
    ("dbscan_handmade", pin_dbscan_handmade),
    ("voxels_known", pin_voxels_known),
    ("overlap", pin_overlap),
]
