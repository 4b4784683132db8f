"""The geometry workload on the GPU (back-projection, DBSCAN noise removal,
voxel sets, voxel overlap), through the C ABI, against the oracle.

Bars: every output is compared exactly -- the points bit for bit (both sides
compute them in single precision, each operation rounded in the same order),
the keep flags, voxel lists, offsets and overlap counts element by element.
"""
import numpy as np
import pytest

import disc_inputs as di
from disc_inputs.scene import depth_scene
from gpu_common import dev_bits, torch
from oracle import geometry as og

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    t = torch()
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_03935_amd as disc

    disc.load()
    return disc


def _run_bp(gpu, sc, stride):
    t = torch()
    pts, off = gpu.backproject(t.from_numpy(sc.depth).cuda(), dev_bits(sc.bits), sc.h, sc.w, sc.camera, stride)
    t.cuda.synchronize()
    return pts.cpu().numpy(), off.cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("h,w,stride", [(120, 160, 1), (97, 130, 3), (480, 640, 2)])
def test_backproject_vs_oracle(gpu, h, w, stride):
    sc = depth_scene(di.frame_seed(9, h), h, w, n_obj=14 if h < 480 else 40)
    pts, off = _run_bp(gpu, sc, stride)
    rp, roff = og.backproject(sc.depth, sc.bits, sc.w, sc.camera, stride)
    assert np.array_equal(off, roff), "offsets"
    assert np.array_equal(pts.view(np.uint32), rp.view(np.uint32)), "points (bit for bit)"


def test_backproject_edge_cases(gpu):
    t = torch()
    h, w = 33, 70
    sc = depth_scene(di.frame_seed(9, 1), h, w, n_obj=5, min_area=1)
    bits = np.concatenate([sc.bits, np.zeros((1,) + sc.bits.shape[1:], np.uint64)])  # an empty mask last
    sc2 = type(sc)(sc.depth, bits, h, w, sc.camera)
    pts, off = _run_bp(gpu, sc2, 1)
    rp, roff = og.backproject(sc.depth, bits, w, sc.camera, 1)
    assert np.array_equal(off, roff) and off[-1] == off[-2]
    assert np.array_equal(pts.view(np.uint32), rp.view(np.uint32))
    # no masks
    pts0, off0 = gpu.backproject(t.from_numpy(sc.depth).cuda(), dev_bits(bits[:0]), h, w, sc.camera, 1)
    assert off0.cpu().tolist() == [0] and pts0.shape[0] == 0


@pytest.mark.parametrize("eps,min_pts", [(0.03, 8), (0.05, 20), (0.02, 1)])
def test_dbscan_vs_oracle(gpu, eps, min_pts):
    t = torch()
    sc = depth_scene(di.frame_seed(9, 2), 130, 180, n_obj=14)
    pts, off = _run_bp(gpu, sc, 1)
    keep = gpu.dbscan_denoise(t.from_numpy(pts).cuda(), t.from_numpy(off.astype(np.int32)).cuda(), eps, min_pts)
    want = og.dbscan_keep(pts, off, eps, min_pts)
    got = keep.cpu().numpy()
    assert np.array_equal(got, want), f"{(got != want).sum()} of {len(want)} flags differ"
    if min_pts > 1:
        assert 0 < (1 - want).sum() < len(want), "the scene has both noise and kept points"


@pytest.mark.parametrize("voxel", [0.02, 0.05])
def test_voxelize_vs_oracle(gpu, voxel):
    t = torch()
    sc = depth_scene(di.frame_seed(9, 3), 240, 320, n_obj=24)
    pts, off = _run_bp(gpu, sc, 2)
    dp, doff = t.from_numpy(pts).cuda(), t.from_numpy(off.astype(np.int32)).cuda()
    keep = gpu.dbscan_denoise(dp, doff, 0.04, 6)
    for k in (keep, None):
        vox, voff, status = gpu.voxelize(dp, doff, voxel, keep=k)
        rv, roff = og.voxelize(pts, off, None if k is None else keep.cpu().numpy(), voxel)
        assert not status.cpu().numpy().any()
        assert np.array_equal(voff.cpu().numpy(), roff), "voxel offsets"
        assert np.array_equal(vox.cpu().numpy(), rv), "voxel lists"


def test_voxel_overlap_vs_oracle(gpu):
    """Segments of one frame against the voxel sets of a second view of the
    same scene (shifted camera) and against themselves."""
    t = torch()
    sc = depth_scene(di.frame_seed(9, 4), 200, 260, n_obj=18)
    sc2 = depth_scene(di.frame_seed(9, 4), 200, 260, n_obj=18)
    sc2.camera["t"] = sc2.camera["t"] + np.array([0.03, 0.0, -0.02])
    sets = []
    for s in (sc, sc2):
        pts, off = _run_bp(gpu, s, 1)
        vox, voff, _ = gpu.voxelize(t.from_numpy(pts).cuda(), t.from_numpy(off.astype(np.int32)).cuda(), 0.05)
        sets.append((vox, voff))
    (va, oa), (vb, ob) = sets
    na, nb = oa.shape[0] - 1, ob.shape[0] - 1
    pairs = np.array([(i, j) for i in range(na) for j in range(nb)] + [(i, i) for i in range(na)] + [(-1, 0), (0, nb)],
                     np.int32)
    cnt = gpu.voxel_overlap(va, oa, vb, ob, t.from_numpy(pairs).cuda())
    want = og.voxel_overlap(va.cpu().numpy(), oa.cpu().numpy().astype(np.int64), vb.cpu().numpy(),
                            ob.cpu().numpy().astype(np.int64), [tuple(p) for p in pairs[:-2]])
    got = cnt.cpu().numpy()
    assert np.array_equal(got[:-2], want)
    assert got[-2] == 0 and got[-1] == 0, "pairs out of range count 0"
    assert got[:-2].max() > 0
    same = gpu.voxel_overlap(va, oa, va, oa, t.from_numpy(np.array([(i, i) for i in range(na)], np.int32)).cuda())
    assert np.array_equal(same.cpu().numpy(), np.diff(oa.cpu().numpy())), "a set overlaps itself completely"


def test_cloud_edge_cases(gpu):
    """Empty segments, a one-point segment, a segment with more distinct voxels
    than one workgroup sorts in LDS at once (10000: two chunks merged by rank)
    and a point whose voxel lies beyond the key range (status 1, the point
    left out)."""
    t = torch()
    rng = np.random.default_rng(71)
    v = 0.05
    grid = np.stack(np.meshgrid(np.arange(100), np.arange(100), [0], indexing="ij"), -1).reshape(-1, 3)
    segs = [np.zeros((0, 3)), np.array([[0.3, 0.2, 1.0]]), 0.3 + 0.01 * rng.standard_normal((5, 3)), np.zeros((0, 3)),
            (grid + 0.5) * v,                                            # 10000 distinct voxels
            np.concatenate([rng.uniform(-1, 1, (40, 3)), [[1e6, 0.0, 0.0]]])]  # one point far out
    pts = np.concatenate(segs).astype(np.float32)
    off = np.cumsum([0] + [len(x) for x in segs]).astype(np.int64)
    dp, doff = t.from_numpy(pts).cuda(), t.from_numpy(off.astype(np.int32)).cuda()
    keep = gpu.dbscan_denoise(dp, doff, 0.05, 3).cpu().numpy()
    assert np.array_equal(keep, og.dbscan_keep(pts, off, 0.05, 3))
    vox, voff, status = gpu.voxelize(dp, doff, v)
    voff, status, vox = voff.cpu().numpy(), status.cpu().numpy(), vox.cpu().numpy()
    assert status.tolist() == [0, 0, 0, 0, 0, 1]
    far = np.arange(len(pts)) != len(pts) - 1  # the oracle without the out-of-range point
    rv, roff = og.voxelize(pts, off, far.astype(np.uint8), v)
    assert np.array_equal(voff, roff), "voxel counts"
    for s in range(6):
        assert np.array_equal(vox[voff[s]:voff[s + 1]], rv[roff[s]:roff[s + 1]]), f"segment {s}"


def test_large_segment_voxels(gpu):
    """A 4 m x 4 m floor at 2 cm voxels (40000 distinct voxels, five sorted
    chunks merged by rank) beside small segments, with points in shuffled
    order and several points per voxel: the same sorted voxel list as the
    oracle."""
    t = torch()
    rng = np.random.default_rng(72)
    v = 0.02
    ij = np.stack(np.meshgrid(np.arange(200), np.arange(200), indexing="ij"), -1).reshape(-1, 2)
    floor = np.concatenate([(ij + rng.uniform(0.05, 0.95, ij.shape)) * v for _ in range(2)])
    floor = np.concatenate([floor, np.full((len(floor), 1), 0.013)], axis=1)
    floor = floor[rng.permutation(len(floor))]
    segs = [0.5 + 0.1 * rng.standard_normal((300, 3)), floor, np.zeros((0, 3)), rng.uniform(-3, 3, (9000, 3))]
    pts = np.concatenate(segs).astype(np.float32)
    off = np.cumsum([0] + [len(x) for x in segs]).astype(np.int64)
    vox, voff, status = gpu.voxelize(t.from_numpy(pts).cuda(), t.from_numpy(off.astype(np.int32)).cuda(), v)
    voff, status, vox = voff.cpu().numpy(), status.cpu().numpy(), vox.cpu().numpy()
    rv, roff = og.voxelize(pts, off, None, v)
    assert not status.any()
    assert roff[2] - roff[1] == 40000
    assert np.array_equal(voff, roff)
    assert np.array_equal(vox, rv)
