"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol include/disc.h declares, and rejects bad arguments before touching the
device."""
import ctypes
import os
import re

import pytest

import paper_2603_03935_amd as disc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "disc.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(disc_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(disc.LIB_PATH):
        import paper_2603_03935_amd.build as b

        b.build()
    return disc.load()


def test_exports_every_declared_symbol(lib):
    names = declared_symbols()
    assert names, "no declarations parsed"
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, f"libdisc.so lacks {missing}"
    assert sorted(disc.EXPORTS) == names, "binding's export list differs from the header"


def test_abi_version_and_defaults(lib):
    assert lib.disc_abi_version() == 5
    o = disc.Options()
    lib.disc_options_default(ctypes.byref(o))
    assert (o.spatial, o.distinct, o.gemm_dtype, o.edt_layout, o.pool_tile, o.pool_rows) == (0, 1, -1, -1, -1, -1)
    assert abs(o.eps - 1e-6) < 1e-12 and o.workspace is None and o.workspace_bytes == 0


FAKE = 1 << 20  # aligned, never dereferenced: validation fails before any device work


def good():
    t = disc.Tokens(FAKE, disc.DISC_F32, 30, 40, 1024, 16, None)
    m = disc.Masks(FAKE, 5, 480, 640)
    p = disc.Proj(FAKE, disc.DISC_F32, 1024, 768)
    o = disc.Out(FAKE, 5, 768, None, None)
    return t, m, p, o


def call(lib, t, m, p, o, opts=None):
    return lib.disc_embed_masks_ex(ctypes.byref(t) if t else None, ctypes.byref(m) if m else None,
                                   ctypes.byref(p) if p else None, ctypes.byref(o) if o else None,
                                   ctypes.byref(opts) if opts else None, None)


@pytest.mark.parametrize("mutate,code", [
    (lambda t, m, p, o: setattr(t, "gh", 29), 2),
    (lambda t, m, p, o: setattr(t, "c", 1000), 9),
    (lambda t, m, p, o: setattr(t, "dtype", 7), 3),
    (lambda t, m, p, o: setattr(t, "scale", FAKE), 1),
    (lambda t, m, p, o: setattr(t, "dtype", disc.DISC_F8E4M3), 1),
    (lambda t, m, p, o: setattr(t, "data", FAKE + 4), 4),
    (lambda t, m, p, o: setattr(t, "patch", 4), 9),
    (lambda t, m, p, o: setattr(m, "m", -1), 1),
    (lambda t, m, p, o: setattr(m, "bits", None), 1),
    (lambda t, m, p, o: setattr(m, "h", 2000), 9),
    (lambda t, m, p, o: setattr(p, "c", 512), 2),
    (lambda t, m, p, o: setattr(p, "e", 700), 9),
    (lambda t, m, p, o: setattr(p, "dtype", disc.DISC_F8E4M3), 3),
    (lambda t, m, p, o: setattr(o, "m", 4), 2),
    (lambda t, m, p, o: setattr(o, "e", 512), 2),
    (lambda t, m, p, o: setattr(o, "data", None), 1),
])
def test_validation_rejects(lib, mutate, code):
    t, m, p, o = good()
    mutate(t, m, p, o)
    st = call(lib, t, m, p, o)
    assert st == code, (st, disc.last_error())
    assert disc.last_error()


def test_null_arguments(lib):
    t, m, p, o = good()
    assert call(lib, None, m, p, o) == 1
    assert call(lib, t, None, p, o) == 1
    assert call(lib, t, m, None, o) == 1
    assert call(lib, t, m, p, None) == 1
    opts = disc.Options()
    lib.disc_options_default(ctypes.byref(opts))
    opts.spatial = 3
    assert call(lib, t, m, p, o, opts) == 1
    lib.disc_options_default(ctypes.byref(opts))
    opts.edt_layout = 3
    assert call(lib, t, m, p, o, opts) == 1
    lib.disc_options_default(ctypes.byref(opts))
    opts.pool_tile = 3
    assert call(lib, t, m, p, o, opts) == 1
    lib.disc_options_default(ctypes.byref(opts))
    opts.pool_rows = 96
    assert call(lib, t, m, p, o, opts) == 1


def test_workspace_bytes_is_host_only(lib):
    t, m, p, o = good()
    n = lib.disc_workspace_bytes(ctypes.byref(t), ctypes.byref(m), 1, ctypes.byref(p), None)
    # at least the spatial weights, GEMM weights and pooled features of 5 masks
    assert n >= 5 * 1200 * 4 + 5 * 1200 * 4 + 5 * 1024 * 4
    t.gh = 1
    assert lib.disc_workspace_bytes(ctypes.byref(t), ctypes.byref(m), 1, ctypes.byref(p), None) == 0


def test_stage_validation(lib):
    m = disc.Masks(FAKE, 3, 10, 10)
    assert lib.disc_edt_sq(ctypes.byref(m), None, None) == 1
    assert lib.disc_edt_sq(ctypes.byref(m), FAKE + 8, None) == 4
    assert lib.disc_pack_masks(None, 1, 4, 4, FAKE, None) == 1
    assert lib.disc_pack_masks(FAKE, 1, 0, 4, FAKE, None) == 1
    t = disc.Tokens(FAKE, disc.DISC_F32, 4, 4, 64, 16, None)
    opts = disc.Options()
    lib.disc_options_default(ctypes.byref(opts))
    mm = disc.Masks(FAKE, 3, 64, 64)
    assert lib.disc_patch_weights(ctypes.byref(t), ctypes.byref(mm), 8, ctypes.byref(opts), FAKE, None) == 2
    assert lib.disc_token_stats(ctypes.byref(t), -1.0, None, None, None, None) == 1


def test_zero_masks_is_noop(lib):
    t, m, p, o = good()
    m.m = 0
    o.m = 0
    assert call(lib, t, m, p, o) == 0


def test_query_validation(lib):
    """disc_query_topk rejects bad arguments on the host (nothing is launched)."""
    def q(m=10, e=64, k=4, dt=disc.DISC_F32, qn=3, text=FAKE, sim=FAKE):
        return lib.disc_query_topk(FAKE, m, text, dt, qn, e, k, sim, FAKE, FAKE, None)
    assert q(e=60) == 9 and q(e=0) == 9 and q(e=8192) == 9
    assert q(k=0) == 9 and q(k=257) == 9
    assert q(dt=disc.DISC_F8E4M3) == 3
    assert q(m=-1) == 1 and q(text=None) == 1 and q(sim=None) == 1
    assert q(text=FAKE + 8) == 4
    assert q(qn=0) == 0  # no queries: nothing to do


def test_quality_and_fusion_validation(lib):
    """disc_view_quality / disc_angle_score / disc_fuse reject bad arguments on
    the host (nothing is launched); zero observations are a no-op."""
    def vq(m=10, e=64, h=480, w=640, lam=3.3, emb=FAKE, area=FAKE, comp=None):
        return lib.disc_view_quality(area, FAKE, emb, FAKE, None, m, e, h, w, lam, FAKE, comp, None)
    assert vq(e=62) == 9 and vq(e=0) == 9 and vq(e=8192) == 9
    assert vq(h=0) == 2 and vq(w=-1) == 2
    assert vq(lam=0.0) == 1 and vq(lam=-1.0) == 1 and vq(lam=float("nan")) == 1
    assert vq(m=-1) == 1 and vq(area=None) == 1 and vq(emb=FAKE + 4) == 4 and vq(comp=FAKE + 8) == 4
    assert vq(m=0) == 0

    def ang(m=10, nv=100, rays=FAKE, off=FAKE):
        return lib.disc_angle_score(rays, FAKE, nv, off, m, FAKE, None)
    assert ang(m=-1) == 1 and ang(nv=-1) == 1 and ang(nv=1 << 30) == 9
    assert ang(off=None) == 1 and ang(rays=None) == 1
    assert ang(m=0) == 0

    def fu(m=10, e=64, n_map=5, ids=FAKE, emb=FAKE, map_emb=FAKE):
        return lib.disc_fuse(ids, FAKE, emb, m, e, FAKE, map_emb, n_map, None, None)
    assert fu(e=6) == 9 and fu(n_map=(1 << 28) + 1) == 9
    assert fu(m=-1) == 1 and fu(n_map=-1) == 1 and fu(ids=None) == 1 and fu(map_emb=None) == 1
    assert fu(emb=FAKE + 4) == 4 and fu(map_emb=FAKE + 8) == 4
    assert fu(m=0) == 0


def test_out_quality_pointer_alignment(lib):
    """dbar and area outputs must be 4-byte aligned."""
    t, mk, pj, _ = good()
    o = disc.Out(FAKE, 5, 768, None, None, FAKE + 2, None)
    assert lib.disc_embed_masks(ctypes.byref(t), ctypes.byref(mk), ctypes.byref(pj), ctypes.byref(o)) == 4
    o = disc.Out(FAKE, 5, 768, None, None, None, FAKE + 1)
    assert lib.disc_embed_masks(ctypes.byref(t), ctypes.byref(mk), ctypes.byref(pj), ctypes.byref(o)) == 4


def test_geometry_validation(lib):
    """The geometry entry points reject bad arguments on the host."""
    cam = disc.make_camera({"fx": 500.0, "fy": 500.0, "cx": 1.0, "cy": 1.0, "R": [[1, 0, 0], [0, 1, 0], [0, 0, 1]],
                            "t": [0, 0, 0], "depth_min": 0.1, "depth_max": 9.0})
    mk = disc.Masks(FAKE, 3, 48, 64)
    bc = lambda stride=1, c=cam, depth=FAKE, off=FAKE: lib.disc_backproject_count(  # noqa: E731
        depth, ctypes.byref(mk), ctypes.byref(c) if c is not None else None, stride, off, None)
    assert bc(stride=0) == 9 and bc(stride=65) == 9
    assert bc(c=None) == 1 and bc(depth=None) == 1 and bc(off=None) == 1
    zero = disc.make_camera({"fx": 0.0, "fy": 500.0, "cx": 1.0, "cy": 1.0, "R": [[1, 0, 0], [0, 1, 0], [0, 0, 1]],
                             "t": [0, 0, 0], "depth_min": 0.1, "depth_max": 9.0})
    assert bc(c=zero) == 1
    db = lambda m=2, n=100, eps=0.05, mp=5, keep=FAKE: lib.disc_dbscan_denoise(  # noqa: E731
        FAKE, FAKE, m, n, eps, mp, keep, None)
    assert db(m=70000) == 9 and db(n=(1 << 23) + 1) == 9 and db(m=-1) == 1
    assert db(eps=0.0) == 1 and db(eps=float("nan")) == 1 and db(mp=0) == 1 and db(keep=None) == 1
    assert db(n=0) == 0
    vx = lambda m=2, n=100, v=0.05, voff=FAKE: lib.disc_voxelize(  # noqa: E731
        FAKE, FAKE, None, m, n, v, voff, FAKE, None, None)
    assert vx(v=0.0) == 1 and vx(v=-1.0) == 1 and vx(voff=None) == 1 and vx(m=70000) == 9
    assert lib.disc_voxel_overlap(FAKE, FAKE, 1, FAKE, FAKE, 1, FAKE, -1, FAKE, None) == 1
    assert lib.disc_voxel_overlap(FAKE, FAKE, 1, FAKE, FAKE, 1, None, 3, FAKE, None) == 1
    assert lib.disc_voxel_overlap(FAKE, FAKE, 1, FAKE, FAKE, 1, FAKE, 0, FAKE, None) == 0


def test_noalloc_limits_before_device_work(lib):
    """The entry point that allocates nothing rejects a caller workspace and a
    frame whose workspace exceeds its scratch array on the host (a 1080p
    FP8 frame with 500 masks needs more than the array holds)."""
    t, m, p, o = good()
    opts = disc.make_options()
    opts.workspace = ctypes.c_void_p(FAKE)
    opts.workspace_bytes = 1 << 30
    rc = lib.disc_embed_masks_noalloc(ctypes.byref(t), ctypes.byref(m), ctypes.byref(p), ctypes.byref(o),
                                      ctypes.byref(opts), None)
    assert rc == disc.DISC_ERR_INVALID_ARGUMENT and b"workspace" in lib.disc_last_error()
    t = disc.Tokens(FAKE, disc.DISC_F8E4M3, 68, 120, 1280, 16, FAKE)
    m = disc.Masks(FAKE, 500, 1080, 1920)
    p = disc.Proj(FAKE, disc.DISC_BF16, 1280, 1024)
    o = disc.Out(FAKE, 500, 1024, None, None)
    need = lib.disc_workspace_bytes(ctypes.byref(t), ctypes.byref(m), 1, ctypes.byref(p), None)
    assert need > disc.NOALLOC_SCRATCH_BYTES
    rc = lib.disc_embed_masks_noalloc(ctypes.byref(t), ctypes.byref(m), ctypes.byref(p), ctypes.byref(o), None, None)
    assert rc == disc.DISC_ERR_LIMIT and b"scratch" in lib.disc_last_error()
