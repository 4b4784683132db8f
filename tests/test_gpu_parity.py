"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: squared EDT bit-exact; spatial weights and token statistics within a
relative 1e-5; embeddings per mask cos >= 1 - 1e-6 (FP32 path) and
cos >= 0.9995 (BF16 / FP8 paths); statuses identical.
"""
import numpy as np
import pytest

import disc_inputs as di
import oracle
from gpu_common import (COS_FP32, COS_LOWP, REL_S, check_embeddings, dev_bits, dev_proj, dev_tokens, frame_input,
                        oracle_frame, torch)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    t = torch()
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_03935_amd as disc

    disc.load()  # fails loudly when the library is missing
    return disc


def _edt_gpu(disc, bits, h, w):
    e = disc.edt_sq(dev_bits(bits), h, w)
    torch().cuda.synchronize()
    return e.cpu().numpy()


# ---------------------------------------------------------------- EDT

def test_edt_cfg1_cfg2(gpu):
    for name in ("cfg1", "cfg2"):
        fr = di.workload(name).frames[0]
        got = _edt_gpu(gpu, fr.bits, fr.h, fr.w)
        want = oracle.edt_sq(fr.bits, fr.w)
        bad = np.nonzero((got != want).reshape(len(got), -1).any(axis=1))[0]
        assert bad.size == 0, f"{name}: EDT differs on masks {bad[:10]}"


def adversarial_masks(h, w, rng):
    u = []
    z = lambda: np.zeros((h, w), dtype=np.uint8)
    a = z(); a[h // 2, :] = 1; u.append(a)                      # 1-px horizontal line across the frame
    a = z(); a[:, w // 3] = 1; u.append(a)                      # 1-px vertical line
    a = z(); idx = np.arange(min(h, w)); a[idx, idx] = 1; u.append(a)  # diagonal
    a = (np.indices((h, w)).sum(axis=0) % 2).astype(np.uint8); u.append(a)  # checkerboard
    u.append(np.ones((h, w), dtype=np.uint8))                     # full frame
    a = np.ones((h, w), dtype=np.uint8); a[rng.integers(0, h, 9), rng.integers(0, w, 9)] = 0; u.append(a)  # holes
    a = z(); a[0, :] = 1; a[-1, :] = 1; a[:, 0] = 1; a[:, -1] = 1; u.append(a)  # frame border
    a = z(); a[0, 0] = 1; a[h - 1, w - 1] = 1; a[h // 2, w // 2] = 1; u.append(a)  # single pixels
    a = z(); a[:, w - 3:] = 1; u.append(a)                      # right edge band
    u.append((rng.random((h, w)) < 0.97).astype(np.uint8))
    u.append((rng.random((h, w)) < 0.03).astype(np.uint8))
    a = z(); yy, xx = np.indices((h, w)); a[((yy - h / 2) ** 2 + (xx - w / 2) ** 2) < (min(h, w) / 2.2) ** 2] = 1; u.append(a)
    return np.stack(u)


@pytest.mark.parametrize("h,w", [(30, 100), (31, 130), (62, 64), (63, 63), (126, 200), (127, 129), (254, 70),
                                 (255, 65), (510, 90), (511, 77), (1150, 77), (5, 1500)])
def test_edt_adversarial(gpu, h, w):
    """Ragged widths, 1-px structures, full frames and every band-count class."""
    rng = np.random.default_rng(h * 1000 + w)
    u8 = adversarial_masks(h, w, rng)
    bits = di.pack_masks(u8)
    got = _edt_gpu(gpu, bits, h, w)
    want = oracle.edt_sq(bits, w)
    for i in range(len(u8)):
        assert np.array_equal(got[i], want[i]), f"{h}x{w} adversarial mask {i}: {np.argwhere(got[i] != want[i])[:5]}"


def test_edt_large_masks_1080p(gpu):
    bits = di.masks_mixed(77, 24, 1080, 1920, 0.02, 0.35)
    got = _edt_gpu(gpu, bits, 1080, 1920)
    want = oracle.edt_sq(bits, 1920)
    bad = np.nonzero((got != want).reshape(len(got), -1).any(axis=1))[0]
    assert bad.size == 0, f"1080p EDT differs on masks {bad}"


def test_edt_deep_tall_items(gpu):
    """Items taller than 512 rows whose interior lies more than 255 pixels
    from the outside (their 16-bit search is redone exactly): EDT bit-exact
    and the layouts agree bit for bit on the patch weights."""
    h, w = 1080, 1920
    yy, xx = np.indices((h, w))
    u8 = np.zeros((5, h, w), np.uint8)
    u8[0] = ((yy - 540) ** 2 + (xx - 960) ** 2) <= 520 ** 2
    u8[1] = 1
    u8[2, 10:1070, 100:1800] = 1
    u8[3] = ((yy - 540) / 530.0) ** 2 + ((xx - 700) / 300.0) ** 2 <= 1.0
    u8[4] = u8[0]
    u8[4, 540, :] = 0  # a cut through the middle: two halves of depth < 270
    bits = di.pack_masks(u8)
    got = _edt_gpu(gpu, bits, h, w)
    want = oracle.edt_sq(bits, w)
    for i in range(len(u8)):
        assert np.array_equal(got[i], want[i]), f"deep tall mask {i}: {np.argwhere(got[i] != want[i])[:5]}"
    assert want.max() > 255 ** 2
    b = dev_bits(bits)
    w0 = gpu.patch_weights(b, h, w, 16, distinct=0, edt_layout=0).cpu().numpy()
    w2 = gpu.patch_weights(b, h, w, 16, distinct=0, edt_layout=2).cpu().numpy()
    assert np.array_equal(w0, w2), "direct search disagrees with the band layout"


@pytest.mark.parametrize("P", [8, 10, 12, 14, 16, 20, 32, 64])
def test_edt_tall_patch_sizes(gpu, P):
    """Items taller than 512 rows (ellipses, a near-full box, a cut disc,
    random holes, thin columns with many runs per row) at patch sizes that
    leave 1 to 8 whole patches per strip: the direct search's patch weights
    equal the band layout's bit for bit and match the oracle, and its squared
    distances match the oracle."""
    h, w = 700, 400
    rng = np.random.default_rng(P)
    yy, xx = np.indices((h, w))
    u8 = np.zeros((6, h, w), np.uint8)
    u8[0] = ((yy - 350) / 340.0) ** 2 + ((xx - 200) / 190.0) ** 2 <= 1.0
    u8[1, 3:697, 5:390] = 1
    u8[2] = ((yy - 350) / 345.0) ** 2 + ((xx - 120) / 60.0) ** 2 <= 1.0
    u8[3] = rng.random((h, w)) < 0.97  # many short runs
    u8[3, :2] = 0
    u8[4] = ((yy - 350) ** 2 + (xx - 200) ** 2) <= 300 ** 2
    u8[4, 340:350, :] = 0
    u8[5, 1:699, 7:391:3] = 1  # thin columns: many runs per row
    bits = di.pack_masks(u8)
    b = dev_bits(bits)
    w0 = gpu.patch_weights(b, h, w, P, distinct=0, edt_layout=0).cpu().numpy()
    w2 = gpu.patch_weights(b, h, w, P, distinct=0, edt_layout=2).cpu().numpy()
    assert np.array_equal(w0, w2), f"P={P}: direct search disagrees with the band layout"
    s = oracle.spatial_weights(bits, w, P, 0)
    err = np.abs(w2.astype(np.float64) - s).max() / max(np.abs(s).max(), 1e-30)
    assert err < REL_S, err
    if P == 16:
        got = _edt_gpu(gpu, bits, h, w)
        want = oracle.edt_sq(bits, w)
        for i in range(len(u8)):
            assert np.array_equal(got[i], want[i]), f"tall mask {i}: {np.argwhere(got[i] != want[i])[:5]}"


@pytest.mark.parametrize("name,h,w,P", [("cfg2", 480, 640, 16), ("adv", 511, 200, 14), ("adv", 300, 130, 16),
                                        ("adv", 100, 90, 8), ("adv", 40, 333, 64)])
def test_edt_layouts_agree_bitwise(gpu, name, h, w, P):
    """Short-band, long-band and direct-search layouts of the distance
    transform give the same patch weights bit for bit (and match the oracle),
    across every class."""
    if name == "cfg2":
        bits = di.workload("cfg2").frames[0].bits
    else:
        bits = di.pack_masks(adversarial_masks(h, w, np.random.default_rng(h + w + P)))
    b = dev_bits(bits)
    w0 = gpu.patch_weights(b, h, w, P, distinct=0, edt_layout=0).cpu().numpy()
    w1 = gpu.patch_weights(b, h, w, P, distinct=0, edt_layout=1).cpu().numpy()
    w2 = gpu.patch_weights(b, h, w, P, distinct=0, edt_layout=2).cpu().numpy()
    assert np.array_equal(w0, w1), "band layouts disagree"
    assert np.array_equal(w0, w2), "direct search disagrees with the band layouts"
    s = oracle.spatial_weights(bits, w, P, 0)
    err = np.abs(w1.astype(np.float64) - s).max() / max(np.abs(s).max(), 1e-30)
    assert err < REL_S, err


# ---------------------------------------------------------------- weights and statistics

@pytest.mark.parametrize("spatial,distinct", [(0, 1), (0, 0), (1, 1), (1, 0)])
def test_patch_weights_modes(gpu, spatial, distinct):
    for name in ("cfg1", "cfg2"):
        fr = di.workload(name).frames[0]
        tok = fr.tokens
        data, scale = dev_tokens(tok)
        w = gpu.patch_weights(dev_bits(fr.bits), fr.h, fr.w, tok.patch, data, scale, spatial, distinct)
        got = w.cpu().numpy().astype(np.float64)
        s = oracle.spatial_weights(fr.bits, fr.w, tok.patch, spatial)
        if distinct:
            _, _, D = oracle.token_stats(oracle.decode_tokens(tok.data, tok.dtype, tok.scale), 1e-6)
            s = s * D[None, :]
        assert np.array_equal(got > 0, s > 0), f"{name}: weight support differs"
        err = np.abs(got - s).max() / max(np.abs(s).max(), 1e-30)
        assert err <= REL_S, f"{name} spatial={spatial} distinct={distinct}: rel err {err:.3e}"


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f8"])
def test_token_stats(gpu, dtype):
    for tok in (di.tokens_normal(5, 30, 40, 1024, dtype, 16), di.tokens_structured(6, 45, 80, 1280, dtype, 16)):
        data, scale = dev_tokens(tok)
        mean, r, D = gpu.token_stats(data, tok.patch, scale)
        f64 = oracle.decode_tokens(tok.data, tok.dtype, tok.scale)
        om, orr, oD = oracle.token_stats(f64, 1e-6)
        assert np.abs(mean.cpu().numpy() - om).max() <= REL_S * max(np.abs(f64).max(), 1.0)
        assert np.abs(r.cpu().numpy() - orr).max() <= REL_S * orr.max()
        assert np.abs(D.cpu().numpy() - oD).max() <= REL_S * oD.max()


def test_fp8_bad_scales(gpu):
    """A NaN, an infinite or a negative FP8 scale anywhere in a frame gives
    every mask of that frame status 3 and a zero row (with and without D);
    the other frames of the batch are untouched and match the oracle."""
    h, w, patch, C, E = 160, 200, 16, 256, 256
    gh, gw = -(-h // patch), -(-w // patch)
    tok = di.tokens_normal(81, gh, gw, C, "f8", patch)
    bits = di.masks_mixed(82, 6, h, w, 0.02, 0.3)
    P = di.projection(83, C, E, "bf16")
    frames = []
    for k, bad in enumerate([np.nan, np.inf, -0.5, None]):
        sc = tok.scale.copy()
        if bad is not None:
            sc[7 + 13 * k] = bad
        frames.append(di.Frame(di.Tokens(tok.data, "f8", sc, patch), bits, h, w))
    for distinct in (1, 0):
        outs = run_frames(gpu, frames, P, "bf16", options=gpu.make_options(distinct=distinct))
        for k in range(3):
            assert (outs[k].status.cpu().numpy() == 3).all(), f"frame {k}: status {outs[k].status.cpu().numpy()}"
            assert not outs[k].out.cpu().numpy().any(), f"frame {k}: rows must be zero"
        ref = oracle_frame(frames[3], P, "bf16", distinct=distinct)
        st = outs[3].status.cpu().numpy()
        assert np.array_equal(st, ref["status"])
        check_embeddings(outs[3].out.cpu().numpy(), st, ref, COS_LOWP, f"clean frame, distinct={distinct}")


def test_fp8_every_code(gpu):
    """Every finite e4m3fn code is decoded exactly: token p holds code p in
    every channel (scale 1, with two scaled tokens), so each token's residual
    norm sqrt(C) |v_p - mean| shows a wrong value of its code."""
    codes = np.array([c for c in range(256) if c & 0x7F != 0x7F], dtype=np.uint8)  # 254 finite codes
    G, C = 256, 64
    data = np.zeros((G, C), dtype=np.uint8)
    data[:codes.size] = codes[:, None]
    data[codes.size:] = np.array([0x38, 0xB8], dtype=np.uint8)[:, None]  # +1, -1
    scale = np.ones(G, dtype=np.float32)
    scale[codes.size:] = [0.5, 3.0]
    tok = di.Tokens(data.reshape(16, 16, C), "f8", scale, 16)
    d, sc = dev_tokens(tok)
    mean, r, D = gpu.token_stats(d, tok.patch, sc)
    f64 = oracle.decode_tokens(tok.data, tok.dtype, tok.scale)
    om, orr, oD = oracle.token_stats(f64, 1e-6)
    assert np.isfinite(f64).all()
    assert np.abs(mean.cpu().numpy() - om).max() <= REL_S * np.abs(f64).max()
    got_r = r.cpu().numpy().astype(np.float64)
    bad = np.nonzero(np.abs(got_r - orr) > 1e-5 * orr + 1e-7 * orr.max())[0]
    assert bad.size == 0, f"codes decoded wrongly: {[hex(int(data[i, 0])) for i in bad[:8]]}"


# ---------------------------------------------------------------- pooling / projection

@pytest.mark.parametrize("gemm", [0, 1])
def test_pool_project_given_weights(gpu, gemm):
    """One-hot weights return token rows, uniform weights the mean; vs oracle."""
    rng = np.random.default_rng(3)
    gh, gw, C, E, patch = 9, 11, 256, 384, 16
    G = gh * gw
    tok = di.tokens_normal(8, gh, gw, C, "f32", patch)
    P = di.projection(9, C, E, "f32")
    wts = np.zeros((70, G), dtype=np.float32)
    for i in range(G // 2):
        wts[i, 2 * i] = 1.0
    wts[50:60] = 1.0
    wts[60:69] = rng.random((9, G)).astype(np.float32) * (rng.random((9, G)) < 0.2)
    # row 69 stays zero -> status 1
    data, _ = dev_tokens(tok)
    res = gpu.pool_project(data, torch().from_numpy(wts).cuda(), dev_proj(P, "f32"), patch, gemm_dtype=gemm)
    f64 = oracle.decode_tokens(tok.data, "f32")
    ref = oracle.pool_project(f64, wts.astype(np.float64), P.astype(np.float64))
    pooled = res.pooled.cpu().numpy()
    if gemm == 0:
        assert np.allclose(pooled[:G // 2], f64[::2][:G // 2], rtol=0, atol=0), "one-hot weights must return the token row"
        assert np.allclose(pooled[:69], ref["pooled"][:69], rtol=1e-5, atol=1e-5)
    check_embeddings(res.out.cpu().numpy(), res.status.cpu().numpy(), ref, COS_FP32 if gemm == 0 else COS_LOWP, "given weights")


# ---------------------------------------------------------------- whole path

def run_frames(disc, frames, P, pdtype, pooled=False, options=None):
    ins = [frame_input(f) for f in frames]
    outs = disc.embed_frames(ins, dev_proj(P, pdtype), pooled=pooled, options=options)
    torch().cuda.synchronize()
    return outs


@pytest.mark.parametrize("name", ["cfg1", "cfg2"])
def test_embed_fp32_configs(gpu, name):
    wl = di.workload(name)
    fr = wl.frames[0]
    out = run_frames(gpu, [fr], wl.proj, wl.proj_dtype, pooled=True)[0]
    ref = oracle_frame(fr, wl.proj, wl.proj_dtype)
    c = check_embeddings(out.out.cpu().numpy(), out.status.cpu().numpy(), ref, COS_FP32, name)
    print(f"{name}: masks {len(c)} min cos {c.min():.10f} median {np.median(c):.10f}")
    pooled = out.pooled.cpu().numpy()
    ok = ref["status"] == 0
    rel = np.abs(pooled[ok] - ref["pooled"][ok]).max() / np.abs(ref["pooled"][ok]).max()
    assert rel < 1e-4, f"pooled features rel err {rel:.3e}"


@pytest.mark.parametrize("tdtype,pdtype", [("bf16", "bf16"), ("f8", "bf16"), ("f32", "bf16")])
@pytest.mark.parametrize("structured", [False, True])
def test_embed_lowp(gpu, tdtype, pdtype, structured):
    h, w, patch, C, E = 480, 640, 16, 1024, 768
    s = 4242 + structured
    tok = (di.tokens_structured(s, 30, 40, C, tdtype, patch) if structured else di.tokens_normal(s, 30, 40, C, tdtype, patch))
    fr = di.Frame(tok, di.masks_mixed(s, 96, h, w, 1e-3, 0.3), h, w)
    P = di.projection(s + 1, C, E, pdtype)
    out = run_frames(gpu, [fr], P, pdtype)[0]
    ref = oracle_frame(fr, P, pdtype)
    c = check_embeddings(out.out.cpu().numpy(), out.status.cpu().numpy(), ref, COS_LOWP, f"{tdtype}/{pdtype}")
    print(f"{tdtype} structured={structured}: min cos {c.min():.7f} median {np.median(c):.7f}")


def test_fp8_zero_tokens_pooled(gpu):
    """All-zero tokens (FP8 scale 0) inside masks: their weight still counts
    in Z, as in the FP64 definition, so the pooled features (not only the
    unit embeddings) match the oracle."""
    h, w, patch, C, E = 200, 264, 16, 256, 256
    gh, gw = -(-h // patch), -(-w // patch)
    vals = di.tokens_structured(77, gh, gw, C, "f64", patch).data.reshape(gh * gw, C).copy()
    zero = [r * gw + c for r in range(3, 8) for c in range(4, 10)]
    vals[zero] = 0.0
    tok = di.tokens_from_values(vals.reshape(gh, gw, C), "f8", patch)
    # a zero scale makes the token exactly zero whatever its codes
    tok.scale[zero] = 0.0
    tok.data.reshape(gh * gw, C)[zero] = np.random.default_rng(5).integers(0, 126, (len(zero), C), dtype=np.uint8)
    u8 = np.zeros((4, h, w), np.uint8)
    u8[0, 40:130, 50:170] = 1                      # covers the zero block and more
    u8[1, 48:128, 64:160] = 1                      # inside the zero block
    u8[2, 20:190, 20:250] = 1                      # a large box around it
    u8[3] = di.unpack_masks(di.masks_mixed(78, 1, h, w, 0.05, 0.2), w)[0]
    fr = di.Frame(tok, di.pack_masks(u8), h, w)
    P = di.projection(79, C, E, "bf16")
    out = run_frames(gpu, [fr], P, "bf16", pooled=True)[0]
    ref = oracle_frame(fr, P, "bf16")
    st = out.status.cpu().numpy()
    assert np.array_equal(st, ref["status"])
    ok = ref["status"] == 0
    pooled = out.pooled.cpu().numpy().astype(np.float64)
    rel = np.abs(pooled[ok] - ref["pooled"][ok]).max() / np.abs(ref["pooled"][ok]).max()
    assert rel < 5e-3, f"pooled features with zero tokens: rel err {rel:.3e}"
    check_embeddings(out.out.cpu().numpy(), st, ref, COS_LOWP, "fp8 zero tokens")


def test_embed_modes_fp32(gpu):
    wl = di.workload("cfg2")
    fr = wl.frames[0]
    for spatial in (0, 1):
        for distinct in (0, 1):
            opts = gpu.make_options(spatial, distinct)
            out = run_frames(gpu, [fr], wl.proj, wl.proj_dtype, options=opts)[0]
            ref = oracle_frame(fr, wl.proj, wl.proj_dtype, spatial, distinct)
            check_embeddings(out.out.cpu().numpy(), out.status.cpu().numpy(), ref, COS_FP32, f"mode {spatial}/{distinct}")


def test_ragged_batch_and_batch_invariance(gpu):
    """Mixed resolutions in one call; every frame's result equals the frame
    alone, bit for bit, and the oracle within tolerance."""
    frames = []
    for i, (h, w, m) in enumerate([(480, 640, 40), (720, 1280, 65), (480, 640, 1), (720, 1280, 90), (336, 336, 8)]):
        patch = 14 if h == 336 else 16
        gh, gw = -(-h // patch), -(-w // patch)
        frames.append(di.Frame(di.tokens_normal(100 + i, gh, gw, 1024, "bf16", patch),
                               di.masks_mixed(100 + i, m, h, w, 1e-3, 0.3), h, w))
    P = di.projection(7, 1024, 768, "bf16")
    mix = run_frames(gpu, frames, P, "bf16")
    for i, fr in enumerate(frames):
        alone = run_frames(gpu, [fr], P, "bf16")[0]
        a, b = alone.out.cpu().numpy(), mix[i].out.cpu().numpy()
        assert np.array_equal(a, b), f"frame {i}: result in the batch differs from the frame alone"
        ref = oracle_frame(fr, P, "bf16")
        check_embeddings(b, mix[i].status.cpu().numpy(), ref, COS_LOWP, f"ragged frame {i}")


def test_degenerate_cases(gpu):
    h, w, patch, C, E = 64, 96, 16, 128, 128
    u8 = np.zeros((4, h, w), dtype=np.uint8)
    u8[1, 10:40, 20:70] = 1
    u8[2, :, :] = 1
    u8[3, 5, 5] = 1
    bits = di.pack_masks(u8)
    tok = di.tokens_normal(1, 4, 6, C, "f32", patch)
    P = di.projection(2, C, E, "f32")
    fr = di.Frame(tok, bits, h, w)
    out = run_frames(gpu, [fr], P, "f32")[0]
    check_embeddings(out.out.cpu().numpy(), out.status.cpu().numpy(), oracle_frame(fr, P, "f32"), COS_FP32, "empty mask")
    # constant token map: D == 0 everywhere -> spatial weights
    const = di.tokens_from_values(np.tile(np.random.default_rng(0).normal(size=C), (4, 6, 1)), "f32", patch)
    frc = di.Frame(const, bits, h, w)
    outc = run_frames(gpu, [frc], P, "f32", pooled=True)[0]
    refc = oracle_frame(frc, P, "f32")
    check_embeddings(outc.out.cpu().numpy(), outc.status.cpu().numpy(), refc, COS_FP32, "constant map")
    # zero projection -> status 2
    outz = run_frames(gpu, [fr], np.zeros((C, E), dtype=np.float32), "f32")[0]
    st = outz.status.cpu().numpy()
    assert list(st) == [1, 2, 2, 2] and not outz.out.cpu().numpy().any()
    # no masks
    fr0 = di.Frame(tok, bits[:0], h, w)
    out0 = run_frames(gpu, [fr0], P, "f32")[0]
    assert out0.out.shape == (0, E)


def test_pack_masks(gpu):
    rng = np.random.default_rng(11)
    u8 = (rng.random((5, 37, 130)) < 0.4).astype(np.uint8)
    bits = gpu.pack_masks(torch().from_numpy(u8).cuda())
    assert np.array_equal(bits.cpu().numpy().view(np.uint64), di.pack_masks(u8))


# ---------------------------------------------------------------- full-size workloads (sampled)

def test_cfg3_full_batch_sampled(gpu):
    """64-frame BF16 batch in one call, one sampled mask per frame vs oracle."""
    wl = di.workload("cfg3")
    outs = run_frames(gpu, wl.frames, wl.proj, "bf16")
    rng = np.random.default_rng(5)
    cs = []
    for i, fr in enumerate(wl.frames):
        j = int(rng.integers(0, fr.m))
        ref = oracle_frame(fr, wl.proj, "bf16", idx=[j])
        got = outs[i].out[j:j + 1].cpu().numpy()
        cs.append(check_embeddings(got, outs[i].status[j:j + 1].cpu().numpy(), ref, COS_LOWP, f"cfg3 frame {i}"))
    c = np.concatenate(cs)
    print(f"cfg3 sampled {len(c)}: min cos {c.min():.7f}")


def test_cfg5_full_batch_sampled(gpu):
    """16 frames 1080x1920, FP8 tokens, 500 masks each: sampled masks vs oracle."""
    wl = di.workload("cfg5")
    outs = run_frames(gpu, wl.frames, wl.proj, "bf16")
    rng = np.random.default_rng(6)
    cs = []
    for i, fr in enumerate(wl.frames):
        idx = sorted(rng.choice(fr.m, size=2, replace=False).tolist())
        ref = oracle_frame(fr, wl.proj, "bf16", idx=idx)
        got = outs[i].out[idx].cpu().numpy()
        cs.append(check_embeddings(got, outs[i].status[idx].cpu().numpy(), ref, COS_LOWP, f"cfg5 frame {i}"))
    c = np.concatenate(cs)
    print(f"cfg5 sampled {len(c)}: min cos {c.min():.7f}")


@pytest.mark.parametrize("name,frames", [("cfg2", None), ("cfg3", 6), ("cfg5", 2)])
def test_pool_tile_widths_agree_bitwise(gpu, name, frames):
    """Every pooling tile shape the autotuner searches (1, 2, 4 x 64 channels
    and 64 or 128 masks per workgroup) and the tuned choice give the same
    pooled features and embeddings, bit for bit."""
    wl = di.workload(name, frames=frames)
    ins = [frame_input(f) for f in wl.frames]
    proj = dev_proj(wl.proj, wl.proj_dtype)
    res = {}
    shapes = [(-1, -1), (1, 64), (2, 64), (4, 64), (1, 128), (2, 128)]
    for nt, rows in shapes:
        outs = gpu.embed_frames(ins, proj, pooled=True, options=gpu.make_options(pool_tile=nt, pool_rows=rows))
        res[(nt, rows)] = [(o.out.cpu().numpy(), o.pooled.cpu().numpy()) for o in outs]
    for key in shapes[1:]:
        for i, ((a, pa), (b, pb)) in enumerate(zip(res[shapes[0]], res[key])):
            assert np.array_equal(pa, pb), f"{name}: pooled features of shape {key} differ from the tuned one on frame {i}"
            assert np.array_equal(a, b), f"{name}: embeddings of shape {key} differ from the tuned one on frame {i}"


def test_mask_order_and_subset_invariance(gpu):
    """A mask's embedding does not depend on the other masks of its frame:
    a 500-mask 1080p frame, the same masks reversed, and subsets above and
    below the size at which the pooling order moves the largest boxes to the
    front give each mask the same pooled features and embedding, bit for bit."""
    wl = di.workload("cfg5", frames=1)
    fr = wl.frames[0]
    proj = dev_proj(wl.proj, wl.proj_dtype)
    m = fr.m
    orders = {"all": np.arange(m), "reversed": np.arange(m)[::-1].copy(),
              "300": np.random.default_rng(3).permutation(m)[:300], "200": np.arange(0, m, 2)[:200]}
    res = {}
    for name, idx in orders.items():
        sub = di.Frame(fr.tokens, np.ascontiguousarray(fr.bits[idx]), fr.h, fr.w)
        o = gpu.embed_frames([frame_input(sub)], proj, pooled=True)[0]
        res[name] = (idx, o.out.cpu().numpy(), o.pooled.cpu().numpy())
    _, full, fullp = res["all"]
    for name, (idx, out, pooled) in res.items():
        assert np.array_equal(pooled, fullp[idx]), f"pooled features of the {name} masks differ from the full frame"
        assert np.array_equal(out, full[idx]), f"embeddings of the {name} masks differ from the full frame"


@pytest.mark.parametrize("name,frames", [("cfg2", None), ("cfg3", 3)])
def test_embed_edt_layouts_agree_bitwise(gpu, name, frames):
    """Whole calls with every distance-transform layout give the same pooled
    features and embeddings, bit for bit.  Small batches split the token
    statistics over other launches (channel sums with the mask scan; the
    frame means with the direct search's patch sums, or in their own launch
    after the band layouts, which then also pack P for a BF16 projection), so
    this also checks that every such arrangement computes the same r."""
    wl = di.workload(name, frames=frames)
    ins = [frame_input(f) for f in wl.frames]
    proj = dev_proj(wl.proj, wl.proj_dtype)
    res = {}
    for lay in (-1, 0, 1, 2):
        outs = gpu.embed_frames(ins, proj, pooled=True, options=gpu.make_options(edt_layout=lay))
        res[lay] = [(o.out.cpu().numpy(), o.pooled.cpu().numpy()) for o in outs]
    for lay in (0, 1, 2):
        for i, ((a, pa), (b, pb)) in enumerate(zip(res[-1], res[lay])):
            assert np.array_equal(pa, pb), f"{name} frame {i}: pooled features with layout {lay} differ"
            assert np.array_equal(a, b), f"{name} frame {i}: embeddings with layout {lay} differ"


def test_projection_split_invariance(gpu):
    """The BF16 projection runs whole-K tiles on a full cfg3 batch (and on the
    cfg3 frames taken twice) and split-K tiles (group sums added in group
    order) on a few of its frames: the same frames get the same bits every
    way."""
    wl = di.workload("cfg3")
    ins = [frame_input(f) for f in wl.frames]
    proj = dev_proj(wl.proj, wl.proj_dtype)
    full = gpu.embed_frames(ins, proj)
    few = gpu.embed_frames(ins[:3], proj)
    m = sum(o.out.shape[0] for o in full)
    assert -(-m // 64) * (768 // 64) >= 256, "the full batch must take the whole-K path"
    big = gpu.embed_frames(ins + ins, proj)
    for i in range(3):
        a = full[i].out.cpu().numpy()
        assert np.array_equal(a, few[i].out.cpu().numpy()), f"frame {i}: split-K result differs"
        assert np.array_equal(a, big[i].out.cpu().numpy()), f"frame {i}: result in the doubled batch differs"
        assert np.array_equal(a, big[len(ins) + i].out.cpu().numpy()), f"frame {i}: second copy differs"


# ---------------------------------------------------------------- open-vocabulary query

def _check_topk(scores, idx, ref, tol, what):
    """Scores within tol of the oracle's; indices identical where the oracle's
    consecutive scores are separated by more than 2 tol, otherwise any index
    whose oracle similarity is within tol of the oracle's score at that rank."""
    q, k = ref["idx"].shape
    for j in range(q):
        assert np.allclose(scores[j], ref["scores"][j], rtol=0, atol=tol), f"{what}: scores of query {j}"
        for r in range(k):
            want = ref["idx"][j, r]
            if want < 0:
                assert idx[j, r] == -1
                continue
            s = ref["scores"][j]
            gap_ok = (r == 0 or s[r - 1] - s[r] > 2 * tol) and (r == k - 1 or s[r] - s[r + 1] > 2 * tol)
            if gap_ok:
                assert idx[j, r] == want, f"{what}: query {j} rank {r}: {idx[j, r]} vs {want}"
            else:
                assert abs(ref["sim"][j, idx[j, r]] - s[r]) <= tol, f"{what}: query {j} rank {r} near-tie invalid"
        assert len(set(idx[j][idx[j] >= 0].tolist())) == int((idx[j] >= 0).sum()), "an instance listed twice"


@pytest.mark.parametrize("tdt", ["f32", "bf16"])
def test_query_topk_vs_oracle(gpu, tdt):
    t = torch()
    rng = np.random.default_rng(41)
    m, e, q, k = 3001, 768, 37, 10
    emb = rng.standard_normal((m, e)).astype(np.float32)
    emb[7] = 0.0
    emb[100:110] = emb[99]  # exact ties: lower index first
    text = rng.standard_normal((q, e)).astype(np.float32)
    text[3] = emb[100] * 2.0  # best match: the tied group, in index order
    if tdt == "bf16":
        tq, _ = di.quantize(text.astype(np.float64), "bf16")
        text_dev = t.from_numpy(tq.view(np.int16)).cuda().view(t.bfloat16)
        text_ref = oracle.decode_tokens(tq.reshape(1, q, e), "bf16").reshape(q, e)
    else:
        text_dev = t.from_numpy(text).cuda()
        text_ref = text.astype(np.float64)
    scores, idx, sim = gpu.query_topk(t.from_numpy(emb).cuda(), text_dev, k)
    ref = oracle.query_topk(emb.astype(np.float64), text_ref, k)
    tol = 2e-6
    assert np.abs(sim.cpu().numpy() - ref["sim"]).max() <= tol
    _check_topk(scores.cpu().numpy(), idx.cpu().numpy(), ref, tol, tdt)
    assert idx.cpu().numpy()[3].tolist() == list(range(99, 109)), "identical instances rank by index"


def test_query_topk_on_embeddings(gpu):
    """The query over the embeddings of a frame, k larger than m (padding)."""
    t = torch()
    fr = di.workload("cfg1").frames[0]
    P = di.workload("cfg1").proj
    out = gpu.embed_frames([frame_input(fr)], dev_proj(P, "f32"))[0].out
    rng = np.random.default_rng(43)
    text = rng.standard_normal((5, 768)).astype(np.float32)
    scores, idx, sim = gpu.query_topk(out, t.from_numpy(text).cuda(), 12)
    ref = oracle.query_topk(out.cpu().numpy().astype(np.float64), text.astype(np.float64), 12)
    _check_topk(scores.cpu().numpy(), idx.cpu().numpy(), ref, 2e-6, "cfg1 embeddings")
    assert (idx.cpu().numpy()[:, 8:] == -1).all() and np.isinf(scores.cpu().numpy()[:, 8:]).all()


def test_object_scene_modes_vs_oracle(gpu):
    """The synthetic object scene (overlapping objects, outline patches that
    mix features, outlier tokens) through every weighting mode."""
    from disc_inputs.scene import object_scene

    sc = object_scene(di.frame_seed(8, 0))
    P = di.projection(di.frame_seed(8, 1), 1024, 768, "f32")
    for spatial, distinct in [(0, 1), (0, 0), (1, 1), (1, 0)]:
        out = run_frames(gpu, [sc.frame], P, "f32", options=gpu.make_options(spatial, distinct))[0]
        ref = oracle_frame(sc.frame, P, "f32", spatial, distinct)
        check_embeddings(out.out.cpu().numpy(), out.status.cpu().numpy(), ref, COS_FP32, f"scene {spatial}/{distinct}")


def test_edt_max_width(gpu):
    """The widest frame accepted (8448 columns = 256 strips): masks spanning
    many strips, a full-width band and blobs cut by strip edges."""
    h, w = 40, 8448
    rng = np.random.default_rng(8448)
    u8 = np.zeros((4, h, w), np.uint8)
    u8[0, 5:30, :] = 1
    u8[1, :, 100:8400] = 1
    u8[1, 20, 4000:4100] = 0
    u8[2] = rng.random((h, w)) < 0.6
    yy, xx = np.indices((h, w))
    u8[3] = ((yy - 20) / 18.0) ** 2 + ((xx - 6000) / 2400.0) ** 2 <= 1.0
    bits = di.pack_masks(u8)
    got = _edt_gpu(gpu, bits, h, w)
    want = oracle.edt_sq(bits, w)
    for i in range(4):
        assert np.array_equal(got[i], want[i]), f"max-width mask {i}"


@pytest.mark.parametrize("patch,C,E", [(8, 128, 128), (64, 256, 256), (16, 2048, 1024)])
def test_embed_extreme_shapes(gpu, patch, C, E):
    """Smallest and largest patch sizes, and the largest channel count and
    embedding width, FP32 path."""
    h, w = 200, 264
    gh, gw = -(-h // patch), -(-w // patch)
    fr = di.Frame(di.tokens_normal(patch + C, gh, gw, C, "f32", patch),
                  di.masks_mixed(patch + E, 24, h, w, 1e-3, 0.4), h, w)
    P = di.projection(patch, C, E, "f32")
    out = run_frames(gpu, [fr], P, "f32")[0]
    check_embeddings(out.out.cpu().numpy(), out.status.cpu().numpy(), oracle_frame(fr, P, "f32"), COS_FP32,
                     f"patch {patch} C {C} E {E}")
