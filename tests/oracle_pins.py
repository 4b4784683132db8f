"""Pins that fix the oracle to something other than itself.

Every check takes an ``oracle.Oracle`` instance and raises AssertionError when
the oracle disagrees with what the paper and the mathematics fix: brute force
on tiny inputs, closed forms, a library routine for a special case, and
invariants.  ``test_oracle_pins.py`` runs them on the oracle;
``test_oracle_mutants.py`` runs them on deliberately broken copies of the
oracle and expects each copy to fail at least one of them.
"""
from __future__ import annotations

import numpy as np

import disc_inputs as di

# ----------------------------------------------------------------------------
# helpers (none of them calls the oracle)
# ----------------------------------------------------------------------------


def brute_edt(u8: np.ndarray) -> np.ndarray:
    """Squared distance from each mask pixel to the nearest non-mask pixel of
    the integer plane (pixels outside the frame are not in the mask), by
    enumerating every candidate.  u8: [m][h][w]; returns int64 [m][h][w]."""
    u8 = np.asarray(u8).astype(bool)
    m, h, w = u8.shape
    ys, xs = np.mgrid[0:h, 0:w]
    py, px = ys.ravel(), xs.ravel()
    d2 = (py[:, None] - py[None, :]) ** 2 + (px[:, None] - px[None, :]) ** 2
    # nearest pixel outside the frame: straight up, down, left or right
    border = np.minimum.reduce([py + 1, h - py, px + 1, w - px]).astype(np.int64) ** 2
    flat = u8.reshape(m, -1)
    out = np.empty((m, h * w), dtype=np.int64)
    n = h * w
    chunk = max(1, (1 << 22) // (n * n))
    big = np.iinfo(np.int64).max
    for i in range(0, m, chunk):
        M = flat[i:i + chunk]
        cand = np.where(~M[:, None, :], d2[None], big)
        best = np.minimum(cand.min(axis=2), border[None])
        out[i:i + chunk] = np.where(M, best, 0)
    return out.reshape(m, h, w)


def all_masks(h: int, w: int) -> np.ndarray:
    n = h * w
    k = np.arange(1 << n, dtype=np.int64)
    bits = (k[:, None] >> np.arange(n)[None, :]) & 1
    return bits.reshape(-1, h, w).astype(np.uint8)


def rect_mask(h, w, y0, y1, x0, x1):
    u = np.zeros((h, w), dtype=np.uint8)
    u[y0:y1 + 1, x0:x1 + 1] = 1
    return u


def rect_edt(h, w, y0, y1, x0, x1):
    """Closed form for a filled axis-aligned rectangle [y0,y1]x[x0,x1]."""
    e = np.zeros((h, w), dtype=np.int64)
    ys, xs = np.mgrid[y0:y1 + 1, x0:x1 + 1]
    d = np.minimum.reduce([ys - y0 + 1, y1 + 1 - ys, xs - x0 + 1, x1 + 1 - xs])
    e[y0:y1 + 1, x0:x1 + 1] = d * d
    return e


def block_sum(img: np.ndarray, patch: int) -> np.ndarray:
    """Sum of a [h][w] image over patch x patch blocks (partial blocks at the
    bottom/right), flattened patch-row-major."""
    h, w = img.shape
    gh, gw = -(-h // patch), -(-w // patch)
    pad = np.zeros((gh * patch, gw * patch), dtype=np.float64)
    pad[:h, :w] = img
    return pad.reshape(gh, patch, gw, patch).sum(axis=(1, 3)).ravel()


def random_masks(rng, m, h, w, density):
    return (rng.random((m, h, w)) < density).astype(np.uint8)


# ----------------------------------------------------------------------------
# P1: the distance transform
# ----------------------------------------------------------------------------


def pin_edt_exhaustive(orc, h, w):
    u8 = all_masks(h, w)
    got = orc.edt_sq(di.pack_masks(u8), w)
    want = brute_edt(u8)
    bad = np.nonzero((got != want).reshape(len(u8), -1).any(axis=1))[0]
    assert bad.size == 0, f"EDT differs from brute force on {bad.size} of {len(u8)} {h}x{w} masks (first {bad[:5]})"


def pin_edt_random_bruteforce(orc, seed=1, cases=((7, 9), (16, 16), (32, 32), (13, 31), (1, 17), (19, 1))):
    rng = np.random.default_rng(seed)
    for (h, w) in cases:
        for density in (0.05, 0.3, 0.6, 0.85, 0.95):
            u8 = random_masks(rng, 6, h, w, density)
            got = orc.edt_sq(di.pack_masks(u8), w)
            want = brute_edt(u8)
            assert np.array_equal(got, want), f"EDT differs from brute force ({h}x{w}, density {density})"


def pin_edt_scipy(orc, seed=2):
    from scipy import ndimage

    rng = np.random.default_rng(seed)
    cases = [random_masks(rng, 3, 64, 96, d) for d in (0.2, 0.7, 0.97)]
    cases.append(di.unpack_masks(di.masks_ellipses(7, 4, 120, 150, 10, 80), 150))
    cases.append(di.unpack_masks(di.masks_mixed(8, 4, 96, 200, 1e-2, 0.4), 200))
    for u8 in cases:
        m, h, w = u8.shape
        got = orc.edt_sq(di.pack_masks(u8), w)
        for i in range(m):
            padded = np.zeros((h + 2, w + 2), dtype=np.uint8)
            padded[1:-1, 1:-1] = u8[i]
            d = ndimage.distance_transform_edt(padded)[1:-1, 1:-1]
            want = np.rint(d * d).astype(np.int64)
            assert np.array_equal(got[i], want), "EDT differs from scipy.ndimage.distance_transform_edt"


def pin_edt_rectangles(orc):
    h, w = 23, 70
    rects = [(0, h - 1, 0, w - 1), (0, 0, 0, 0), (5, 5, 3, 60), (2, 20, 7, 7), (0, 10, 0, 33),
             (12, h - 1, 40, w - 1), (3, 17, 64, 69), (1, 21, 1, 68), (4, 9, 62, 66)]
    u8 = np.stack([rect_mask(h, w, *r) for r in rects])
    got = orc.edt_sq(di.pack_masks(u8), w)
    for i, r in enumerate(rects):
        assert np.array_equal(got[i], rect_edt(h, w, *r)), f"EDT of rectangle {r} breaks the closed form"


def pin_edt_symmetry(orc, seed=3):
    rng = np.random.default_rng(seed)
    u8 = random_masks(rng, 4, 21, 37, 0.75)
    e = orc.edt_sq(di.pack_masks(u8), 37)
    eT = orc.edt_sq(di.pack_masks(np.ascontiguousarray(u8.transpose(0, 2, 1))), 21)
    assert np.array_equal(eT, e.transpose(0, 2, 1)), "EDT is not transpose-equivariant"
    eF = orc.edt_sq(di.pack_masks(np.ascontiguousarray(u8[:, ::-1, ::-1])), 37)
    assert np.array_equal(eF, e[:, ::-1, ::-1]), "EDT is not flip-equivariant"
    single = np.zeros((1, 9, 9), dtype=np.uint8)
    single[0, 4, 4] = 1
    es = orc.edt_sq(di.pack_masks(single), 9)
    assert es[0, 4, 4] == 1 and es.sum() == 1, "single pixel must have squared distance 1"
    assert ((e >= 1) == (u8 == 1)).all(), "EDT must be >= 1 exactly on the mask"


def pin_edt_bbox_locality(orc, seed=4):
    """A mask away from the frame border has the same EDT in any larger frame."""
    rng = np.random.default_rng(seed)
    small = random_masks(rng, 1, 15, 20, 0.8)[0]
    e_ref = None
    for (H, W, oy, ox) in ((17, 22, 1, 1), (40, 150, 10, 70), (33, 129, 5, 64)):
        big = np.zeros((1, H, W), dtype=np.uint8)
        big[0, oy:oy + 15, ox:ox + 20] = small
        e = orc.edt_sq(di.pack_masks(big), W)[0]
        crop = e[oy:oy + 15, ox:ox + 20]
        assert e.sum() == crop.sum()
        if e_ref is None:
            e_ref = crop
        assert np.array_equal(crop, e_ref), "EDT depends on where the mask sits in the frame"


# ----------------------------------------------------------------------------
# P2: per-patch spatial weights
# ----------------------------------------------------------------------------


def pin_spatial_blocksum(orc, seed=5):
    rng = np.random.default_rng(seed)
    for (h, w, patch) in ((30, 33, 7), (16, 16, 4), (27, 40, 14), (9, 70, 5)):
        u8 = random_masks(rng, 3, h, w, 0.7)
        bits = di.pack_masks(u8)
        e = brute_edt(u8)
        s_edt = orc.spatial_weights(bits, w, patch, 0)
        s_area = orc.spatial_weights(bits, w, patch, 1)
        for i in range(3):
            want = block_sum(np.sqrt(e[i].astype(np.float64)), patch)
            assert np.allclose(s_edt[i], want, rtol=1e-13, atol=1e-12), "EDT patch weights != block sums of sqrt(EDT)"
            cnt = block_sum(u8[i].astype(np.float64), patch)
            assert np.array_equal(s_area[i], cnt), "AREA patch weights != pixel counts per patch"
            assert s_area[i].sum() == u8[i].sum()
            assert np.array_equal(s_edt[i] > 0, cnt > 0), "support must be exactly the touched patches"


def pin_spatial_rectangle(orc):
    h, w, patch = 48, 64, 16
    rects = [(16, 47, 0, 31), (0, 15, 16, 63), (5, 40, 9, 50)]
    u8 = np.stack([rect_mask(h, w, *r) for r in rects])
    s = orc.spatial_weights(di.pack_masks(u8), w, patch, 0)
    for i, r in enumerate(rects):
        want = block_sum(np.sqrt(rect_edt(h, w, *r).astype(np.float64)), patch)
        assert np.allclose(s[i], want, rtol=1e-13, atol=1e-12), f"patch weights of rectangle {r} break the closed form"


# ----------------------------------------------------------------------------
# P3: distinctiveness (Eq. 1)
# ----------------------------------------------------------------------------


def pin_token_two_valued(orc, seed=6):
    rng = np.random.default_rng(seed)
    G, C, k = 37, 11, 9
    u, v = rng.normal(size=C), rng.normal(size=C)
    f = np.tile(v, (G, 1))
    idx = rng.choice(G, size=k, replace=False)
    f[idx] = u
    eps = 1e-6
    mean, r, D = orc.token_stats(f, eps)
    duv = np.sqrt(((u - v) ** 2).sum())
    r_u, r_v = (G - k) / G * duv, k / G * duv
    want_r = np.full(G, r_v)
    want_r[idx] = r_u
    assert np.allclose(mean, (k * u + (G - k) * v) / G, rtol=1e-13, atol=1e-13), "mean of a two-valued map"
    assert np.allclose(r, want_r, rtol=1e-12), "residual norms of a two-valued map break the closed form"
    rbar = (k * r_u + (G - k) * r_v) / G
    assert np.allclose(D, want_r / (rbar + eps), rtol=1e-12), "D of a two-valued map breaks Eq. (1)"


def pin_token_invariances(orc, seed=7):
    rng = np.random.default_rng(seed)
    G, C = 50, 16
    f = rng.normal(size=(G, C)) * rng.uniform(0.2, 3, size=(G, 1))
    _, r, D = orc.token_stats(f, 0.0)
    _, r2, D2 = orc.token_stats(f + rng.normal(size=C)[None, :], 0.0)
    assert np.allclose(r2, r, rtol=1e-10) and np.allclose(D2, D, rtol=1e-10), "D must not change under a common shift"
    _, r3, D3 = orc.token_stats(3.5 * f, 0.0)
    assert np.allclose(r3, 3.5 * r, rtol=1e-12) and np.allclose(D3, D, rtol=1e-12), "r must scale linearly"
    eps = 1e-3
    _, r4, D4 = orc.token_stats(f, eps)
    rbar = r4.mean()
    assert np.isclose(D4.sum(), G * rbar / (rbar + eps), rtol=1e-12), "sum of D must equal G rbar/(rbar+eps)"


# ----------------------------------------------------------------------------
# P4 / P5: pooled feature and output
# ----------------------------------------------------------------------------


def pin_pool_constant_on_support(orc, seed=8):
    """A token map that is constant on a mask's patches pools to that constant,
    with D on and off, whatever the rest of the map holds."""
    rng = np.random.default_rng(seed)
    h, w, patch = 64, 80, 16
    gh, gw = 4, 5
    C, E = 12, 9
    u8 = np.zeros((2, h, w), dtype=np.uint8)
    u8[0, 20:45, 18:60] = 1
    u8[1] = di.unpack_masks(di.masks_ellipses(11, 1, h, w, 8, 20), w)[0]
    bits = di.pack_masks(u8)
    P = rng.normal(size=(C, E))
    for i in range(2):
        f = rng.normal(size=(gh * gw, C))
        touched = block_sum(u8[i].astype(float), patch) > 0
        const = rng.normal(size=C)
        f[touched] = const
        for distinct in (0, 1):
            res = orc.embed(f, gh, gw, patch, bits[i:i + 1], w, P, 0, distinct)
            assert np.allclose(res["pooled"][0], const, rtol=1e-12, atol=1e-12), "constant-on-support map must pool to the constant"


def pin_pool_single_patch(orc, seed=9):
    rng = np.random.default_rng(seed)
    h, w, patch, C, E = 32, 48, 16, 10, 6
    u8 = np.zeros((1, h, w), dtype=np.uint8)
    u8[0, 18:29, 34:46] = 1  # inside patch (1, 2)
    f = rng.normal(size=(6, C))
    P = rng.normal(size=(C, E))
    for distinct in (0, 1):
        res = orc.embed(f, 2, 3, patch, di.pack_masks(u8), w, P, 0, distinct)
        assert np.allclose(res["pooled"][0], f[1 * 3 + 2], rtol=1e-13, atol=1e-13), "single-patch mask must give that patch's token"


def pin_pool_uniform_mean(orc, seed=10):
    rng = np.random.default_rng(seed)
    G, C, E = 20, 7, 5
    f = rng.normal(size=(G, C))
    P = rng.normal(size=(C, E))
    wts = np.zeros((3, G))
    sel = [np.arange(G), np.array([0, 3, 4, 19]), np.array([7])]
    for i, s in enumerate(sel):
        wts[i, s] = 2.5
    res = orc.pool_project(f, wts, P)
    for i, s in enumerate(sel):
        assert np.allclose(res["pooled"][i], f[s].sum(axis=0) / len(s), rtol=1e-13, atol=1e-13), "uniform weights must give the mean"


def pin_pool_zero_weight_row(orc, seed=14):
    """Given weights (the stage entry point): an all-zero weight row has no
    weighted mean (Sec. III-C divides by the weight sum), so it gives a zero
    output row, status 1 (empty) and a zero pooled row; the rows around it keep
    their own weighted means, normalised projections and status 0."""
    rng = np.random.default_rng(seed)
    G, C, E = 12, 5, 4
    f = rng.normal(size=(G, C))
    P = rng.normal(size=(C, E))
    wts = rng.uniform(0.5, 2.0, size=(3, G))
    wts[1] = 0.0
    res = orc.pool_project(f, wts, P)
    assert res["status"].tolist() == [0, 1, 0], "a zero weight row is status 1, the others 0"
    assert not res["out"][1].any() and not res["pooled"][1].any(), "a zero weight row gives zero rows"
    for i in (0, 2):
        F = (wts[i][:, None] * f).sum(axis=0) / wts[i].sum()
        assert np.allclose(res["pooled"][i], F, rtol=1e-13, atol=1e-13), "neighbouring rows keep their weighted mean"
        y = F @ P
        assert np.allclose(res["out"][i], y / np.sqrt((y * y).sum()), rtol=1e-12, atol=1e-13)


def pin_eps_cancels(orc, seed=11):
    rng = np.random.default_rng(seed)
    h, w, patch, C, E = 64, 64, 16, 8, 8
    bits = di.masks_mixed(12, 5, h, w, 0.01, 0.3)
    f = rng.normal(size=(16, C))
    P = rng.normal(size=(C, E))
    a = orc.embed(f, 4, 4, patch, bits, w, P, 0, 1, 1e-6)
    b = orc.embed(f, 4, 4, patch, bits, w, P, 0, 1, 0.75)
    assert np.allclose(a["pooled"], b["pooled"], rtol=1e-12, atol=1e-13), "eps must cancel in the weighted mean"
    assert np.allclose(a["out"], b["out"], rtol=1e-12, atol=1e-13)


def pin_two_valued_rectangle(orc, seed=12):
    """Two-valued token map + rectangle mask: the whole path in closed form."""
    rng = np.random.default_rng(seed)
    h, w, patch = 48, 64, 16
    gh, gw, C = 3, 4, 6
    G = gh * gw
    u, v = rng.normal(size=C), rng.normal(size=C)
    upatch = np.zeros(G, dtype=bool)
    upatch[[1, 5, 6, 11]] = True
    f = np.where(upatch[:, None], u[None, :], v[None, :])
    rect = (8, 40, 4, 50)
    u8 = rect_mask(h, w, *rect)[None]
    perm = np.array([3, 0, 4, 1, 5, 2])  # not an involution, so P != P^T
    P = np.zeros((C, C))
    P[np.arange(C), perm] = 1.0  # (F P)[perm[c]] = F[c]
    eps = 1e-6
    res = orc.embed(f, gh, gw, patch, di.pack_masks(u8), w, P, 0, 1, eps)
    s = block_sum(np.sqrt(rect_edt(h, w, *rect).astype(float)), patch)
    k = upatch.sum()
    duv = np.sqrt(((u - v) ** 2).sum())
    r = np.where(upatch, (G - k) / G * duv, k / G * duv)
    D = r / (r.mean() + eps)
    wt = s * D
    F = (wt[:, None] * f).sum(axis=0) / wt.sum()
    assert np.allclose(res["wts"][0], wt, rtol=1e-12), "weights break the closed form s x D"
    assert np.allclose(res["Z"][0], wt.sum(), rtol=1e-12)
    assert np.allclose(res["pooled"][0], F, rtol=1e-12, atol=1e-13), "pooled feature breaks the closed form"
    y = np.empty(C)
    y[perm] = F
    assert np.allclose(res["out"][0], y / np.sqrt((y * y).sum()), rtol=1e-12, atol=1e-13), "projection/normalisation break the closed form"


def pin_output_geometry(orc, seed=13):
    rng = np.random.default_rng(seed)
    h, w, patch, C = 64, 96, 16, 24
    bits = di.masks_mixed(14, 6, h, w, 0.01, 0.3)
    f = rng.normal(size=(4 * 6, C))
    Q, _ = np.linalg.qr(rng.normal(size=(C, C)))
    res = orc.embed(f, 4, 6, patch, bits, w, Q, 0, 1)
    out, F = res["out"], res["pooled"]
    assert np.allclose(np.linalg.norm(out, axis=1), 1.0, rtol=1e-13), "outputs must be unit vectors"
    Fn = F / np.linalg.norm(F, axis=1, keepdims=True)
    assert np.allclose(out @ out.T, Fn @ Fn.T, rtol=1e-11, atol=1e-12), "orthogonal projection must keep cosines"


def pin_degenerate(orc, seed=15):
    rng = np.random.default_rng(seed)
    h, w, patch, C, E = 32, 32, 16, 5, 4
    u8 = np.zeros((3, h, w), dtype=np.uint8)
    u8[1, 3:20, 5:25] = 1
    u8[2, 0:32, 0:32] = 1
    bits = di.pack_masks(u8)
    f = rng.normal(size=(4, C))
    P = rng.normal(size=(C, E))
    res = orc.embed(f, 2, 2, patch, bits, w, P)
    assert res["status"][0] == 1 and not res["out"][0].any(), "empty mask: zero row, status 1"
    assert (res["status"][1:] == 0).all()
    # constant token map: D == 0 everywhere -> fall back to spatial weights
    const = np.tile(rng.normal(size=C), (4, 1))
    rc = orc.embed(const, 2, 2, patch, bits, w, P)
    s = orc.spatial_weights(bits, w, patch, 0)
    assert (rc["status"][1:] == 0).all()
    assert np.allclose(rc["wts"][1:], s[1:], rtol=0, atol=0), "zero D must fall back to the spatial weights"
    assert np.allclose(rc["pooled"][1:], const[0], rtol=1e-13), "constant map pools to the constant"
    rz = orc.embed(f, 2, 2, patch, bits, w, np.zeros((C, E)))
    assert (rz["status"][1:] == 2).all() and not rz["out"].any(), "zero projection: zero row, status 2"


def pin_decoders(orc):
    known = {0x00: 0.0, 0x01: 2.0 ** -9, 0x07: 7 * 2.0 ** -9, 0x08: 2.0 ** -6, 0x38: 1.0, 0x39: 1.125,
             0x40: 2.0, 0x7E: 448.0, 0xB8: -1.0, 0xFE: -448.0, 0x80: -0.0}
    for code, val in known.items():
        assert orc.e4m3_value(code) == val, f"e4m3 code {code:#x}"
    assert np.isnan(orc.e4m3_value(0x7F)) and np.isnan(orc.e4m3_value(0xFF))
    bf = np.array([0x3F80, 0xC000, 0x3E80, 0x0000, 0x7F7F], dtype=np.uint16)
    got = orc.decode_tokens(bf.reshape(1, 1, -1), "bf16").ravel()
    assert got[0] == 1.0 and got[1] == -2.0 and got[2] == 0.25 and got[3] == 0.0
    assert got[4] == float.fromhex("0x1.fep127")
    q = np.array([[0x38, 0x40], [0xB8, 0x7E]], dtype=np.uint8)
    sc = np.array([0.5, 3.0], dtype=np.float32)
    d = orc.decode_tokens(q.reshape(2, 1, 2), "f8", sc)
    assert np.array_equal(d, np.array([[0.5, 1.0], [-3.0, 1344.0]])), "FP8 tokens decode as scale * value"


# ---------------------------------------------------------------- open-vocabulary query (R-QUERY)

def _rank(sim_row: np.ndarray, k: int):
    """Top-k by an explicit sort key (score descending, index ascending)."""
    order = sorted(range(len(sim_row)), key=lambda i: (-sim_row[i], i))[:k]
    return order


def pin_query_orthonormal(orc):
    """Orthonormal instance embeddings: a query equal to instance i (up to a
    positive scale) finds i with similarity 1 and every other instance at 0,
    the zeros ranked by index; a zero query scores 0 everywhere."""
    e = np.eye(6)
    text = np.stack([3.0 * e[4], e[1], np.zeros(6)])
    r = orc.query_topk(e, text, 4)
    assert r["idx"][0].tolist() == [4, 0, 1, 2] and r["idx"][1].tolist() == [1, 0, 2, 3]
    assert np.array_equal(r["scores"][0], [1.0, 0.0, 0.0, 0.0])
    assert np.array_equal(r["sim"][2], np.zeros(6)) and r["idx"][2].tolist() == [0, 1, 2, 3]
    r = orc.query_topk(e[:2], text[:1], 4)
    assert r["idx"][0].tolist() == [0, 1, -1, -1] and np.isinf(r["scores"][0, 2]) and r["scores"][0, 2] < 0


def pin_query_bruteforce(orc, seed=31):
    """Similarities against numpy (normalise, then matrix product) and the
    ranking against an explicit sort; scaling an instance by a positive
    factor changes nothing."""
    rng = np.random.default_rng(seed)
    emb = rng.standard_normal((57, 19))
    text = rng.standard_normal((7, 19))
    emb[5] = 0.0
    r = orc.query_topk(emb, text, 9)
    en = np.linalg.norm(emb, axis=1)
    tn = np.linalg.norm(text, axis=1)
    want = (text / tn[:, None]) @ np.where(en[:, None] > 0, emb / np.where(en > 0, en, 1)[:, None], 0).T
    assert np.allclose(r["sim"], want, rtol=0, atol=1e-13), "cosine similarities"
    for j in range(7):
        assert r["idx"][j].tolist() == _rank(r["sim"][j], 9), f"ranking of query {j}"
        assert np.array_equal(r["scores"][j], r["sim"][j][r["idx"][j]])
    emb2 = emb.copy()
    emb2[11] *= 7.5
    r2 = orc.query_topk(emb2, text, 9)
    assert np.allclose(r2["sim"], r["sim"], atol=1e-14) and np.array_equal(r2["idx"], r["idx"])
    # ties go to the lower index
    r3 = orc.query_topk(np.stack([emb[3], emb[3], emb[3]]), text[:1], 3)
    assert r3["idx"][0].tolist() == [0, 1, 2]


def pin_heatmap_two_valued(orc, seed=33):
    """R-HEAT on a two-valued map (k patches u, the rest v, u and v
    orthogonal) with a permutation projection: a text along the projected u
    scores D_u (Eq. 1 closed form) on the u patches and 0 on the v patches, a
    text along minus the projected v scores -D_v there and 0 on u, a zero
    text scores 0.  A transposed projection, a dropped or inverted D, or a
    missing norm all break it."""
    rng = np.random.default_rng(seed)
    G, C, k = 23, 7, 5
    u = np.zeros(C); u[1] = 2.0; u[4] = -1.0
    v = np.zeros(C); v[0] = 3.0; v[2] = 0.5; v[6] = 1.5
    f = np.tile(v, (G, 1))
    idx = rng.choice(G, size=k, replace=False)
    f[idx] = u
    perm = np.array([3, 6, 0, 5, 1, 2, 4])  # not an involution: P and P^T differ
    P = np.zeros((C, C))
    P[np.arange(C), perm] = 1.0
    yu, yv = u @ P, v @ P
    eps = 1e-6
    duv = np.sqrt(((u - v) ** 2).sum())
    r_u, r_v = (G - k) / G * duv, k / G * duv
    rbar = (k * r_u + (G - k) * r_v) / G
    D_u, D_v = r_u / (rbar + eps), r_v / (rbar + eps)
    text = np.stack([5.0 * yu, -0.25 * yv, np.zeros(C)])
    h = orc.query_heatmap(f, P, text, eps)
    isu = np.zeros(G, bool)
    isu[idx] = True
    want = np.zeros((3, G))
    want[0, isu] = D_u
    want[1, ~isu] = -D_v
    assert np.allclose(h, want, rtol=1e-12, atol=1e-14), "two-valued heat-map breaks its closed form"


def pin_heatmap_invariances(orc, seed=34):
    """A constant token map has D = 0 everywhere, so its heat-map is 0; the
    heat-map does not change when a text or the token map is scaled by a
    positive factor; and with an orthogonal projection Q, (tokens, Q, t)
    gives the heat-map of (tokens, identity, t Q^T) (cosines are preserved)."""
    rng = np.random.default_rng(seed)
    G, C, q = 31, 12, 4
    f = rng.normal(size=(G, C)) * rng.uniform(0.3, 2.0, size=(G, 1))
    t = rng.normal(size=(q, C))
    Q, _ = np.linalg.qr(rng.normal(size=(C, C)))
    h = orc.query_heatmap(f, Q, t)
    # the mean of equal values is exact up to rounding, so D is at most ~1e-16 / eps
    assert np.allclose(orc.query_heatmap(np.tile(f[3], (G, 1)), Q, t), 0.0, atol=1e-8), "constant map must give 0"
    assert np.allclose(orc.query_heatmap(2.5 * f, Q, 0.3 * t, 1e-6 * 2.5), h, rtol=1e-11, atol=1e-13), "scale"
    h_id = orc.query_heatmap(f, np.eye(C), t @ Q.T)
    assert np.allclose(h, h_id, rtol=1e-10, atol=1e-12), "orthogonal projection must preserve the cosines"
    assert np.all(np.abs(h) <= orc.token_stats(f, 1e-6)[2][None, :] * (1 + 1e-12)), "|heat| <= D"


# ---------------------------------------------------------------- view quality and fusion (R-Q, R-FUSE)

def pin_dbar_patch_counts(orc, seed=41):
    """Dbar by patch pixel counts: sum_p count_p D_p / sum_p count_p, where
    count_p (the mask's pixels in patch p) comes from a block sum of the u8
    mask; a mask inside one patch takes that patch's D exactly."""
    rng = np.random.default_rng(seed)
    h, w, P = 23, 37, 5
    gh, gw = -(-h // P), -(-w // P)
    D = rng.uniform(0.1, 3.0, gh * gw)
    u8 = random_masks(rng, 4, h, w, 0.35)
    u8[3] = 0
    u8[3, 11:14, 21:24] = 1  # inside patch (2, 4)
    bits = di.pack_masks(u8)
    dbar, area = orc.mask_dbar(bits, w, P, D)
    for i in range(3):
        cnt = block_sum(u8[i].astype(np.float64), P).reshape(-1)
        assert area[i] == u8[i].sum()
        assert abs(dbar[i] - (cnt * D).sum() / cnt.sum()) < 1e-12, f"Dbar of mask {i}"
    assert area[3] == 9 and dbar[3] == D[2 * gw + 4]
    empty = di.pack_masks(np.zeros((1, h, w), np.uint8))
    d0, a0 = orc.mask_dbar(empty, w, P, D)
    assert d0[0] == 0.0 and a0[0] == 0


def pin_angle_closed_forms(orc):
    """Head-on views score 1, grazing and back-facing views 0, a view at 60
    degrees 1/2; the score is the per-voxel mean; no voxels gives 0."""
    n = np.array([[0.0, 0.0, 1.0]] * 6)
    c60 = np.cos(np.pi / 3)
    rays = np.array([[0, 0, -1.0], [1.0, 0, 0], [0, 0, 1.0], [np.sin(np.pi / 3), 0, -c60], [0, -1.0, 0], [0, 0, -1.0]])
    off = np.array([0, 1, 2, 3, 4, 6, 6], dtype=np.int32)
    a = orc.angle_score(rays, n, off)
    assert np.allclose(a, [1.0, 0.0, 0.0, 0.5, 0.5, 0.0], atol=1e-15), a
    # rotation invariance: rotate rays and normals together
    rng = np.random.default_rng(42)
    R, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    rays2 = rng.standard_normal((40, 3))
    rays2 /= np.linalg.norm(rays2, axis=1)[:, None]
    n2 = rng.standard_normal((40, 3))
    n2 /= np.linalg.norm(n2, axis=1)[:, None]
    off2 = np.array([0, 7, 7, 25, 40], dtype=np.int32)
    a2 = orc.angle_score(rays2, n2, off2)
    a3 = orc.angle_score(rays2 @ R.T, n2 @ R.T, off2)
    assert np.allclose(a2, a3, atol=1e-14)
    want = [np.mean(np.maximum(0, -np.einsum("ij,ij->i", rays2[s:t], n2[s:t]))) if t > s else 0.0
            for s, t in zip(off2[:-1], off2[1:])]
    assert np.allclose(a2, want, atol=1e-14)


def pin_quality_factors(orc):
    """Each factor from its closed form: S_size grows linearly with the area
    up to the plateau at H W / lambda; S_sem is the cosine clipped to [0, 1]
    (1 along g, 1/sqrt(2) at 45 degrees, 0 orthogonal or opposite); S_dist
    maps Dbar in [0, 1] onto [1/2, 1]; Q is the product."""
    H, W = 30, 40
    g = np.array([0.0, 2.0, 0.0])
    emb = np.array([[0, 5.0, 0], [1.0, 1.0, 0], [1.0, 0, 0], [0, -1.0, 0], [0, 3.0, 0]])
    area = np.array([100, 0, 1200, 363, 364], dtype=np.int32)
    dbar = np.array([0.0, 1.0, 0.4, 2.0, 1.0])
    ang = np.array([1.0, 0.25, 1.0, 1.0, 0.5])
    Q, comp = orc.view_quality(area, dbar, emb, g, ang, H, W)
    size = np.array([3.3 * 100 / 1200, 0.0, 1.0, 3.3 * 363 / 1200, 1.0])
    assert np.allclose(comp[:, 0], size, atol=1e-15)
    assert np.allclose(comp[:, 2], [1.0, 1 / np.sqrt(2), 0.0, 0.0, 1.0], atol=1e-15)
    assert np.allclose(comp[:, 3], [0.5, 1.0, 0.7, 1.5, 1.0], atol=1e-15)
    assert np.array_equal(comp[:, 1], ang)
    assert np.allclose(Q, comp.prod(axis=1), atol=1e-15)
    assert Q[4] == 0.5 and Q[1] == 0.0
    Q2, _ = orc.view_quality(area, dbar, 7.0 * emb, 0.1 * g, ang, H, W)
    assert np.allclose(Q2, Q, atol=1e-15), "Q does not depend on the embeddings' scale"
    Qn, compn = orc.view_quality(area, dbar, emb, g, None, H, W)
    assert np.array_equal(compn[:, 1], np.ones(5)), "no angle input: S_angle = 1"
    Qz, _ = orc.view_quality(area, dbar, np.zeros_like(emb), g, ang, H, W)
    assert np.array_equal(Qz, np.zeros(5)), "a zero embedding has S_sem = 0"


def _fuse_argmax(ids, q, map_q, n_map):
    """Winner per instance: the first observation of the largest Q above the
    instance's current Q."""
    win = {}
    for t in range(n_map):
        cand = [i for i in range(len(ids)) if ids[i] == t and q[i] > map_q[t]]
        if cand:
            best = max(q[i] for i in cand)
            win[t] = min(i for i in cand if q[i] == best)
    return win


def pin_fuse_argmax(orc, seed=43):
    """Fusion equals a per-instance argmax over the observations (ties to the
    first) gated by the stored Q; untouched instances keep their feature."""
    rng = np.random.default_rng(seed)
    n_map, m, e = 9, 40, 5
    map_q = rng.uniform(0.2, 0.6, n_map)
    map_q[2] = 2.0  # never beaten
    map_emb = rng.standard_normal((n_map, e))
    ids = rng.integers(-1, n_map, m).astype(np.int32)
    ids[ids == 7] = 6  # instance 7 is never observed
    q = np.round(rng.uniform(0.0, 1.0, m), 1)  # many exact ties
    emb = rng.standard_normal((m, e))
    mq, me, won = orc.fuse(ids, q, emb, map_q, map_emb)
    win = _fuse_argmax(ids, q, map_q, n_map)
    for t in range(n_map):
        if t in win:
            assert mq[t] == q[win[t]] and np.array_equal(me[t], emb[win[t]]), f"instance {t}"
        else:
            assert mq[t] == map_q[t] and np.array_equal(me[t], map_emb[t]), f"instance {t} untouched"
    assert sorted(np.nonzero(won)[0].tolist()) == sorted(win.values())
    assert 7 not in win and 2 not in win
    # feeding the observations one at a time gives the same map
    mq1, me1 = map_q.copy(), map_emb.copy()
    for i in range(m):
        mq1, me1, _ = orc.fuse(ids[i:i + 1], q[i:i + 1], emb[i:i + 1], mq1, me1)
    assert np.array_equal(mq1, mq) and np.array_equal(me1, me)
    # explicit ties: the first of two equal observations wins; an observation
    # equal to the stored Q does not replace it
    mq2, me2, won2 = orc.fuse(np.array([0, 0, 1], np.int32), np.array([0.9, 0.9, 0.5]), emb[:3],
                              np.array([0.1, 0.5]), map_emb[:2])
    assert won2.tolist() == [1, 0, 0] and np.array_equal(me2[0], emb[0]) and np.array_equal(me2[1], map_emb[1])


ALL_PINS = [
    ("edt_exhaustive_4x4", lambda o: pin_edt_exhaustive(o, 4, 4)),
    ("edt_random_bruteforce", pin_edt_random_bruteforce),
    ("edt_scipy", pin_edt_scipy),
    ("edt_rectangles", pin_edt_rectangles),
    ("edt_symmetry", pin_edt_symmetry),
    ("edt_bbox_locality", pin_edt_bbox_locality),
    ("spatial_blocksum", pin_spatial_blocksum),
    ("spatial_rectangle", pin_spatial_rectangle),
    ("token_two_valued", pin_token_two_valued),
    ("token_invariances", pin_token_invariances),
    ("pool_constant_on_support", pin_pool_constant_on_support),
    ("pool_single_patch", pin_pool_single_patch),
    ("pool_uniform_mean", pin_pool_uniform_mean),
    ("pool_zero_weight_row", pin_pool_zero_weight_row),
    ("eps_cancels", pin_eps_cancels),
    ("two_valued_rectangle", pin_two_valued_rectangle),
    ("output_geometry", pin_output_geometry),
    ("degenerate", pin_degenerate),
    ("decoders", pin_decoders),
    ("query_orthonormal", pin_query_orthonormal),
    ("heatmap_two_valued", pin_heatmap_two_valued),
    ("heatmap_invariances", pin_heatmap_invariances),
    ("query_bruteforce", pin_query_bruteforce),
    ("dbar_patch_counts", pin_dbar_patch_counts),
    ("angle_closed_forms", pin_angle_closed_forms),
    ("quality_factors", pin_quality_factors),
    ("fuse_argmax", pin_fuse_argmax),
]
