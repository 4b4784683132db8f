"""Two facts the direct column search of the distance transform relies on,
checked on the oracle's exact squared EDT (CPU only).

For a mask whose bounding box has at most 510 rows (an item of at most 512
rows with its two padding rows), the rows just above and below the box are
outside the mask, so every e inside the box is at most 255^2.  Hence a row
pass value g >= 255 can never give a candidate below e, and clamping g to 255
changes no e: the search then fits 16-bit arithmetic.  Both are checked
against the separable definition e(y, x) = min_v (y - v)^2 + g(v, x)^2 with g
the horizontal distance to the nearest outside pixel (frame edges outside).

Taller items (up to 1152 rows): every e is at most 575^2, g is clamped to
576 and stored as T(g) = g^2 below 255, 255^2 + (g - 255) above, a 16-bit
lower bound of g^2 that can be decoded.  The packed search over T is exact for
rows whose e is below 255^2, and the groups that end at 255^2 or above are
searched again over the decoded g^2; a CPU model of one column of that search
is checked against the oracle on deep tall masks.
"""
import numpy as np

import disc_inputs as di


def _row_g(m):
    """Horizontal distance of every pixel to the nearest outside pixel."""
    h, w = m.shape
    g = np.zeros((h, w), dtype=np.int64)
    cols = np.arange(w)
    for y in range(h):
        zeros = np.concatenate(([-1], np.nonzero(~m[y])[0], [w]))
        i = np.searchsorted(zeros, cols)
        g[y] = np.minimum(cols - zeros[np.maximum(i - 1, 0)], zeros[np.minimum(i, len(zeros) - 1)] - cols)
        g[y][~m[y]] = 0
    return g


def _masks():
    rng = np.random.default_rng(5)
    h, w = 300, 760
    out = []
    yy, xx = np.mgrid[:h, :w]
    # wide ellipses (g far above 255 inside), a full-width band, a box touching the frame edge
    out.append(((yy - 150) / 140.0) ** 2 + ((xx - 380) / 370.0) ** 2 <= 1.0)
    out.append((yy >= 40) & (yy < 250))
    out.append((yy < 200) & (xx >= 300))
    for _ in range(3):
        cy, cx = rng.integers(60, 240), rng.integers(100, 660)
        ry, rx = rng.integers(20, 60), rng.integers(150, 340)
        out.append(((yy - cy) / ry) ** 2 + ((xx - cx) / rx) ** 2 <= 1.0)
    bits = di.pack_masks(np.stack(out).astype(np.uint8))
    return bits, di.unpack_masks(bits, w).astype(bool), w


def test_edt_bounded_by_box_rows_and_g_clamp_exact(orc):
    bits, masks, w = _masks()
    e = orc.edt_sq(bits, w).astype(np.int64)
    clamped = 0
    for k, m in enumerate(masks):
        ys = np.nonzero(m.any(axis=1))[0]
        y0, y1 = ys.min(), ys.max()
        assert y1 - y0 + 1 <= 510
        rows = np.arange(y0, y1 + 1)
        bound = np.minimum(rows - y0 + 1, y1 + 1 - rows) ** 2
        assert (e[k, y0:y1 + 1].max(axis=1) <= bound).all(), f"mask {k}: e above the box-row bound"
        assert e[k].max() <= 255 ** 2
        g = _row_g(m)
        clamped += int((g > 255).sum())
        gc = np.minimum(g, 255)
        # separable definition over the box rows and its two outside rows (g = 0 there)
        vs = np.arange(y0 - 1, y1 + 2)
        gv = np.zeros((len(vs), m.shape[1]), dtype=np.int64)
        inside = (vs >= 0) & (vs < m.shape[0])
        gv[inside] = gc[vs[inside]]
        for y in range(y0, y1 + 1):
            cand = (y - vs)[:, None] ** 2 + gv ** 2
            assert np.array_equal(cand.min(axis=0), e[k, y]), f"mask {k} row {y}: clamped g changes e"
    assert clamped > 10000, "the masks must exercise the clamp"


# ---------------------------------------------------------------- items taller than 512 rows

def _encode_tall(g):
    """Table entry of the search for items of up to 1152 rows: g is clamped
    to 576 (every e there is at most 575^2); T = g^2 below 255, 255^2 + (g -
    255) from 255 on."""
    g1 = np.minimum(g, 576)
    gc = np.minimum(g1, 255)
    return gc * gc + (g1 - gc)


def _decode_tall(t):
    t = np.asarray(t, dtype=np.int64)
    return np.where(t < 65025, t, (t - 64770) ** 2)


def test_tall_table_encoding():
    g = np.arange(0, 8449, dtype=np.int64)
    t = _encode_tall(g)
    assert t.max() < 1 << 16
    assert (np.diff(t) >= 0).all(), "T must grow with g"
    assert (t <= g * g).all(), "T must never exceed g^2 (a lower bound of every candidate)"
    assert np.array_equal(_decode_tall(t[:577]), g[:577] ** 2), "decoding must give g^2 up to the clamp"
    assert (t[255:] >= 255 ** 2).all()


def _lane_search(T, n, exact_of):
    """One column of the search as the kernel runs it for groups of 4 rows:
    packed 16-bit candidates (d + i)^2 + min(T[u - d - i], T[u + d + i]),
    saturating at 65535, distances in steps of 4 while d^2 is below the
    group's largest best value; a group with a best value of at least 255^2
    is searched again over exact g^2 = exact_of(T).  T has the item's rows
    (padding rows 0 and n - 1 hold 0) and zero guard rows around them."""
    pad = 8 + 1200
    Tp = np.zeros(n + 2 * pad, dtype=np.int64)
    Tp[pad:pad + n] = T
    Ep = exact_of(Tp)
    out = np.zeros(n, dtype=np.int64)
    for u0 in range(0, n, 4):
        rows = np.arange(u0, u0 + 4)
        best = Tp[pad + rows].copy()
        d = 1
        while d * d < best.max():
            for i in range(4):
                dd = d + i
                c = np.minimum(np.minimum(Tp[pad + rows - dd], Tp[pad + rows + dd]) + min(dd * dd, 65535), 65535)
                best = np.minimum(best, c)
            d += 4
        if best.max() >= 65025:
            best = Ep[pad + rows].copy()
            d = 1
            while d * d < best.max():
                for i in range(4):
                    dd = d + i
                    best = np.minimum(best, dd * dd + np.minimum(Ep[pad + rows - dd], Ep[pad + rows + dd]))
                d += 4
        out[u0:u0 + 4] = best[:min(4, n - u0)]
    return out[:n]


def test_tall_item_search_exact(orc):
    """Masks with boxes of 600-1150 rows and depths beyond 255: the encoded
    table and the packed search with its exact re-search give the oracle's
    e on every pixel of sampled columns."""
    h, w = 1152, 700
    yy, xx = np.mgrid[:h, :w]
    ms = [((yy - 576) / 574.0) ** 2 + ((xx - 350) / 340.0) ** 2 <= 1.0,   # depth ~340
          ((yy - 500) / 300.0) ** 2 + ((xx - 300) / 60.0) ** 2 <= 1.0,    # tall and thin
          (yy >= 1) & (yy < 1151) & (xx >= 20) & (xx < 680)]              # a box: depth 330
    bits = di.pack_masks(np.stack(ms).astype(np.uint8))
    e = orc.edt_sq(bits, w).astype(np.int64)
    deep = 0
    rng = np.random.default_rng(11)
    for k, m in enumerate(ms):
        ys = np.nonzero(m.any(axis=1))[0]
        y0, y1 = ys.min(), ys.max()
        n = y1 - y0 + 3
        assert 512 < n <= 1152
        g = _row_g(m)
        cols = np.nonzero(m.any(axis=0))[0]
        for x in rng.choice(cols, size=min(12, cols.size), replace=False):
            gcol = np.zeros(n, dtype=np.int64)
            gcol[1:n - 1] = g[y0:y1 + 1, x]
            got = _lane_search(_encode_tall(gcol), n, _decode_tall)
            want = np.zeros(n, dtype=np.int64)
            want[1:n - 1] = e[k, y0:y1 + 1, x]
            assert np.array_equal(got[1:n - 1], want[1:n - 1]), f"mask {k} column {x}"
            deep += int((want >= 65025).sum())
    assert deep > 1000, "the masks must exercise the exact re-search"
