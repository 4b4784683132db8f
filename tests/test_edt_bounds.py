"""Two facts the direct column search of the distance transform relies on,
checked on the oracle's exact squared EDT (CPU only).

For a mask whose bounding box has at most 510 rows (an item of at most 512
rows with its two padding rows), the rows just above and below the box are
outside the mask, so every e inside the box is at most 255^2.  Hence a row
pass value g >= 255 can never give a candidate below e, and clamping g to 255
changes no e: the search then fits 16-bit arithmetic.  Both are checked
against the separable definition e(y, x) = min_v (y - v)^2 + g(v, x)^2 with g
the horizontal distance to the nearest outside pixel (frame edges outside).
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
