"""The geometry oracle against its pins, and planted mistakes in copies of it
(each must fail at least one pin).  CPU only."""
import os
import sys
import types

import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import geometry_pins as gp  # noqa: E402
from oracle import geometry  # noqa: E402

SRC = geometry.__file__

MUTANTS = [
    ("fx_for_fy", "yc = ((ys - cy) * z) / fy", "yc = ((ys - cy) * z) / fx"),
    ("pose_transposed", "world = [((R[k, 0] * pc[0] + R[k, 1] * pc[1]) + R[k, 2] * pc[2]) + t[k]",
     "world = [((R[0, k] * pc[0] + R[1, k] * pc[1]) + R[2, k] * pc[2]) + t[k]"),
    ("no_translation", "+ R[k, 2] * pc[2]) + t[k] for k", "+ R[k, 2] * pc[2]) for k"),
    ("stride_ignored_rows", "for y in range(0, h, stride):", "for y in range(0, h, 1):"),
    ("depth_max_ignored", "if not np.isfinite(z) or z < dmin or z > dmax:", "if not np.isfinite(z) or z < dmin:"),
    ("core_strict", "core[s:s + chunk] = (_sqdist(seg[s:s + chunk], seg) <= eps2).sum(axis=1) >= min_pts",
     "core[s:s + chunk] = (_sqdist(seg[s:s + chunk], seg) <= eps2).sum(axis=1) > min_pts"),
    ("no_border_points", "k[s:s + chunk] |= (_sqdist(seg[s:s + chunk], cs) <= eps2).any(axis=1)", "pass"),
    ("radius_not_squared", "eps2 = F(eps) * F(eps)", "eps2 = F(eps)"),
    ("voxel_trunc", "c = np.floor(p / F(v)).astype(np.int64)", "c = np.trunc(p / F(v)).astype(np.int64)"),
    ("keep_ignored", "p = points[a:b] if keep is None else points[a:b][np.asarray(keep[a:b]).astype(bool)]",
     "p = points[a:b]"),
    ("overlap_union", "out[k] = len(sa & sb)", "out[k] = len(sa | sb)"),
]


@pytest.mark.parametrize("name,check", gp.ALL_GEOMETRY_PINS, ids=[p[0] for p in gp.ALL_GEOMETRY_PINS])
def test_geometry_pin(name, check):
    check(geometry)


@pytest.mark.parametrize("mid,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_geometry_mutant_is_caught(mid, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {mid} not found exactly once"
    mod = types.ModuleType(f"geometry_{mid}")
    exec(compile(src.replace(old, new), f"<{mid}>", "exec"), mod.__dict__)
    caught = []
    for name, check in gp.ALL_GEOMETRY_PINS:
        try:
            check(mod)
        except AssertionError:
            caught.append(name)
        except Exception:
            caught.append(name + "(error)")
        if caught:
            break
    assert caught, f"mutant {mid} passes every pin"
