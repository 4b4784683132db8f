"""Host logic of the benchmark: the algorithmic work counts its roofline uses
(bounding boxes from packed bits, touched patches), checked against the
unpacked masks."""
import numpy as np

import bench
import disc_inputs as di


def test_bbox_and_touched_patches_match_unpacked_masks():
    for seed, (h, w, P) in enumerate([(70, 130, 16), (33, 65, 14), (64, 64, 8)]):
        bits = di.masks_mixed(100 + seed, 12, h, w, 0.002, 0.4)
        u = di.unpack_masks(bits, w).copy()
        u[0] = 0  # an empty mask
        bits = di.pack_masks(u)
        bb = bench._bbox(bits)
        assert bb[0] is None
        for i in range(1, len(u)):
            ys, xs = np.nonzero(u[i])
            assert bb[i] == (ys.min(), ys.max(), xs.min(), xs.max())
        gh, gw = -(-h // P), -(-w // P)
        pad = np.zeros((len(u), gh * P, gw * P), dtype=np.uint8)
        pad[:, :h, :w] = u
        want = int((pad.reshape(len(u), gh, P, gw, P).max(axis=(2, 4)) > 0).sum())
        assert bench._touched_patches(bits, h, w, P) == want


def test_workload_units_counts():
    wl = di.workload("cfg1")
    units, tot = bench.workload_units(wl, gemm_bf16=False)
    f = wl.frames[0]
    assert tot["masks"] == f.m
    assert units["proj"][1] == 2.0 * f.m * 1024 * 768
    assert units["pool"][1] == 2.0 * tot["touched_patches"] * 1024
    assert units["edt"][1] == bench.EDT_OPS_PER_PIXEL * tot["edt_pixels"]
    assert units["scan"][1] == f.bits.nbytes
    r = bench.roofline("edt", 1.0, units, "cfg1")
    assert r["bound"] == "alu" and abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-15


def test_stage_rooflines():
    wl = di.workload("cfg1")
    units, tot = bench.workload_units(wl, gemm_bf16=False)
    avg = {"scan": 0.01, "edt": 0.1, "token_stats": 0.02, "weights": 0.005, "pool": 0.03, "proj": 0.02}
    r = bench.stage_rooflines(avg, units, tot)
    assert set(r) == set(avg)
    assert r["scan"]["bound"] == "hbm" and abs(r["scan"]["achieved"] - units["scan"][1] / 1e-5 / 1e9) < 1e-6
    assert r["proj"]["bound"] == "mfma" and r["proj"]["peak"] == bench.PEAK_TFLOPS["f32"]
    f = wl.frames[0]
    C, E = 1024, 768
    assert abs(r["proj"]["hbm_gbs"] * 2e-5 * 1e9 - (f.m * C * 4 + C * E * 4 + f.m * E * 4)) < 1e-3
    for v in r.values():
        assert abs(v["frac"] - v["achieved"] / v["peak"]) < 1e-15


def test_served_arrivals_rate_and_mix():
    """The served leg's open-loop arrivals: 16 streams at 30 x rate frames/s,
    sorted, within the horizon, streams 0-7 on the 480x640 half of the pool."""
    for rate in (1.0, 4.0):
        arr = bench._arrivals(di, 5.0, rate, 32, 990)
        t = np.array([a for a, _ in arr])
        assert np.all(np.diff(t) >= 0) and t.min() >= 0 and t.max() < 5.0
        n = len(arr)
        want = 16 * 30 * rate * 5.0
        assert abs(n - want) < 4 * np.sqrt(want), (n, want)
        idx = np.array([i for _, i in arr])
        assert set(idx) <= set(range(32))
        small = np.isin(idx % 16, np.arange(8))
        assert 0.4 < small.mean() < 0.6


def test_host_info():
    info = bench.host_info()
    assert info["nproc"] >= 1 and info["affinity"] >= 1
