#!/usr/bin/env python3
"""Benchmark of DISC's single-pass, distance-weighted mask feature extraction
(arXiv 2603.03935, Sec. III-C) on one MI355X.

A step is one pass of the whole hot path -- bounding-box scan (which also
lists the distance-transform work), exact EDT fused with the per-patch
sqrt(EDT) sums, token statistics (Eq. 1), weight finalisation, pooling GEMM,
projection GEMM with L2 normalisation -- over one batch of synthetic input
already resident in HBM.

Default run (one JSON line on stdout; progress on stderr):
  * the plain-FP32 single frame (480x640, 30x40x1024 tokens with 16-px
    patches, 128 instance masks, projection 1024x768), one disc_embed_frames
    call per step: ``value`` is its mask embeddings/s over exactly K timed
    steps; ``roofline`` the dominant kernel's algorithmic rate, its duration
    from HIP events recorded on the launch stream around that stage in every
    timed step; stage breakdown and p50/p99 step latency from untimed passes;
  * ``batched_bf16`` (64 frames, BF16) and ``large_fp8`` (16 frames 1080p, FP8
    tokens): masks/s, frames/s, p50/p99 batch latency and stage breakdown;
  * ``served_bf16``: the serving loop (16 camera streams, Poisson 30 frames/s
    each, 480x640 and 720x1280 frames, Poisson(80) masks; continuous batching
    with graph replay): 2 s warm-up, 20 s at the nominal 480 frames/s, a rate
    sweep (x2, x4, ...) up to the first rate whose p99 exceeds 33 ms, and the
    saturated throughput;
  * ``cpu_baseline``: the FP64 oracle as it stands on the host, one thread and
    every thread of the GPU's host share; the same oracle checks sampled masks
    of every leg (``accuracy``: min / median / worst-10 cosine, max abs error);
  * short legs for the open-vocabulary query, view quality / fusion, the
    weighting-mode ablation and the geometry workload.
``--config cfg3`` / ``cfg5`` make a batched workload the main one instead.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks (dense).  ALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# 32-bit integer VALU operations per second.
PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"bf16": 2500.0, "f32": 157.3}
PEAK_ALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic integer operations of the exact separable EDT per pixel of the
# region it must transform (bounding box plus a one-pixel ring): row pass 4
# (two sweeps, an increment and a select each), g^2 1, lower-envelope
# construction 6 (each row pushed once and popped at most once, a 3-op
# intersection test per push and per pop), envelope walk 4 (one comparison of
# two parabolas per row), e 2, sqrt and patch sum 3.
EDT_OPS_PER_PIXEL = 20
CONFIG_DESC = {
    "cfg1": "plain FP32, one 336x336 frame, 8 ellipse masks, tokens 24x24x1024 (14-px patches), proj 1024x768",
    "cfg2": "plain FP32, one 480x640 frame, 128 instance masks, tokens 30x40x1024 (16-px patches), proj 1024x768",
    "cfg3": "batched BF16, 64 frames 480x640, Poisson(60) masks/frame, tokens 30x40x1024, proj 1024x768",
    "cfg5": "large FP8, 16 frames 1080x1920, 500 masks/frame, tokens 68x120x1280 e4m3fn+scale, proj 1280x1024 BF16",
}
KERNEL_SOURCES = {"scan": "k_scan.hip", "edt": "k_edt.hip", "token_stats": "k_stats.hip",
                  "weights": "k_stats.hip", "pool": "k_gemm.hip", "proj": "k_gemm.hip"}


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="cfg2", choices=sorted(CONFIG_DESC))
    ap.add_argument("--batch-steps", type=int, default=20, help="timed steps of the cfg3 leg (cfg5: half)")
    ap.add_argument("--cpu-seconds", type=float, default=8.0, help="oracle time per CPU-baseline run (1 and N threads)")
    ap.add_argument("--cpu-threads", type=int, default=0, help="threads of the all-core CPU baseline (0: host share)")
    ap.add_argument("--serve-seconds", type=float, default=20.0, help="measured duration at the nominal offered load")
    ap.add_argument("--serve-warmup", type=float, default=2.0, help="warm-up arrivals before the served measurement")
    ap.add_argument("--sweep-seconds", type=float, default=4.0, help="duration of each rate of the served sweep")
    ap.add_argument("--skip", default="", help="comma list of legs to leave out: cfg3, cfg5, serve, query, quality, "
                                               "ablation, geometry, cpu")
    ap.add_argument("--no-trace", action="store_true", help="skip per-stage event timing")
    ap.add_argument("--edt-layout", type=int, default=-1, choices=[-1, 0, 1, 2],
                    help="distance-transform band layout (-1: chosen per call)")
    ap.add_argument("--pool-tile", type=int, default=-1, choices=[-1, 1, 2, 4],
                    help="pooling channels per workgroup in units of 64 (-1: autotuned)")
    ap.add_argument("--pool-rows", type=int, default=-1, choices=[-1, 64, 128],
                    help="pooling masks per workgroup (-1: autotuned)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (3 times) and exit: the reference that "
                         "scales the FETCH_SIZE / WRITE_SIZE counters to bytes")
    a = ap.parse_args()
    a.skip = set(x.strip() for x in a.skip.split(",") if x.strip())
    return a


# ---------------------------------------------------------------- algorithmic work

def _bbox(bits: np.ndarray):
    """Per mask (y0, y1, x0, x1) from packed bits, or None when empty."""
    rows = bits.any(axis=2)
    cols = np.bitwise_or.reduce(bits, axis=1)
    out = []
    for i in range(bits.shape[0]):
        ys = np.flatnonzero(rows[i])
        if ys.size == 0:
            out.append(None)
            continue
        ks = np.flatnonzero(cols[i])
        lo, hi = int(cols[i][ks[0]]), int(cols[i][ks[-1]])
        x0 = 64 * int(ks[0]) + ((lo & -lo).bit_length() - 1)
        x1 = 64 * int(ks[-1]) + hi.bit_length() - 1
        out.append((int(ys[0]), int(ys[-1]), x0, x1))
    return out


def _touched_patches(bits: np.ndarray, h: int, w: int, P: int) -> int:
    """Number of (mask, patch) pairs with at least one mask pixel."""
    m, _, wq = bits.shape
    gh, gw = -(-h // P), -(-w // P)
    pad = np.zeros((m, gh * P, wq), dtype=np.uint64)
    pad[:, :h] = bits
    rowor = np.bitwise_or.reduce(pad.reshape(m, gh, P, wq), axis=2)
    u = np.unpackbits(rowor.view(np.uint8), axis=2, bitorder="little")[:, :, :gw * P]
    return int(u.reshape(m, gh, gw, P).any(axis=3).sum())


def workload_units(wl, gemm_bf16: bool):
    """Algorithmic work of one step per stage: (bound, amount, unit)."""
    M = wl.total_masks
    C = wl.frames[0].tokens.c
    E = wl.proj.shape[1]
    bits_bytes = sum(f.bits.nbytes for f in wl.frames)
    tok_bytes = 0
    r_bytes = 0
    w_bytes = 0
    edt_px = 0
    nnz = 0
    for f in wl.frames:
        t = f.tokens
        G = t.gh * t.gw
        tok_bytes += t.data.nbytes + (t.scale.nbytes if t.scale is not None else 0)
        r_bytes += 4 * G
        w_bytes += f.m * G * (2 if gemm_bf16 else 4)
        for bb in _bbox(f.bits):
            if bb is not None:
                edt_px += (bb[1] - bb[0] + 3) * (bb[3] - bb[2] + 3)
        nnz += _touched_patches(f.bits, f.h, f.w, t.patch)
    gdt = "bf16" if gemm_bf16 else "f32"
    gb = 2 if gemm_bf16 else 4
    # bytes a GEMM must move at least: pooling reads each frame's tokens (as
    # the GEMM operand) and the weights once and writes X; projection reads X
    # and P once and writes the FP32 rows
    pool_bytes = tok_bytes + w_bytes + M * C * gb
    proj_bytes = M * C * gb + C * E * gb + M * E * 4
    hbm_views = {"pool": pool_bytes, "proj": proj_bytes}
    return {
        "scan": ("hbm", bits_bytes, "B"),
        "edt": ("alu", EDT_OPS_PER_PIXEL * edt_px, "op"),
        "token_stats": ("hbm", tok_bytes + r_bytes, "B"),
        "weights": ("hbm", w_bytes, "B"),
        "pool": ("mfma:" + gdt, 2.0 * nnz * C, "flop"),
        "proj": ("mfma:" + gdt, 2.0 * M * C * E, "flop"),
    }, {"masks": M, "edt_pixels": edt_px, "touched_patches": nnz, "hbm_views": hbm_views}


def _source_sha(stage: str) -> str:
    p = os.path.join(ROOT, "paper_2603_03935_amd", "csrc", KERNEL_SOURCES[stage])
    with open(p, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic(stage: str, workload: str):
    """HBM bytes per launch from the committed counter runs, if they were taken
    on the current source of the kernel (else None)."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        tab = json.load(f)
    ent = tab.get(f"{stage}/{workload}")
    if not ent or ent.get("source_sha") != _source_sha(stage):
        return None
    return ent["hbm_bytes_per_launch"]


def stage_rooflines(avg: dict, units, totals) -> dict:
    """Every stage against its own bound (from the untimed breakdown pass);
    the GEMM stages also against HBM with the bytes they must move."""
    out = {}
    for st, ms in avg.items():
        if st not in units or ms <= 0:
            continue
        bound, amount, _ = units[st]
        t = ms / 1000.0
        if bound == "hbm":
            r = {"bound": "hbm", "achieved": amount / t / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
        elif bound == "alu":
            r = {"bound": "alu", "achieved": amount / t / 1e12, "peak": PEAK_ALU_TOPS, "unit": "Tops/s"}
        else:
            r = {"bound": "mfma", "achieved": amount / t / 1e12, "peak": PEAK_TFLOPS[bound.split(":")[1]],
                 "unit": "TFLOP/s"}
        r["frac"] = r["achieved"] / r["peak"]
        hb = totals.get("hbm_views", {}).get(st)
        if hb:
            r["hbm_gbs"] = hb / t / 1e9
            r["hbm_frac"] = r["hbm_gbs"] / PEAK_HBM_GBS
        r["avg_ms"] = ms
        out[st] = r
    return out


def roofline(stage: str, avg_ms: float, units, workload: str):
    bound, amount, _ = units[stage]
    t = avg_ms / 1000.0
    if bound == "hbm":
        r = {"bound": "hbm", "achieved": amount / t / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    elif bound == "alu":
        r = {"bound": "alu", "achieved": amount / t / 1e12, "peak": PEAK_ALU_TOPS, "unit": "Tops/s"}
    else:
        dt = bound.split(":")[1]
        r = {"bound": "mfma", "achieved": amount / t / 1e12, "peak": PEAK_TFLOPS[dt], "unit": "TFLOP/s"}
    r["frac"] = r["achieved"] / r["peak"]
    r["traffic"] = _traffic(stage, workload)
    r["kernel"] = stage
    r["avg_ms"] = avg_ms
    r["algorithmic_per_launch"] = amount
    return r


# ---------------------------------------------------------------- served leg

def _arrivals(di, seconds: float, rate_x: float, n_frames: int, seed_frame: int):
    """Open-loop arrivals of the serving mix: 16 streams with exponential gaps
    at 30 x rate_x frames/s each, streams 0-7 carrying the 480x640 frames of
    the pool and 8-15 the 720x1280 ones.  Returns [(t, frame index)]."""
    out = []
    for s in range(16):
        n = int(seconds * 30 * rate_x * 2) + 16
        gaps = di.exponential_gaps(di.frame_seed(4, seed_frame), s, n, 1.0 / (30.0 * rate_x))
        t = np.cumsum(gaps)
        for k, tt in enumerate(t[t < seconds]):
            idx = (s % 8) + (8 if s >= 8 else 0) + 16 * (k % 2)
            out.append((float(tt), idx % n_frames))
    out.sort()
    return out


def _offer(srv, ins, outs, arrivals):
    """Submit the arrivals at their times (late ones at once), wait for all;
    returns the wall time from the first arrival to the last completion."""
    t0 = time.perf_counter()
    tickets = []
    for ta, idx in arrivals:
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        tickets.append(srv.submit_frame(ins[idx], outs[idx])[0])
    for t in tickets:
        if srv.wait(t) != 0:
            raise RuntimeError("served frame failed")
    return time.perf_counter() - t0


def served_leg(disc, di, dev, seconds: float, warm_seconds: float, sweep_seconds: float, p99_limit_ms: float = 33.0):
    """Serving loop, BF16 operands, the serving mix (16 streams, Poisson 30
    frames/s each; 480x640 and 720x1280 frames, Poisson(80) masks), inputs
    resident.  Warm-up arrivals first (graph capture, caches), then the
    nominal offered load (480 frames/s) for `seconds` with latency
    arrival -> completion as the server measures it, then a sweep of the
    offered rate (x2, x4, ...) for `sweep_seconds` each that stops at the
    first rate whose p99 exceeds one frame period (33 ms), then the saturated
    throughput with every frame submitted at once."""
    import torch

    wl = di.workload("cfg4")
    proj = dev.dev_proj(wl.proj, "bf16")
    ins = []
    for f in wl.frames:
        data, scale = dev.dev_tokens(f.tokens)
        ins.append(disc.FrameInput(data, dev.dev_bits(f.bits), f.h, f.w, f.tokens.patch, scale))
    outs = [disc.alloc_outputs([x], wl.proj.shape[1])[0] for x in ins]
    torch.cuda.synchronize()
    cfg = dict(proj=proj, tok_dtype=disc.DISC_BF16, c=1024, e=wl.proj.shape[1], max_frames=8, max_masks=2400,
               max_h=720, max_w=1280, min_patch=16, lanes=2, use_graph=True, mem_budget=16 << 30)
    masks_of = [x.m for x in ins]

    def level(srv, rate_x, secs, seed):
        arr = _arrivals(di, secs, rate_x, len(ins), seed)
        srv.reset_stats()
        wall = _offer(srv, ins, outs, arr)
        st = srv.stats()
        masks = sum(masks_of[i] for _, i in arr)
        return {"rate_x": rate_x, "offered_fps": 480.0 * rate_x, "frames": len(arr), "masks": masks,
                "seconds": wall, "frames_per_s": len(arr) / wall, "masks_per_s": masks / wall,
                "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "max_ms": st["max_ms"], "batches": st["batches"],
                "mean_batch_frames": st["mean_batch_frames"]}

    res = {"streams": 16, "fps_per_stream": 30, "frame_pool": len(ins), "p99_limit_ms": p99_limit_ms}
    with disc.Server(**cfg) as srv:
        _offer(srv, ins, outs, _arrivals(di, warm_seconds, 1.0, len(ins), 989))  # warm-up, not reported
        res["warmup_seconds"] = warm_seconds
        res["nominal"] = level(srv, 1.0, seconds, 990)
        sweep = []
        rate = 2.0
        while rate <= 64.0:
            lv = level(srv, rate, sweep_seconds, 990 + int(rate))
            sweep.append(lv)
            if lv["p99_ms"] > p99_limit_ms:
                break
            rate *= 2.0
        res["sweep"] = sweep
        ok = [lv["rate_x"] for lv in [res["nominal"]] + sweep if lv["p99_ms"] <= p99_limit_ms]
        res["max_rate_x_within_limit"] = max(ok) if ok else None
    # saturated: every frame of the mix submitted back to back, several rounds
    with disc.Server(**cfg) as srv:
        for x, o in zip(ins[:4], outs[:4]):
            srv.wait(srv.submit_frame(x, o)[0])
        srv.reset_stats()
        rounds = 8
        t0 = time.perf_counter()
        tickets = [srv.submit_frame(ins[i], outs[i])[0] for _ in range(rounds) for i in range(len(ins))]
        for t in tickets:
            if srv.wait(t) != 0:
                raise RuntimeError("served frame failed")
        wall = time.perf_counter() - t0
        st = srv.stats()
    masks = rounds * sum(masks_of)
    res["saturated"] = {"frames": rounds * len(ins), "masks": masks, "seconds": wall, "masks_per_s": masks / wall,
                        "frames_per_s": rounds * len(ins) / wall, "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
                        "mean_batch_frames": st["mean_batch_frames"]}
    return res


# ---------------------------------------------------------------- query leg

def query_leg(disc, di, reps: int = 20):
    """Open-vocabulary query: 1024 text embeddings against 8000 instance
    embeddings (the mask count of the large FP8 workload) of width 1024,
    top-10 per query.  The similarity GEMM is timed against the FP32 MFMA
    peak (2 q m e flops)."""
    import torch

    m, e, q, k = 8000, 1024, 1024, 10
    emb = torch.from_numpy(di.normal_rows(di.frame_seed(6, 0), m, e, "f32")[0]).cuda()
    text = torch.from_numpy(di.normal_rows(di.frame_seed(6, 1), q, e, "f32")[0]).cuda()
    for _ in range(3):
        disc.query_topk(emb, text, k)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        disc.query_topk(emb, text, k)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    flops = 2.0 * q * m * e
    return {"queries": q, "instances": m, "width": e, "k": k, "ms_per_call": ms,
            "queries_per_s": q / (ms / 1000.0), "sim_tflops": flops / (ms / 1000.0) / 1e12,
            "sim_frac_of_fp32_mfma_peak": flops / (ms / 1000.0) / 1e12 / PEAK_TFLOPS["f32"]}


def _time_ms(fn, reps: int) -> float:
    import torch

    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def quality_leg(disc, di, dev, ins, proj, outs, opts, reps: int = 50):
    """View quality and fusion (Sec. III-C, Eqs. 2-3): the extra cost of the
    mean distinctiveness and area outputs in the embedding call of the bench
    workload, and the three streaming kernels at mapping scale -- Q for 100k
    observations of width 768, S_angle over 4M voxels in 20k detections, and
    fusion of 100k observations into a 20k-instance map.  Bandwidth figures
    count the algorithmic bytes (every input element read once, every output
    written once) against the HBM peak."""
    import torch

    q_outs = disc.alloc_outputs(ins, outs[0].out.shape[1], quality=True)
    plain_ms = _time_ms(lambda: disc.embed_frames(ins, proj, outputs=outs, options=opts), reps)
    q_ms = _time_ms(lambda: disc.embed_frames(ins, proj, outputs=q_outs, options=opts), reps)

    rng = np.random.default_rng(di.frame_seed(7, 0))
    m, e = 100_000, 768
    emb = torch.from_numpy(di.normal_rows(di.frame_seed(7, 1), m, e, "f32")[0]).cuda()
    g = torch.from_numpy(di.normal_rows(di.frame_seed(7, 2), 1, e, "f32")[0][0]).cuda()
    area = torch.from_numpy(rng.integers(1, 480 * 640 // 4, m).astype(np.int32)).cuda()
    dbar = torch.from_numpy(rng.uniform(0.2, 2.0, m).astype(np.float32)).cuda()
    ang = torch.from_numpy(rng.uniform(0.0, 1.0, m).astype(np.float32)).cuda()
    vq_ms = _time_ms(lambda: disc.view_quality(area, dbar, emb, g, 480, 640, ang), reps)
    vq_bytes = m * e * 4 + m * (4 + 4 + 4) + m * 4 + m * 16

    nd, nv = 20_000, 4_000_000
    lens = rng.multinomial(nv - nd * 50, np.full(nd, 1.0 / nd)) + 50
    off = torch.from_numpy(np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)).cuda()
    rays = torch.nn.functional.normalize(torch.from_numpy(rng.standard_normal((nv, 3), dtype=np.float32)).cuda(), dim=1)
    nrm = torch.nn.functional.normalize(torch.from_numpy(rng.standard_normal((nv, 3), dtype=np.float32)).cuda(), dim=1)
    an_ms = _time_ms(lambda: disc.angle_score(rays, nrm, off), reps)
    an_bytes = nv * 24 + (nd + 1) * 4 + nd * 4

    n_map = 20_000
    ids = torch.from_numpy(rng.integers(0, n_map, m).astype(np.int32)).cuda()
    q = torch.from_numpy(rng.uniform(0.0, 1.0, m).astype(np.float32)).cuda()
    map_q0 = torch.from_numpy(rng.uniform(0.0, 0.9, n_map).astype(np.float32)).cuda()
    map_emb = torch.zeros((n_map, e), dtype=torch.float32, device="cuda")
    map_q = map_q0.clone()
    won = torch.empty((m,), dtype=torch.int32, device="cuda")

    def fuse_once():
        map_q.copy_(map_q0)  # same decisions every repetition
        disc.fuse(ids, q, emb, map_q, map_emb, won=won)

    fu_ms = _time_ms(fuse_once, reps)  # includes the 80 KB reset copy of map_q
    winners = int(won.sum().item())
    fu_bytes = m * (4 + 4 + 4) + winners * e * 8 + n_map * 4
    gbs = lambda b, ms: b / (ms / 1000.0) / 1e9  # noqa: E731
    return {"embed_ms": plain_ms, "embed_with_dbar_area_ms": q_ms, "dbar_area_overhead": q_ms / plain_ms - 1.0,
            "view_quality": {"observations": m, "width": e, "ms": vq_ms, "gbs": gbs(vq_bytes, vq_ms),
                             "frac_of_hbm_peak": gbs(vq_bytes, vq_ms) / PEAK_HBM_GBS},
            "angle_score": {"detections": nd, "voxels": nv, "ms": an_ms, "gbs": gbs(an_bytes, an_ms),
                            "frac_of_hbm_peak": gbs(an_bytes, an_ms) / PEAK_HBM_GBS},
            "fuse": {"observations": m, "instances": n_map, "winners": winners, "ms": fu_ms,
                     "gbs": gbs(fu_bytes, fu_ms), "frac_of_hbm_peak": gbs(fu_bytes, fu_ms) / PEAK_HBM_GBS}}


def geometry_leg(disc, di, dev, reps: int = 20):
    """The mapping side of each segment (Sec. III-B) on one synthetic RGB-D
    frame (480x640, 40 overlapping dome-shaped objects in front of a plane,
    range-scaled depth noise, 0.3 % outlier and 1 % missing readings):
    back-projection of every mask pixel (stride 1), DBSCAN noise removal
    (eps 3 cm, 8 points), voxel sets (2 cm) and the exact overlap of every
    segment with every segment of a second view of the scene (camera moved
    3 cm)."""
    import torch
    from disc_inputs.scene import depth_scene

    sc = depth_scene(di.frame_seed(9, 0), 480, 640, n_obj=40)
    depth = torch.from_numpy(sc.depth).cuda()
    bits = dev.dev_bits(sc.bits)
    m = sc.bits.shape[0]
    bp_ms = _time_ms(lambda: disc.backproject(depth, bits, sc.h, sc.w, sc.camera, 1), reps)
    pts, off = disc.backproject(depth, bits, sc.h, sc.w, sc.camera, 1)
    n = pts.shape[0]
    db_ms = _time_ms(lambda: disc.dbscan_denoise(pts, off, 0.03, 8), reps)
    keep = disc.dbscan_denoise(pts, off, 0.03, 8)
    vx_ms = _time_ms(lambda: disc.voxelize(pts, off, 0.02, keep=keep), reps)
    va, oa, _ = disc.voxelize(pts, off, 0.02, keep=keep)
    cam2 = dict(sc.camera)
    cam2["t"] = cam2["t"] + np.array([0.03, 0.0, -0.02])
    p2, o2 = disc.backproject(depth, bits, sc.h, sc.w, cam2, 1)
    vb, ob, _ = disc.voxelize(p2, o2, 0.02)
    pairs = torch.from_numpy(np.array([(i, j) for i in range(m) for j in range(m)], np.int32)).cuda()
    ov_ms = _time_ms(lambda: disc.voxel_overlap(va, oa, vb, ob, pairs), reps)
    return {"frame": "480x640 RGB-D, %d segments" % m, "points": int(n), "kept": int(keep.sum().item()),
            "voxels": int(va.shape[0]), "pairs": int(pairs.shape[0]),
            "backproject_ms": bp_ms, "backproject_mpts_per_s": n / (bp_ms / 1000.0) / 1e6,
            "dbscan_ms": db_ms, "dbscan_mpts_per_s": n / (db_ms / 1000.0) / 1e6,
            "voxelize_ms": vx_ms, "voxelize_mpts_per_s": n / (vx_ms / 1000.0) / 1e6,
            "overlap_ms": ov_ms, "overlap_pairs_per_s": pairs.shape[0] / (ov_ms / 1000.0),
            "note": "backproject and voxelize include one host synchronisation each (sizing their outputs)"}


ABLATION_MODES = {"edt_x_D": (0, 1), "edt_only": (0, 0), "area_x_D": (1, 1), "area_naive_average": (1, 0)}


def ablation_leg(disc, di, dev, ins, proj, outs, masks: int, reps: int = 50):
    """The weighting modes at the bench workload (EDT x D as built, EDT
    alone, the pixel-count (AREA) weighting with and without D, and the naive
    average over the mask), and how close each mode's embedding comes to the
    known object features of a synthetic object scene (40 overlapping
    ellipses on a background, 480x640, patch tokens mixing the features of
    the pixels they cover, noise and 12 high-norm outlier tokens): cosine of
    each mask's embedding with its object's projected feature."""
    import torch
    from disc_inputs.scene import object_scene

    res = {}
    scene = object_scene(di.frame_seed(8, 0))
    fr = scene.frame
    data, scale = dev.dev_tokens(fr.tokens)
    sin = disc.FrameInput(data, dev.dev_bits(fr.bits), fr.h, fr.w, fr.tokens.patch, scale)
    P = di.projection(di.frame_seed(8, 1), fr.tokens.data.shape[-1], 768, "f32")
    sproj = torch.from_numpy(P).cuda()
    ref = scene.truth @ P.astype(np.float64)
    ref /= np.linalg.norm(ref, axis=1)[:, None]
    for name, (sp, dd) in ABLATION_MODES.items():
        o = disc.make_options(sp, dd)
        ms = _time_ms(lambda: disc.embed_frames(ins, proj, outputs=outs, options=o), reps)
        got = disc.embed_frames([sin], sproj, options=o)[0].out.cpu().numpy().astype(np.float64)
        cos = (got * ref).sum(axis=1)
        res[name] = {"spatial": "edt" if sp == 0 else "area", "distinct": bool(dd), "ms_per_step": ms,
                     "masks_per_s": masks / (ms / 1000.0), "scene_masks": int(len(cos)),
                     "scene_cos_mean": float(cos.mean()), "scene_cos_p10": float(np.percentile(cos, 10))}
    return res


# ---------------------------------------------------------------- workload legs

def gemm_bf16_of(wl) -> bool:
    return not (wl.proj_dtype == "f32" and wl.frames[0].tokens.dtype == "f32")


def run_workload(disc, di, dev, name: str, steps: int, warmup: int, opts, trace: bool, live_roof: bool,
                 sample_masks: int):
    """One workload: warm-up, an untimed pass with every stage between HIP
    events (stage breakdown), exactly `steps` timed steps (wall clock around
    them; with live_roof the dominant stage is also bracketed by events on its
    launch stream, its average duration giving the roofline), then an untimed
    pass with per-step events (p50/p99 step latency).  Returns the result and
    the host copies of `sample_masks` output rows spread over the batch (the
    oracle leg checks them)."""
    import torch

    wl = di.workload(name)
    ins = []
    for f in wl.frames:
        data, scale = dev.dev_tokens(f.tokens)
        ins.append(disc.FrameInput(data, dev.dev_bits(f.bits), f.h, f.w, f.tokens.patch, scale))
    proj = dev.dev_proj(wl.proj, wl.proj_dtype)
    outs = disc.alloc_outputs(ins, wl.proj.shape[1])
    stream = torch.cuda.current_stream()
    units, totals = workload_units(wl, gemm_bf16_of(wl))

    def step():
        disc.embed_frames(ins, proj, outputs=outs, options=opts, stream=stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    stages = {}
    if trace:
        disc.trace_select(None)
        disc.trace_reset()
        disc.trace_enable(True)
        for _ in range(min(steps, 50)):
            step()
        torch.cuda.synchronize()
        disc.trace_enable(False)
        stages = disc.trace_read()
    avg = {k: (ms / n if n else 0.0) for k, (ms, n) in stages.items()}
    dom = max(avg, key=avg.get) if avg else None
    if dom and live_roof:
        disc.trace_select([dom])
        disc.trace_reset()
        disc.trace_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    roof = None
    if dom and live_roof:
        disc.trace_enable(False)
        live_ms, live_n = disc.trace_read()[dom]
        disc.trace_select(None)
        roof = roofline(dom, live_ms / max(live_n, 1), units, name)
    ms_per_step = wall * 1000.0 / steps
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    for i in range(steps):
        starts[i].record(stream)
        step()
        ends[i].record(stream)
    torch.cuda.synchronize()
    lat = np.array([a.elapsed_time(b) for a, b in zip(starts, ends)])
    # output rows to check against the oracle: spread over frames and masks
    picks = []
    nf = len(wl.frames)
    per = max(1, sample_masks // nf)
    for fi in range(nf):
        m = wl.frames[fi].m
        if len(picks) >= sample_masks or m == 0:
            continue
        k = min(m, per, sample_masks - len(picks))
        idx = sorted(set(int(x) for x in np.linspace(0, m - 1, k).round()))
        picks.append((fi, idx, outs[fi].out[idx].cpu().numpy(), outs[fi].status[idx].cpu().numpy()))
    res = {"workload": name, "desc": CONFIG_DESC[name], "frames": nf, "masks_per_step": totals["masks"],
           "steps": steps, "ms_per_step": ms_per_step, "masks_per_s": totals["masks"] / (ms_per_step / 1000.0),
           "frames_per_s": nf / (ms_per_step / 1000.0), "p50_ms": float(np.percentile(lat, 50)),
           "p99_ms": float(np.percentile(lat, 99)), "stage_avg_ms": avg,
           "stage_roofline": stage_rooflines(avg, units, totals), "edt_pixels": totals["edt_pixels"],
           "touched_patches": totals["touched_patches"],
           "dtype": "f32" if not gemm_bf16_of(wl) else ("f8+bf16" if wl.frames[0].tokens.dtype == "f8" else "bf16")}
    return res, roof, {"wl": wl, "picks": picks}, (ins, proj, outs, totals)


# ---------------------------------------------------------------- oracle leg (CPU baseline + accuracy)

def host_info() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count()
    return {"model": model, "nproc": os.cpu_count(), "affinity": aff}


def oracle_leg(checks: dict, main_wl, seconds: float, threads: int) -> tuple:
    """The FP64 oracle as it stands (single-threaded C, no tuning), timed on
    the host: one thread over the first 16 masks of the main workload's frame
    0, repeated for `seconds`; then `threads` threads at once, each running
    the same single-threaded oracle on the same sample, for `seconds`.  Its
    results for the masks sampled from every GPU leg give that leg's
    accuracy: per-mask cosine against the FP64 result (min, median, worst 10),
    the largest absolute element difference and the status agreement."""
    from concurrent.futures import ThreadPoolExecutor

    from tests.gpu_common import cosines, oracle_frame

    fr = main_wl.frames[0]
    n = min(fr.m, 16)
    idx = list(range(n))

    def run_for(secs):
        done = reps = 0
        t0 = time.perf_counter()
        while True:
            oracle_frame(fr, main_wl.proj, main_wl.proj_dtype, idx=idx)
            done += n
            reps += 1
            if time.perf_counter() - t0 > secs:
                return done, time.perf_counter() - t0

    d1, e1 = run_for(seconds)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(lambda _: run_for(seconds), range(threads)))
    dn = sum(p[0] for p in parts)
    en = max(p[1] for p in parts)
    info = host_info()
    cpu = {"value": dn / en, "unit": "mask embeddings/s", "cores": threads, "kind": "oracle",
           "sample": f"{main_wl.name} frame 0, its first {n} masks (token statistics, full-frame FP64 EDT, pooling, "
                     f"projection per call), repeated: {threads} threads x {en:.1f} s, each the single-threaded "
                     f"oracle",
           "single_core": {"value": d1 / e1, "cores": 1, "seconds": e1, "masks": d1},
           "host": info}
    acc = {}
    for name, chk in checks.items():
        wl = chk["wl"]
        cos_all, err, stat_ok, nm = [], 0.0, True, 0
        bound = 1.0 - 1e-6 if not gemm_bf16_of(wl) else 0.9995
        for fi, idx2, got, st in chk["picks"]:
            ref = oracle_frame(wl.frames[fi], wl.proj, wl.proj_dtype, idx=idx2)
            stat_ok &= bool(np.array_equal(st, ref["status"]))
            okm = ref["status"] == 0
            nm += len(idx2)
            if okm.any():
                cos_all.extend(cosines(got[okm].astype(np.float64), ref["out"][okm]).tolist())
            err = max(err, float(np.abs(got.astype(np.float64) - ref["out"]).max()))
        c = np.sort(np.array(cos_all))
        acc[name] = {"masks_checked": nm, "bound_cos": bound, "min_cos": float(c[0]) if c.size else None,
                     "median_cos": float(np.median(c)) if c.size else None, "worst10_cos": c[:10].tolist(),
                     "max_abs_err": err, "status_equal": stat_ok,
                     "pass": bool(stat_ok and (c.size == 0 or c[0] >= bound))}
    return cpu, acc


# ---------------------------------------------------------------- main

def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this program runs on one GPU; --gpus must be 1 "
                                   "(the path shards by frames with no exchange between GPUs)"}))
        sys.exit(2)
    import torch

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 4, "copies": 3}))
        return

    import disc_inputs as di
    import disc_inputs.device as dev
    import paper_2603_03935_amd as disc

    disc.load()
    opts = disc.make_options(edt_layout=args.edt_layout, pool_tile=args.pool_tile, pool_rows=args.pool_rows)
    main_res, roof, main_chk, (ins, proj, outs, totals) = run_workload(
        disc, di, dev, args.config, args.steps, args.warmup, opts, not args.no_trace, True,
        sample_masks=128 if args.config in ("cfg1", "cfg2") else 24)
    checks = {args.config: main_chk}
    ms_per_step = main_res["ms_per_step"]
    value = main_res["masks_per_s"]
    progress(f"main {args.config}: {value:.0f} masks/s")

    # batched BF16 and large FP8 workloads (throughput, latency, breakdown)
    batched = {}
    if args.config == "cfg2":
        for name, steps, leg in (("cfg3", args.batch_steps, "batched_bf16"), ("cfg5", max(args.batch_steps // 2, 3),
                                                                             "large_fp8")):
            if name in args.skip:
                continue
            r, _, chk, _ = run_workload(disc, di, dev, name, steps, 3, opts, not args.no_trace, False,
                                        sample_masks=32 if name == "cfg3" else 12)
            batched[leg] = r
            checks[name] = chk
            torch.cuda.empty_cache()
            progress(f"{leg} ({name}): {r['masks_per_s']:.0f} masks/s")

    served = None
    if "serve" not in args.skip and args.config == "cfg2":
        served = served_leg(disc, di, dev, args.serve_seconds, args.serve_warmup, args.sweep_seconds)
        progress("served leg done")
    query = None if "query" in args.skip else query_leg(disc, di)
    quality = None if "quality" in args.skip else quality_leg(disc, di, dev, ins, proj, outs, opts)
    ablation = None if "ablation" in args.skip else ablation_leg(disc, di, dev, ins, proj, outs, totals["masks"])
    geometry = None if "geometry" in args.skip else geometry_leg(disc, di, dev)

    # the oracle: CPU baseline (one thread, then every host thread of the
    # GPU's share) and the accuracy of every leg's sampled masks
    cpu = None
    if "cpu" not in args.skip:
        threads = args.cpu_threads or min(int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or host_info()["affinity"], 16)
        cpu, acc = oracle_leg(checks, main_chk["wl"], args.cpu_seconds, max(1, threads))
        main_res["accuracy"] = acc.get(args.config)
        for leg, r in batched.items():
            r["accuracy"] = acc.get(r["workload"])
        progress("oracle leg done")

    config = {k: v for k, v in main_res.items() if k not in ("masks_per_s", "ms_per_step", "steps", "dtype")}
    res = {
        "metric": "mask embeddings/sec and p99 frame latency, BF16 served vs FP32 plain, 1 MI355X",
        "value": value,
        "unit": "mask embeddings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_res["dtype"],
        "data": "synthetic",
        "config": config,
        "roofline": roof,
        "cpu_baseline": cpu,
        "batched_bf16": batched.get("batched_bf16"),
        "large_fp8": batched.get("large_fp8"),
        "served_bf16": served,
        "query_topk": query,
        "view_quality_fusion": quality,
        "ablation": ablation,
        "geometry": geometry,
    }
    print(json.dumps(res))


def progress(msg: str):
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


if __name__ == "__main__":
    main()
