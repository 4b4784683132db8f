"""Seeded synthetic inputs for DISC feature extraction (arXiv 2603.03935).

This module draws inputs only: masks, patch-token maps, projections, mask
counts and arrival gaps, plus the quantised forms (BF16, per-token-scaled OCP
e4m3fn) a caller would hand to the library.  It contains none of the method's
arithmetic and is shared by the HIP path's tests/benchmark and the CPU oracle.

The draws live in ``gen.c`` (compiled on first use into ``libdisc_gen.so``).

Workload recipes (the paper's RGB-D mapping workloads -- Replica, ScanNet and
HM3D frames with FastSAM masks and OpenCLIP ViT tokens, Sec. IV -- are not
available; these synthetic stand-ins take their shapes):

* ``cfg1``: one 336x336 frame, 8 filled ellipses (semi-axes U(10,120)), tokens
  24x24x1024 FP32 N(0,1) with 14-px patches, projection 1024x768 FP32 N(0,1/C).
* ``cfg2``: one 480x640 frame, 128 instance-like masks (area log-uniform
  0.1%-30%), tokens 30x40x1024 FP32, 16-px patches, projection 1024x768 FP32.
* ``cfg3``: 64 such frames with Poisson(60) masks each (clipped to 1..300),
  BF16 tokens and projection.
* ``cfg4``: serving mix, 480x640 (30x40 grid) and 720x1280 (45x80 grid)
  frames, Poisson(80) masks, BF16.
* ``cfg5``: 16 frames 1080x1920, 500 masks each (area 0.01%-20%), tokens
  68x120x1280 e4m3fn with per-token FP32 scales, projection 1280x1024 BF16.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB_PATH = os.path.join(_HERE, "libdisc_gen.so")
_lib = None

DTYPE_F32, DTYPE_BF16, DTYPE_F8, DTYPE_F64 = 0, 1, 2, 3
_DTYPE_CODES = {"f32": DTYPE_F32, "bf16": DTYPE_BF16, "f8": DTYPE_F8, "f64": DTYPE_F64}


def build(force: bool = True) -> str:
    """Compile gen.c into libdisc_gen.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        u64, i32, i64, dbl, vp = ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        lib.disc_gen_masks_ellipses.argtypes = [u64, i32, i32, i32, dbl, dbl, vp]
        lib.disc_gen_masks_mixed.argtypes = [u64, i32, i32, i32, dbl, dbl, vp]
        lib.disc_gen_quantize_bf16.argtypes = [vp, i64, vp]
        lib.disc_gen_quantize_e4m3.argtypes = [vp, i64, vp]
        lib.disc_gen_quantize_fp8_rows.argtypes = [vp, i64, i32, vp, vp]
        lib.disc_gen_normal_rows.argtypes = [u64, u64, i64, i32, dbl, i32, vp, vp]
        lib.disc_gen_structured_tokens.argtypes = [u64, i32, i32, i32, i32, dbl, i32, dbl, vp]
        lib.disc_gen_poisson_counts.argtypes = [u64, i32, dbl, i32, i32, vp]
        lib.disc_gen_exponential.argtypes = [u64, u64, i32, dbl, vp]
        for f in (lib.disc_gen_masks_ellipses, lib.disc_gen_masks_mixed, lib.disc_gen_quantize_bf16,
                  lib.disc_gen_quantize_e4m3, lib.disc_gen_quantize_fp8_rows, lib.disc_gen_normal_rows,
                  lib.disc_gen_structured_tokens, lib.disc_gen_poisson_counts, lib.disc_gen_exponential):
            f.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


# ---------------------------------------------------------------- masks

def words_per_row(w: int) -> int:
    return (w + 63) // 64


def masks_ellipses(seed: int, m: int, h: int, w: int, amin: float = 10.0, amax: float = 120.0) -> np.ndarray:
    bits = np.zeros((m, h, words_per_row(w)), dtype=np.uint64)
    if m:
        _load().disc_gen_masks_ellipses(seed, m, h, w, amin, amax, _ptr(bits))
    return bits


def masks_mixed(seed: int, m: int, h: int, w: int, lo: float = 1e-3, hi: float = 0.30) -> np.ndarray:
    bits = np.zeros((m, h, words_per_row(w)), dtype=np.uint64)
    if m:
        _load().disc_gen_masks_mixed(seed, m, h, w, lo, hi, _ptr(bits))
    return bits


def pack_masks(u8: np.ndarray) -> np.ndarray:
    """[m][h][w] bool/uint8 -> [m][h][wq] uint64 in the library's bit layout."""
    u8 = np.ascontiguousarray(u8 != 0)
    m, h, w = u8.shape
    wq = words_per_row(w)
    padded = np.zeros((m, h, wq * 64), dtype=np.uint8)
    padded[:, :, :w] = u8
    packed = np.packbits(padded, axis=-1, bitorder="little")  # [m][h][wq*8] bytes
    return np.ascontiguousarray(packed).view(np.uint64).reshape(m, h, wq).copy()


def unpack_masks(bits: np.ndarray, w: int) -> np.ndarray:
    """[m][h][wq] uint64 -> [m][h][w] uint8."""
    bits = np.ascontiguousarray(bits, dtype=np.uint64)
    m, h, wq = bits.shape
    by = bits.view(np.uint8).reshape(m, h, wq * 8)
    return np.unpackbits(by, axis=-1, bitorder="little")[:, :, :w].copy()


# ---------------------------------------------------------------- tokens

@dataclass
class Tokens:
    data: np.ndarray            # [gh][gw][c]: float32, uint16 (bf16 bits) or uint8 (e4m3fn codes)
    dtype: str                  # "f32" | "bf16" | "f8"
    scale: Optional[np.ndarray]  # [gh*gw] float32 for "f8", else None
    patch: int

    @property
    def gh(self):
        return self.data.shape[0]

    @property
    def gw(self):
        return self.data.shape[1]

    @property
    def c(self):
        return self.data.shape[2]


def _np_dtype(dtype: str):
    return {"f32": np.float32, "bf16": np.uint16, "f8": np.uint8, "f64": np.float64}[dtype]


def normal_rows(seed: int, rows: int, c: int, dtype: str = "f32", sd: float = 1.0, stream_base: int = 1 << 40):
    out = np.empty((rows, c), dtype=_np_dtype(dtype))
    scale = np.empty(rows, dtype=np.float32) if dtype == "f8" else None
    _load().disc_gen_normal_rows(seed, stream_base, rows, c, sd, _DTYPE_CODES[dtype], _ptr(out),
                                 _ptr(scale) if scale is not None else None)
    return out, scale


def tokens_normal(seed: int, gh: int, gw: int, c: int, dtype: str = "f32", patch: int = 16) -> Tokens:
    data, scale = normal_rows(seed, gh * gw, c, dtype)
    return Tokens(data.reshape(gh, gw, c), dtype, scale, patch)


def quantize(values: np.ndarray, dtype: str):
    """Quantise a double array [G][C] the way a caller hands tokens over."""
    v = np.ascontiguousarray(values, dtype=np.float64)
    if dtype == "f32":
        return v.astype(np.float32), None
    if dtype == "f64":
        return v.copy(), None
    if dtype == "bf16":
        out = np.empty(v.shape, dtype=np.uint16)
        _load().disc_gen_quantize_bf16(_ptr(v), v.size, _ptr(out))
        return out, None
    if dtype == "f8":
        G = int(np.prod(v.shape[:-1]))
        C = v.shape[-1]
        q = np.empty(v.shape, dtype=np.uint8)
        sc = np.empty(G, dtype=np.float32)
        _load().disc_gen_quantize_fp8_rows(_ptr(v), G, C, _ptr(q), _ptr(sc))
        return q, sc
    raise ValueError(dtype)


def quantize_e4m3_codes(values: np.ndarray) -> np.ndarray:
    v = np.ascontiguousarray(values, dtype=np.float64)
    out = np.empty(v.shape, dtype=np.uint8)
    _load().disc_gen_quantize_e4m3(_ptr(v), v.size, _ptr(out))
    return out


def tokens_structured(seed: int, gh: int, gw: int, c: int, dtype: str = "f32", patch: int = 16,
                      regions: int = 6, noise: float = 0.1, outliers: int = 3, gain: float = 5.0) -> Tokens:
    vals = np.empty((gh * gw, c), dtype=np.float64)
    _load().disc_gen_structured_tokens(seed, gh, gw, c, regions, noise, outliers, gain, _ptr(vals))
    data, scale = quantize(vals, dtype)
    return Tokens(data.reshape(gh, gw, c), dtype, scale, patch)


def tokens_from_values(values: np.ndarray, dtype: str, patch: int) -> Tokens:
    gh, gw, c = values.shape
    data, scale = quantize(values.reshape(gh * gw, c), dtype)
    return Tokens(data.reshape(gh, gw, c), dtype, scale, patch)


def projection(seed: int, c: int, e: int, dtype: str = "f32") -> np.ndarray:
    """P[c][e] ~ N(0, 1/c)."""
    out, _ = normal_rows(seed, c, e, dtype, sd=1.0 / np.sqrt(c), stream_base=1 << 41)
    return out


def poisson_counts(seed: int, n: int, mean: float, lo: int, hi: int) -> np.ndarray:
    out = np.empty(n, dtype=np.int32)
    _load().disc_gen_poisson_counts(seed, n, mean, lo, hi, _ptr(out))
    return out


def exponential_gaps(seed: int, stream: int, n: int, mean: float) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    _load().disc_gen_exponential(seed, stream, n, mean, _ptr(out))
    return out


# ---------------------------------------------------------------- workloads

BASE_SEED = 20260303


def frame_seed(cfg: int, frame: int) -> int:
    return BASE_SEED + 1000 * cfg + frame


@dataclass
class Frame:
    tokens: Tokens
    bits: np.ndarray  # [m][h][wq] uint64
    h: int
    w: int

    @property
    def m(self):
        return self.bits.shape[0]


@dataclass
class Workload:
    name: str
    frames: List[Frame]
    proj: np.ndarray
    proj_dtype: str
    meta: dict = field(default_factory=dict)

    @property
    def total_masks(self):
        return sum(f.m for f in self.frames)


def make_frame(cfg: int, frame: int, h: int, w: int, m: int, patch: int, c: int, dtype: str,
               kind: str = "mixed", lo: float = 1e-3, hi: float = 0.30) -> Frame:
    s = frame_seed(cfg, frame)
    if kind == "ellipses":
        bits = masks_ellipses(s, m, h, w, 10.0, 120.0)
    else:
        bits = masks_mixed(s, m, h, w, lo, hi)
    gh, gw = -(-h // patch), -(-w // patch)
    return Frame(tokens_normal(s, gh, gw, c, dtype, patch), bits, h, w)


def workload(name: str, frames: Optional[int] = None) -> Workload:
    """The synthetic stand-ins described in the module docstring."""
    if name == "cfg1":
        f = make_frame(1, 0, 336, 336, 8, 14, 1024, "f32", kind="ellipses")
        return Workload(name, [f], projection(frame_seed(1, 999), 1024, 768, "f32"), "f32")
    if name == "cfg2":
        f = make_frame(2, 0, 480, 640, 128, 16, 1024, "f32")
        return Workload(name, [f], projection(frame_seed(2, 999), 1024, 768, "f32"), "f32")
    if name == "cfg3":
        n = 64 if frames is None else frames
        counts = poisson_counts(frame_seed(3, 998), n, 60.0, 1, 300)
        fr = [make_frame(3, i, 480, 640, int(counts[i]), 16, 1024, "bf16") for i in range(n)]
        return Workload(name, fr, projection(frame_seed(3, 999), 1024, 768, "bf16"), "bf16")
    if name == "cfg4":
        n = 32 if frames is None else frames
        counts = poisson_counts(frame_seed(4, 998), n, 80.0, 1, 300)
        fr = []
        for i in range(n):
            big = (i % 16) >= 8  # streams 8..15 carry 720x1280 frames
            h, w = (720, 1280) if big else (480, 640)
            fr.append(make_frame(4, i, h, w, int(counts[i]), 16, 1024, "bf16"))
        return Workload(name, fr, projection(frame_seed(4, 999), 1024, 768, "bf16"), "bf16")
    if name == "cfg5":
        n = 16 if frames is None else frames
        fr = [make_frame(5, i, 1080, 1920, 500, 16, 1280, "f8", lo=1e-4, hi=0.20) for i in range(n)]
        return Workload(name, fr, projection(frame_seed(5, 999), 1280, 1024, "bf16"), "bf16")
    raise ValueError(name)
