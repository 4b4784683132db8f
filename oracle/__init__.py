"""ctypes loader for the FP64 CPU oracle (``disc_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The HIP library never imports this
module and this module never imports the HIP library.

Each wrapper forwards to the C function of the same name; see
``disc_oracle.h`` for the readings of the paper it implements.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "disc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libdisc_oracle.so")

# -O2, no fast-math, single-threaded: the oracle is timed as it stands.
CFLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math"]


def build(force: bool = True, src: str = _SRC, out: str = _LIB_PATH) -> str:
    if force or not os.path.exists(out):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-I", _HERE, src, "-o", tmp, "-lm"])
        os.replace(tmp, out)
    return out


def _declare(lib):
    i32, i64, dbl, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    lib.disc_oracle_decode_bf16.argtypes = [vp, i64, vp]
    lib.disc_oracle_decode_bf16.restype = None
    lib.disc_oracle_decode_f32.argtypes = [vp, i64, vp]
    lib.disc_oracle_decode_f32.restype = None
    lib.disc_oracle_e4m3_value.argtypes = [ctypes.c_uint8]
    lib.disc_oracle_e4m3_value.restype = dbl
    lib.disc_oracle_decode_e4m3.argtypes = [vp, vp, i64, i64, vp]
    lib.disc_oracle_decode_e4m3.restype = None
    lib.disc_oracle_edt_sq.argtypes = [vp, i32, i32, vp]
    lib.disc_oracle_edt_sq_batch.argtypes = [vp, i32, i32, i32, vp]
    lib.disc_oracle_spatial_weights.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32, vp]
    lib.disc_oracle_token_stats.argtypes = [vp, i32, i32, dbl, vp, vp, vp]
    lib.disc_oracle_embed.argtypes = [vp, i32, i32, i32, i32, vp, i32, i32, i32, vp, i32, i32, i32, dbl,
                                      vp, vp, vp, vp, vp]
    lib.disc_oracle_pool_project.argtypes = [vp, i32, i32, vp, i32, vp, i32, vp, vp, vp]
    lib.disc_oracle_query_topk.argtypes = [vp, i32, vp, i32, i32, i32, vp, vp, vp]
    lib.disc_oracle_query_heatmap.argtypes = [vp, i32, i32, vp, i32, vp, i32, dbl, vp]
    lib.disc_oracle_mask_dbar.argtypes = [vp, i32, i32, i32, i32, i32, i32, vp, vp, vp]
    lib.disc_oracle_angle_score.argtypes = [vp, vp, vp, i32, vp]
    lib.disc_oracle_view_quality.argtypes = [vp, vp, vp, vp, vp, i32, i32, i32, i32, dbl, vp, vp]
    lib.disc_oracle_fuse.argtypes = [vp, vp, vp, i32, i32, vp, vp, i32, vp]
    for f in (lib.disc_oracle_edt_sq, lib.disc_oracle_edt_sq_batch, lib.disc_oracle_spatial_weights,
              lib.disc_oracle_token_stats, lib.disc_oracle_embed, lib.disc_oracle_pool_project,
              lib.disc_oracle_query_topk, lib.disc_oracle_query_heatmap, lib.disc_oracle_mask_dbar, lib.disc_oracle_angle_score,
              lib.disc_oracle_view_quality, lib.disc_oracle_fuse):
        f.restype = ctypes.c_int
    return lib


def _p(a):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"], "oracle inputs must be C-contiguous"
    return a.ctypes.data


def _check(rc):
    if rc != 0:
        raise ValueError("oracle rejected its arguments")


class Oracle:
    """Python face of one compiled oracle library."""

    def __init__(self, lib_path: str):
        self.path = lib_path
        self.lib = _declare(ctypes.CDLL(lib_path))

    def decode_tokens(self, data: np.ndarray, dtype: str, scale=None) -> np.ndarray:
        """Caller-format tokens [..][c] -> float64 values [G][c]."""
        data = np.ascontiguousarray(data)
        c = data.shape[-1]
        G = data.size // c
        out = np.empty((G, c), dtype=np.float64)
        lib = self.lib
        if dtype == "f32":
            lib.disc_oracle_decode_f32(_p(np.ascontiguousarray(data, dtype=np.float32)), data.size, _p(out))
        elif dtype == "bf16":
            lib.disc_oracle_decode_bf16(_p(np.ascontiguousarray(data, dtype=np.uint16)), data.size, _p(out))
        elif dtype == "f8":
            sc = np.ascontiguousarray(scale, dtype=np.float32)
            lib.disc_oracle_decode_e4m3(_p(np.ascontiguousarray(data, dtype=np.uint8)), _p(sc), G, c, _p(out))
        elif dtype == "f64":
            out[:] = data.reshape(G, c)
        else:
            raise ValueError(dtype)
        return out

    def e4m3_value(self, code: int) -> float:
        return self.lib.disc_oracle_e4m3_value(code)

    def edt_sq(self, bits: np.ndarray, w: int) -> np.ndarray:
        bits = np.ascontiguousarray(bits, dtype=np.uint64)
        m, h, _ = bits.shape
        e = np.empty((m, h, w), dtype=np.int32)
        _check(self.lib.disc_oracle_edt_sq_batch(_p(bits), m, h, w, _p(e)))
        return e

    def spatial_weights(self, bits: np.ndarray, w: int, patch: int, spatial: int = 0) -> np.ndarray:
        bits = np.ascontiguousarray(bits, dtype=np.uint64)
        m, h, _ = bits.shape
        gh, gw = -(-h // patch), -(-w // patch)
        s = np.empty((m, gh * gw), dtype=np.float64)
        _check(self.lib.disc_oracle_spatial_weights(_p(bits), m, h, w, patch, gh, gw, spatial, _p(s)))
        return s

    def token_stats(self, f: np.ndarray, eps: float = 1e-6):
        f = np.ascontiguousarray(f, dtype=np.float64)
        G, C = f.shape
        mean, r, D = np.empty(C), np.empty(G), np.empty(G)
        _check(self.lib.disc_oracle_token_stats(_p(f), G, C, eps, _p(mean), _p(r), _p(D)))
        return mean, r, D

    def embed(self, f: np.ndarray, gh: int, gw: int, patch: int, bits: np.ndarray, w: int, P: np.ndarray,
              spatial: int = 0, distinct: int = 1, eps: float = 1e-6) -> dict:
        """The whole path for one frame.  f: [gh*gw][C] float64; P: [C][E] float64."""
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(gh * gw, -1)
        P = np.ascontiguousarray(P, dtype=np.float64)
        bits = np.ascontiguousarray(bits, dtype=np.uint64)
        m, h, _ = bits.shape
        C, E = f.shape[1], P.shape[1]
        assert P.shape[0] == C
        out, status = np.empty((m, E)), np.empty(m, dtype=np.int32)
        pooled, Z, wts = np.empty((m, C)), np.empty(m), np.empty((m, gh * gw))
        _check(self.lib.disc_oracle_embed(_p(f), gh, gw, C, patch, _p(bits), m, h, w, _p(P), E, spatial,
                                          distinct, eps, _p(out), _p(status), _p(pooled), _p(Z), _p(wts)))
        return {"out": out, "status": status, "pooled": pooled, "Z": Z, "wts": wts}

    def pool_project(self, f: np.ndarray, wts: np.ndarray, P: np.ndarray) -> dict:
        f = np.ascontiguousarray(f, dtype=np.float64)
        wts = np.ascontiguousarray(wts, dtype=np.float64)
        P = np.ascontiguousarray(P, dtype=np.float64)
        G, C = f.shape
        m, E = wts.shape[0], P.shape[1]
        out, status, pooled = np.empty((m, E)), np.empty(m, dtype=np.int32), np.empty((m, C))
        _check(self.lib.disc_oracle_pool_project(_p(f), G, C, _p(wts), m, _p(P), E, _p(out), _p(status),
                                                 _p(pooled)))
        return {"out": out, "status": status, "pooled": pooled}

    def query_topk(self, emb: np.ndarray, text: np.ndarray, k: int) -> dict:
        """R-QUERY: sim [q][m], top-k scores / indices [q][k] per query."""
        emb = np.ascontiguousarray(emb, dtype=np.float64)
        text = np.ascontiguousarray(text, dtype=np.float64)
        m, e = emb.shape
        q = text.shape[0]
        sim = np.zeros((q, m))
        scores = np.zeros((q, k))
        idx = np.zeros((q, k), dtype=np.int32)
        _check(self.lib.disc_oracle_query_topk(_p(emb), m, _p(text), q, e, k, _p(sim), _p(scores), _p(idx)))
        return {"sim": sim, "scores": scores, "idx": idx}

    def query_heatmap(self, f: np.ndarray, P: np.ndarray, text: np.ndarray, eps: float = 1e-6) -> np.ndarray:
        """R-HEAT: heat [q][G] = D_p cos(text_j, f_p^T P) for tokens f [G][C] (doubles)."""
        f = np.ascontiguousarray(f, dtype=np.float64)
        P = np.ascontiguousarray(P, dtype=np.float64)
        text = np.ascontiguousarray(text, dtype=np.float64)
        G, C = f.shape
        E = P.shape[1]
        q = text.shape[0]
        heat = np.zeros((q, G))
        _check(self.lib.disc_oracle_query_heatmap(_p(f), G, C, _p(P), E, _p(text), q, eps, _p(heat)))
        return heat

    def mask_dbar(self, bits: np.ndarray, w: int, patch: int, D: np.ndarray):
        """R-Q: (Dbar [m], area [m]) of each mask given the frame's D [G]."""
        bits = np.ascontiguousarray(bits)
        m, h, _ = bits.shape
        gh, gw = -(-h // patch), -(-w // patch)
        D = np.ascontiguousarray(D, dtype=np.float64)
        dbar = np.zeros(m)
        area = np.zeros(m, dtype=np.int32)
        _check(self.lib.disc_oracle_mask_dbar(_p(bits), m, h, w, patch, gh, gw, _p(D), _p(dbar), _p(area)))
        return dbar, area

    def angle_score(self, rays: np.ndarray, normals: np.ndarray, off: np.ndarray) -> np.ndarray:
        rays = np.ascontiguousarray(rays, dtype=np.float64)
        normals = np.ascontiguousarray(normals, dtype=np.float64)
        off = np.ascontiguousarray(off, dtype=np.int32)
        m = len(off) - 1
        out = np.zeros(m)
        _check(self.lib.disc_oracle_angle_score(_p(rays), _p(normals), _p(off), m, _p(out)))
        return out

    def view_quality(self, area, dbar, emb, g, angle, H: int, W: int, lam: float = 3.3):
        area = np.ascontiguousarray(area, dtype=np.int32)
        dbar = np.ascontiguousarray(dbar, dtype=np.float64)
        emb = np.ascontiguousarray(emb, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        ang = None if angle is None else np.ascontiguousarray(angle, dtype=np.float64)
        m, e = emb.shape
        Q = np.zeros(m)
        comp = np.zeros((m, 4))
        _check(self.lib.disc_oracle_view_quality(_p(area), _p(dbar), _p(emb), _p(g), _p(ang), m, e, H, W, lam,
                                                 _p(Q), _p(comp)))
        return Q, comp

    def fuse(self, ids, q, emb, map_q, map_emb):
        """R-FUSE on copies of the map; returns (map_q, map_emb, won)."""
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        q = np.ascontiguousarray(q, dtype=np.float64)
        emb = np.ascontiguousarray(emb, dtype=np.float64)
        mq = np.array(map_q, dtype=np.float64)
        me = np.array(map_emb, dtype=np.float64)
        m, e = emb.shape
        won = np.zeros(m, dtype=np.int32)
        _check(self.lib.disc_oracle_fuse(_p(ids), _p(q), _p(emb), m, e, _p(mq), _p(me), len(mq), _p(won)))
        return mq, me, won

    def proj_to_f64(self, P: np.ndarray, dtype: str) -> np.ndarray:
        """Caller-format projection [C][E] -> float64."""
        C, E = P.shape
        return self.decode_tokens(P.reshape(1, C, E), dtype).reshape(C, E)


_default = None


def get() -> Oracle:
    """The oracle built from disc_oracle.c (compiled on first use)."""
    global _default
    if _default is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        _default = Oracle(_LIB_PATH)
    return _default


def decode_tokens(data, dtype, scale=None):
    return get().decode_tokens(data, dtype, scale)


def e4m3_value(code):
    return get().e4m3_value(code)


def edt_sq(bits, w):
    return get().edt_sq(bits, w)


def spatial_weights(bits, w, patch, spatial=0):
    return get().spatial_weights(bits, w, patch, spatial)


def token_stats(f, eps=1e-6):
    return get().token_stats(f, eps)


def embed(*args, **kw):
    return get().embed(*args, **kw)


def pool_project(f, wts, P):
    return get().pool_project(f, wts, P)


def query_topk(emb, text, k):
    return get().query_topk(emb, text, k)


def query_heatmap(f, P, text, eps=1e-6):
    return get().query_heatmap(f, P, text, eps)


def mask_dbar(bits, w, patch, D):
    return get().mask_dbar(bits, w, patch, D)


def angle_score(rays, normals, off):
    return get().angle_score(rays, normals, off)


def view_quality(*args, **kw):
    return get().view_quality(*args, **kw)


def fuse(ids, q, emb, map_q, map_emb):
    return get().fuse(ids, q, emb, map_q, map_emb)


def proj_to_f64(P, dtype):
    return get().proj_to_f64(P, dtype)
