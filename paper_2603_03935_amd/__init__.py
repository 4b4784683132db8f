"""Python binding of libdisc (MI355X / gfx950): DISC's mask-aligned,
distance-weighted feature extraction (arXiv 2603.03935, Sec. III-C).

Argument marshalling only: every step runs in the HIP kernels of
``libdisc.so``; PyTorch provides device memory and the current stream.  There
is no fallback -- importing works without the library, but every call raises
if ``libdisc.so`` is missing.

Entry points mirror ``include/disc.h``:

* :func:`embed_masks`   one frame -> unit embeddings [m][e] (+ status, pooled)
* :func:`embed_frames`  a ragged batch of frames in one call
* :func:`edt_sq`, :func:`patch_weights`, :func:`token_stats`,
  :func:`pool_project`, :func:`pack_masks`  stage entry points
* :func:`query_topk`    open-vocabulary retrieval over the embeddings
* :func:`view_quality`, :func:`angle_score`, :func:`fuse`  view quality Q
  and replace-if-higher feature fusion
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdisc.so")

DISC_F32, DISC_BF16, DISC_F8E4M3 = 0, 1, 2
DISC_ERR_INVALID_ARGUMENT, DISC_ERR_LIMIT = 1, 9
# bytes of the device scratch array of disc_embed_masks_noalloc (DISC_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 64 << 20
SPATIAL_EDT, SPATIAL_AREA = 0, 1
STATUS_NAMES = {
    0: "DISC_OK", 1: "DISC_ERR_INVALID_ARGUMENT", 2: "DISC_ERR_SHAPE", 3: "DISC_ERR_UNSUPPORTED_DTYPE",
    4: "DISC_ERR_ALIGNMENT", 5: "DISC_ERR_OUT_OF_MEMORY", 6: "DISC_ERR_DEVICE", 7: "DISC_ERR_ADMISSION",
    8: "DISC_ERR_UNIMPLEMENTED", 9: "DISC_ERR_LIMIT",
}

# Every symbol include/disc.h declares (checked by the CPU test suite).
EXPORTS = [
    "disc_options_default", "disc_embed_masks", "disc_embed_masks_ex", "disc_embed_frames", "disc_embed_masks_noalloc",
    "disc_workspace_bytes", "disc_release_workspace", "disc_edt_sq", "disc_patch_weights",
    "disc_token_stats", "disc_pool_project", "disc_pack_masks", "disc_last_error", "disc_abi_version",
    "disc_trace_enable", "disc_trace_select", "disc_trace_reset", "disc_trace_read", "disc_trace_stage_name",
    "disc_server_config_default", "disc_server_create", "disc_server_submit", "disc_server_poll",
    "disc_server_wait", "disc_server_drain", "disc_server_get_stats", "disc_server_reset_stats",
    "disc_server_destroy",
    "disc_query_topk", "disc_query_heatmap", "disc_view_quality", "disc_angle_score", "disc_fuse",
    "disc_backproject_count", "disc_backproject", "disc_dbscan_denoise", "disc_voxelize", "disc_voxel_overlap",
]
STAGES = ["scan", "token_stats", "edt", "weights", "pool", "proj"]


class DiscError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


# ---------------------------------------------------------------- C structs

class Tokens(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("gh", ctypes.c_int32),
                ("gw", ctypes.c_int32), ("c", ctypes.c_int32), ("patch", ctypes.c_int32),
                ("scale", ctypes.c_void_p)]


class Masks(ctypes.Structure):
    _fields_ = [("bits", ctypes.c_void_p), ("m", ctypes.c_int32), ("h", ctypes.c_int32), ("w", ctypes.c_int32)]


class Proj(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("c", ctypes.c_int32), ("e", ctypes.c_int32)]


class Camera(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("depth_min", ctypes.c_float),
                ("depth_max", ctypes.c_float)]


def make_camera(cam: dict) -> Camera:
    """dict with fx, fy, cx, cy, R (3x3 camera-to-world), t (3), depth_min, depth_max."""
    c = Camera()
    c.fx, c.fy, c.cx, c.cy = cam["fx"], cam["fy"], cam["cx"], cam["cy"]
    R = [float(v) for row in cam["R"] for v in row]
    for k in range(9):
        c.R[k] = R[k]
    for k in range(3):
        c.t[k] = float(cam["t"][k])
    c.depth_min, c.depth_max = cam["depth_min"], cam["depth_max"]
    return c


class Out(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("m", ctypes.c_int32), ("e", ctypes.c_int32),
                ("mask_status", ctypes.c_void_p), ("pooled", ctypes.c_void_p),
                ("dbar", ctypes.c_void_p), ("area", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("spatial", ctypes.c_int32), ("distinct", ctypes.c_int32), ("eps", ctypes.c_float),
                ("gemm_dtype", ctypes.c_int32), ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("edt_layout", ctypes.c_int32), ("pool_tile", ctypes.c_int32), ("pool_rows", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("proj", Proj), ("tok_dtype", ctypes.c_int32), ("c", ctypes.c_int32),
                ("max_frames", ctypes.c_int32), ("max_masks", ctypes.c_int32), ("max_h", ctypes.c_int32),
                ("max_w", ctypes.c_int32), ("min_patch", ctypes.c_int32), ("max_slots", ctypes.c_int32),
                ("lanes", ctypes.c_int32), ("mem_budget", ctypes.c_size_t), ("use_graph", ctypes.c_int32),
                ("dry_run", ctypes.c_int32), ("fault_batch", ctypes.c_int32), ("admission_timeout_ms", ctypes.c_double),
                ("opts", Options)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("batches", ctypes.c_uint64), ("mean_batch_frames", ctypes.c_double),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("lanes", ctypes.c_int32), ("lane_workspace_bytes", ctypes.c_size_t)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libdisc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libdisc.so not found at {path}; build it with paper_2603_03935_amd/build.py")
    # PyTorch ships its own HIP runtime: load it first so that the library
    # binds to the same runtime instance as the tensors it is handed
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    lib.disc_options_default.argtypes = [P(Options)]
    lib.disc_options_default.restype = None
    lib.disc_embed_masks.argtypes = [P(Tokens), P(Masks), P(Proj), P(Out)]
    lib.disc_embed_masks_ex.argtypes = [P(Tokens), P(Masks), P(Proj), P(Out), P(Options), vp]
    lib.disc_embed_frames.argtypes = [P(Tokens), P(Masks), i32, P(Proj), P(Out), P(Options), vp]
    lib.disc_embed_masks_noalloc.argtypes = [P(Tokens), P(Masks), P(Proj), P(Out), P(Options), vp]
    lib.disc_workspace_bytes.argtypes = [P(Tokens), P(Masks), i32, P(Proj), P(Options)]
    lib.disc_workspace_bytes.restype = ctypes.c_size_t
    lib.disc_release_workspace.argtypes = []
    lib.disc_edt_sq.argtypes = [P(Masks), vp, vp]
    lib.disc_patch_weights.argtypes = [P(Tokens), P(Masks), i32, P(Options), vp, vp]
    lib.disc_token_stats.argtypes = [P(Tokens), ctypes.c_float, vp, vp, vp, vp]
    lib.disc_pool_project.argtypes = [P(Tokens), vp, i32, P(Proj), P(Out), i32, vp]
    lib.disc_pack_masks.argtypes = [vp, i32, i32, i32, vp, vp]
    lib.disc_query_topk.argtypes = [vp, i32, vp, i32, i32, i32, i32, vp, vp, vp, vp]
    lib.disc_query_heatmap.argtypes = [P(Tokens), P(Proj), vp, i32, i32, ctypes.c_float, vp, vp]
    lib.disc_view_quality.argtypes = [vp, vp, vp, vp, vp, i32, i32, i32, i32, ctypes.c_float, vp, vp, vp]
    lib.disc_angle_score.argtypes = [vp, vp, i32, vp, i32, vp, vp]
    lib.disc_fuse.argtypes = [vp, vp, vp, i32, i32, vp, vp, i32, vp, vp]
    lib.disc_backproject_count.argtypes = [vp, P(Masks), P(Camera), i32, vp, vp]
    lib.disc_backproject.argtypes = [vp, P(Masks), P(Camera), i32, vp, vp, vp]
    lib.disc_dbscan_denoise.argtypes = [vp, vp, i32, i32, ctypes.c_float, i32, vp, vp]
    lib.disc_voxelize.argtypes = [vp, vp, vp, i32, i32, ctypes.c_float, vp, vp, vp, vp]
    lib.disc_voxel_overlap.argtypes = [vp, vp, i32, vp, vp, i32, vp, i32, vp, vp]
    lib.disc_last_error.argtypes = []
    lib.disc_last_error.restype = ctypes.c_char_p
    lib.disc_trace_enable.argtypes = [i32]
    lib.disc_trace_enable.restype = None
    lib.disc_trace_select.argtypes = [ctypes.c_uint32]
    lib.disc_trace_select.restype = None
    lib.disc_trace_reset.argtypes = []
    lib.disc_trace_reset.restype = None
    lib.disc_trace_read.argtypes = [i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.disc_trace_read.restype = i32
    lib.disc_trace_stage_name.argtypes = [i32]
    lib.disc_trace_stage_name.restype = ctypes.c_char_p
    lib.disc_server_config_default.argtypes = [P(ServerConfig)]
    lib.disc_server_config_default.restype = None
    lib.disc_server_create.argtypes = [P(ServerConfig), P(vp)]
    lib.disc_server_submit.argtypes = [vp, P(Tokens), P(Masks), P(Out), P(ctypes.c_uint64)]
    lib.disc_server_poll.argtypes = [vp, ctypes.c_uint64, P(i32), P(i32)]
    lib.disc_server_wait.argtypes = [vp, ctypes.c_uint64, P(i32)]
    lib.disc_server_drain.argtypes = [vp]
    lib.disc_server_get_stats.argtypes = [vp, P(ServerStats)]
    lib.disc_server_reset_stats.argtypes = [vp]
    lib.disc_server_destroy.argtypes = [vp]
    lib.disc_server_destroy.restype = None
    for name in ("disc_server_create", "disc_server_submit", "disc_server_poll", "disc_server_wait",
                 "disc_server_drain", "disc_server_get_stats"):
        getattr(lib, name).restype = ctypes.c_int
    lib.disc_abi_version.argtypes = []
    lib.disc_abi_version.restype = i32
    for name in ("disc_embed_masks", "disc_embed_masks_ex", "disc_embed_frames", "disc_release_workspace",
                 "disc_edt_sq", "disc_patch_weights", "disc_token_stats", "disc_pool_project", "disc_pack_masks",
                 "disc_query_topk", "disc_query_heatmap", "disc_view_quality", "disc_angle_score", "disc_fuse",
                 "disc_backproject_count", "disc_backproject", "disc_dbscan_denoise", "disc_voxelize",
                 "disc_voxel_overlap"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        raise DiscError(status, load().disc_last_error().decode(errors="replace"))


def last_error() -> str:
    return load().disc_last_error().decode(errors="replace")


# ---------------------------------------------------------------- marshalling

def _torch():
    import torch

    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream_handle(stream=None) -> Optional[int]:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def token_dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float32:
        return DISC_F32
    if t.dtype == torch.bfloat16:
        return DISC_BF16
    if t.dtype in (torch.uint8, getattr(torch, "float8_e4m3fn", torch.uint8)):
        return DISC_F8E4M3
    raise TypeError(f"unsupported token dtype {t.dtype}")


def proj_dtype_code(p) -> int:
    torch = _torch()
    if p.dtype == torch.float32:
        return DISC_F32
    if p.dtype == torch.bfloat16:
        return DISC_BF16
    raise TypeError(f"unsupported projection dtype {p.dtype}")


def make_tokens(tokens, patch: int, scale=None) -> Tokens:
    gh, gw, c = tokens.shape
    assert tokens.is_contiguous()
    return Tokens(_ptr(tokens), token_dtype_code(tokens), gh, gw, c, patch, _ptr(scale))


def make_masks(bits, h: int, w: int) -> Masks:
    assert bits.is_contiguous() and bits.element_size() == 8
    return Masks(_ptr(bits), bits.shape[0], h, w)


def make_proj(proj) -> Proj:
    c, e = proj.shape
    assert proj.is_contiguous()
    return Proj(_ptr(proj), proj_dtype_code(proj), c, e)


def make_options(spatial: int = SPATIAL_EDT, distinct: int = 1, eps: float = 1e-6, gemm_dtype: int = -1,
                 workspace=None, edt_layout: int = -1, pool_tile: int = -1, pool_rows: int = -1) -> Options:
    o = Options()
    load().disc_options_default(ctypes.byref(o))
    o.spatial, o.distinct, o.eps, o.gemm_dtype = spatial, distinct, eps, gemm_dtype
    o.edt_layout = edt_layout
    o.pool_tile = pool_tile
    o.pool_rows = pool_rows
    if workspace is not None:
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    return o


@dataclass
class FrameInput:
    tokens: object       # torch tensor [gh][gw][c] (float32 / bfloat16 / uint8 e4m3fn codes), on the GPU
    bits: object         # torch int64 tensor [m][h][ceil(w/64)], on the GPU
    h: int
    w: int
    patch: int
    scale: object = None  # float32 [gh*gw] for FP8 tokens

    @property
    def m(self) -> int:
        return int(self.bits.shape[0])


@dataclass
class FrameOutput:
    out: object          # float32 [m][e]
    status: object       # int32 [m]
    pooled: object = None  # float32 [m][c] when requested
    dbar: object = None    # float32 [m] mean distinctiveness, when requested
    area: object = None    # int32 [m] pixel counts, when requested


def alloc_outputs(frames: Sequence[FrameInput], e: int, pooled: bool = False,
                  quality: bool = False) -> List[FrameOutput]:
    """Output buffers; quality=True adds dbar and area (the inputs of view_quality)."""
    torch = _torch()
    res = []
    for f in frames:
        m = f.bits.shape[0]
        dev = f.tokens.device
        res.append(FrameOutput(torch.empty((m, e), dtype=torch.float32, device=dev),
                               torch.empty((m,), dtype=torch.int32, device=dev),
                               torch.empty((m, f.tokens.shape[2]), dtype=torch.float32, device=dev) if pooled else None,
                               torch.empty((m,), dtype=torch.float32, device=dev) if quality else None,
                               torch.empty((m,), dtype=torch.int32, device=dev) if quality else None))
    return res


def _out(o: "FrameOutput") -> "Out":
    return Out(_ptr(o.out), o.out.shape[0], o.out.shape[1], _ptr(o.status), _ptr(o.pooled), _ptr(o.dbar),
               _ptr(o.area))


def embed_frames(frames: Sequence[FrameInput], proj, outputs: Optional[List[FrameOutput]] = None,
                 pooled: bool = False, options: Optional[Options] = None, stream=None,
                 quality: bool = False) -> List[FrameOutput]:
    """disc_embed_frames: one call for a ragged batch of frames."""
    lib = load()
    n = len(frames)
    e = proj.shape[1]
    if outputs is None:
        outputs = alloc_outputs(frames, e, pooled, quality)
    toks = (Tokens * max(n, 1))()
    msks = (Masks * max(n, 1))()
    outs = (Out * max(n, 1))()
    for i, (f, o) in enumerate(zip(frames, outputs)):
        toks[i] = make_tokens(f.tokens, f.patch, f.scale)
        msks[i] = make_masks(f.bits, f.h, f.w)
        outs[i] = _out(o)
    pj = make_proj(proj)
    opts = options if options is not None else make_options()
    _check(lib.disc_embed_frames(toks, msks, n, ctypes.byref(pj), outs, ctypes.byref(opts), _stream_handle(stream)))
    return outputs


def embed_masks(tokens, bits, h: int, w: int, proj, patch: int, scale=None, pooled: bool = False,
                options: Optional[Options] = None, stream=None, quality: bool = False) -> FrameOutput:
    """disc_embed_masks_ex for one frame."""
    return embed_frames([FrameInput(tokens, bits, h, w, patch, scale)], proj, pooled=pooled, options=options,
                        stream=stream, quality=quality)[0]


def embed_masks_noalloc(frame: FrameInput, proj, output: Optional[FrameOutput] = None, pooled: bool = False,
                        options: Optional[Options] = None, stream=None) -> FrameOutput:
    """disc_embed_masks_noalloc: one frame, working in the library's own
    device scratch array (no allocation inside the call)."""
    lib = load()
    if output is None:
        output = alloc_outputs([frame], proj.shape[1], pooled)[0]
    tk = make_tokens(frame.tokens, frame.patch, frame.scale)
    mk = make_masks(frame.bits, frame.h, frame.w)
    ot = _out(output)
    pj = make_proj(proj)
    opts = options if options is not None else make_options()
    _check(lib.disc_embed_masks_noalloc(ctypes.byref(tk), ctypes.byref(mk), ctypes.byref(pj), ctypes.byref(ot),
                                        ctypes.byref(opts), _stream_handle(stream)))
    return output


def workspace_bytes(frames: Sequence[FrameInput], proj, options: Optional[Options] = None) -> int:
    lib = load()
    n = len(frames)
    toks = (Tokens * max(n, 1))()
    msks = (Masks * max(n, 1))()
    for i, f in enumerate(frames):
        toks[i] = make_tokens(f.tokens, f.patch, f.scale)
        msks[i] = make_masks(f.bits, f.h, f.w)
    pj = make_proj(proj)
    opts = options if options is not None else make_options()
    return int(lib.disc_workspace_bytes(toks, msks, n, ctypes.byref(pj), ctypes.byref(opts)))


def edt_sq(bits, h: int, w: int, stream=None):
    """disc_edt_sq -> int32 [m][h][w]."""
    torch = _torch()
    m = bits.shape[0]
    e = torch.empty((m, h, w), dtype=torch.int32, device=bits.device)
    mk = make_masks(bits, h, w)
    _check(load().disc_edt_sq(ctypes.byref(mk), _ptr(e), _stream_handle(stream)))
    return e


def patch_weights(bits, h: int, w: int, patch: int, tokens=None, scale=None, spatial: int = SPATIAL_EDT,
                  distinct: int = 1, eps: float = 1e-6, stream=None, edt_layout: int = -1):
    """disc_patch_weights -> float32 [m][gh*gw]."""
    torch = _torch()
    m = bits.shape[0]
    gh, gw = -(-h // patch), -(-w // patch)
    out = torch.empty((m, gh * gw), dtype=torch.float32, device=bits.device)
    mk = make_masks(bits, h, w)
    tk = make_tokens(tokens, patch, scale) if tokens is not None else None
    opts = make_options(spatial, distinct, eps, edt_layout=edt_layout)
    _check(load().disc_patch_weights(ctypes.byref(tk) if tk is not None else None, ctypes.byref(mk), patch,
                                     ctypes.byref(opts), _ptr(out), _stream_handle(stream)))
    return out


def token_stats(tokens, patch: int, scale=None, eps: float = 1e-6, stream=None):
    """disc_token_stats -> (mean [c], r [G], D [G]) float32."""
    torch = _torch()
    gh, gw, c = tokens.shape
    mean = torch.empty((c,), dtype=torch.float32, device=tokens.device)
    r = torch.empty((gh * gw,), dtype=torch.float32, device=tokens.device)
    D = torch.empty((gh * gw,), dtype=torch.float32, device=tokens.device)
    tk = make_tokens(tokens, patch, scale)
    _check(load().disc_token_stats(ctypes.byref(tk), eps, _ptr(mean), _ptr(r), _ptr(D), _stream_handle(stream)))
    return mean, r, D


def pool_project(tokens, weights, proj, patch: int, scale=None, gemm_dtype: int = -1, pooled: bool = True,
                 stream=None) -> FrameOutput:
    """disc_pool_project with caller-given weights [m][gh*gw] (float32)."""
    torch = _torch()
    m = weights.shape[0]
    e = proj.shape[1]
    res = FrameOutput(torch.empty((m, e), dtype=torch.float32, device=tokens.device),
                      torch.empty((m,), dtype=torch.int32, device=tokens.device),
                      torch.empty((m, tokens.shape[2]), dtype=torch.float32, device=tokens.device) if pooled else None)
    tk = make_tokens(tokens, patch, scale)
    pj = make_proj(proj)
    out = Out(_ptr(res.out), m, e, _ptr(res.status), _ptr(res.pooled))
    _check(load().disc_pool_project(ctypes.byref(tk), _ptr(weights), m, ctypes.byref(pj), ctypes.byref(out),
                                    gemm_dtype, _stream_handle(stream)))
    return res


def pack_masks(u8, stream=None):
    """disc_pack_masks: uint8/bool [m][h][w] on the GPU -> int64 bits [m][h][ceil(w/64)]."""
    torch = _torch()
    m, h, w = u8.shape
    bits = torch.empty((m, h, (w + 63) // 64), dtype=torch.int64, device=u8.device)
    src = u8.to(torch.uint8).contiguous()
    _check(load().disc_pack_masks(_ptr(src), m, h, w, _ptr(bits), _stream_handle(stream)))
    return bits


def query_topk(emb, text, k: int, stream=None):
    """disc_query_topk -> (scores [q][k] float32, idx [q][k] int32, sim [q][m] float32)."""
    torch = _torch()
    m, e = emb.shape
    q = text.shape[0]
    sim = torch.empty((q, max(m, 1)), dtype=torch.float32, device=text.device)
    scores = torch.empty((q, k), dtype=torch.float32, device=text.device)
    idx = torch.empty((q, k), dtype=torch.int32, device=text.device)
    tdt = DISC_BF16 if text.dtype == torch.bfloat16 else DISC_F32
    _check(load().disc_query_topk(_ptr(emb), m, _ptr(text), tdt, q, e, k, _ptr(sim), _ptr(scores), _ptr(idx),
                                  _stream_handle(stream)))
    return scores, idx, sim[:, :m]


def query_heatmap(tokens, proj, text, patch: int, scale=None, eps: float = 1e-6, stream=None):
    """disc_query_heatmap: heat [q][gh][gw] = D_p cos(text_j, f_p^T P)."""
    lib = load()
    torch = _torch()
    gh, gw = tokens.shape[0], tokens.shape[1]
    q = text.shape[0]
    heat = torch.empty((q, gh, gw), dtype=torch.float32, device=tokens.device)
    tk = make_tokens(tokens, patch, scale)
    pj = make_proj(proj)
    tdt = DISC_BF16 if text.dtype == torch.bfloat16 else DISC_F32
    _check(lib.disc_query_heatmap(ctypes.byref(tk), ctypes.byref(pj), _ptr(text), tdt, q, eps, _ptr(heat),
                                  _stream_handle(stream)))
    return heat


def view_quality(area, dbar, emb, g, img_h: int, img_w: int, angle=None, lam: float = 3.3, stream=None):
    """disc_view_quality -> (q [m] float32, comp [m][4] float32: S_size, S_angle, S_sem, S_dist)."""
    torch = _torch()
    m, e = emb.shape
    q = torch.empty((m,), dtype=torch.float32, device=emb.device)
    comp = torch.empty((m, 4), dtype=torch.float32, device=emb.device)
    _check(load().disc_view_quality(_ptr(area), _ptr(dbar), _ptr(emb), _ptr(g), _ptr(angle), m, e, img_h, img_w,
                                    lam, _ptr(q), _ptr(comp), _stream_handle(stream)))
    return q, comp


def angle_score(rays, normals, off, stream=None):
    """disc_angle_score -> angle [m] float32 (rays, normals [nv][3]; off [m+1] int32)."""
    torch = _torch()
    m = off.shape[0] - 1
    angle = torch.empty((max(m, 0),), dtype=torch.float32, device=off.device)
    _check(load().disc_angle_score(_ptr(rays), _ptr(normals), rays.shape[0], _ptr(off), m, _ptr(angle),
                                   _stream_handle(stream)))
    return angle


def fuse(ids, q, emb, map_q, map_emb, won=None, stream=None):
    """disc_fuse: updates map_q / map_emb in place; returns won [m] int32."""
    torch = _torch()
    m, e = emb.shape
    if won is None:
        won = torch.empty((m,), dtype=torch.int32, device=emb.device)
    _check(load().disc_fuse(_ptr(ids), _ptr(q), _ptr(emb), m, e, _ptr(map_q), _ptr(map_emb), map_q.shape[0],
                            _ptr(won), _stream_handle(stream)))
    return won


def backproject(depth, bits, h: int, w: int, cam: dict, stride: int = 1, stream=None):
    """disc_backproject_count + disc_backproject -> (points [n][3] float32, offsets [m+1] int32).
    Synchronises once to size the point buffer."""
    torch = _torch()
    lib = load()
    m = bits.shape[0]
    mk = make_masks(bits, h, w)
    c = make_camera(cam)
    off = torch.empty((m + 1,), dtype=torch.int32, device=depth.device)
    sh = _stream_handle(stream)
    _check(lib.disc_backproject_count(_ptr(depth), ctypes.byref(mk), ctypes.byref(c), stride, _ptr(off), sh))
    n = int(off[m].item())
    pts = torch.empty((max(n, 1), 3), dtype=torch.float32, device=depth.device)
    _check(lib.disc_backproject(_ptr(depth), ctypes.byref(mk), ctypes.byref(c), stride, _ptr(off), _ptr(pts), sh))
    return pts[:n], off


def dbscan_denoise(points, offsets, eps: float, min_pts: int, stream=None):
    """disc_dbscan_denoise -> keep [n] int32."""
    torch = _torch()
    n, m = points.shape[0], offsets.shape[0] - 1
    keep = torch.empty((max(n, 1),), dtype=torch.int32, device=offsets.device)
    _check(load().disc_dbscan_denoise(_ptr(points), _ptr(offsets), m, n, eps, min_pts, _ptr(keep),
                                      _stream_handle(stream)))
    return keep[:n]


def voxelize(points, offsets, voxel: float, keep=None, stream=None):
    """disc_voxelize -> (voxels [nv][3] int32, voffsets [m+1] int32, status [m] int32).
    Synchronises once to trim the voxel buffer."""
    torch = _torch()
    n, m = points.shape[0], offsets.shape[0] - 1
    dev = offsets.device
    voff = torch.empty((m + 1,), dtype=torch.int32, device=dev)
    vox = torch.empty((max(n, 1), 3), dtype=torch.int32, device=dev)
    status = torch.empty((max(m, 1),), dtype=torch.int32, device=dev)
    _check(load().disc_voxelize(_ptr(points), _ptr(offsets), _ptr(keep), m, n, voxel, _ptr(voff), _ptr(vox),
                                _ptr(status), _stream_handle(stream)))
    nv = int(voff[m].item())
    return vox[:nv], voff, status[:m]


def voxel_overlap(va, oa, vb, ob, pairs, stream=None):
    """disc_voxel_overlap -> counts [np] int32."""
    torch = _torch()
    np_ = pairs.shape[0]
    out = torch.empty((max(np_, 1),), dtype=torch.int32, device=pairs.device)
    _check(load().disc_voxel_overlap(_ptr(va), _ptr(oa), oa.shape[0] - 1, _ptr(vb), _ptr(ob), ob.shape[0] - 1,
                                     _ptr(pairs), np_, _ptr(out), _stream_handle(stream)))
    return out[:np_]


def release_workspace():
    _check(load().disc_release_workspace())


def trace_enable(on: bool = True):
    load().disc_trace_enable(1 if on else 0)


def trace_select(stages=None):
    """Time only the named stages while tracing is on (None: all)."""
    mask = 0xFFFFFFFF if stages is None else sum(1 << STAGES.index(s) for s in stages)
    load().disc_trace_select(mask)


def trace_reset():
    load().disc_trace_reset()


def trace_read() -> dict:
    """{stage: (total_ms, launches)} since the last reset."""
    lib = load()
    res = {}
    for i, name in enumerate(STAGES):
        ms, n = ctypes.c_double(), ctypes.c_int64()
        lib.disc_trace_read(i, ctypes.byref(ms), ctypes.byref(n))
        res[name] = (ms.value, n.value)
    return res


# ---------------------------------------------------------------- serving

class Server:
    """disc_server_*: a continuous-batching request loop (see include/disc.h).

    Inputs of a submitted request must stay alive (and unchanged) until its
    ticket completes; this wrapper keeps references to them until then."""

    def __init__(self, proj=None, tok_dtype: int = DISC_BF16, c: int = 1024, e: int = 768, max_frames: int = 16,
                 max_masks: int = 1024, max_h: int = 720, max_w: int = 1280, min_patch: int = 14,
                 max_slots: int = 64, lanes: int = 2, mem_budget: int = 4 << 30, use_graph: bool = True,
                 dry_run: int = 0, fault_batch: int = -1, admission_timeout_ms: float = 0.0,
                 options: Optional[Options] = None):
        lib = load()
        cfg = ServerConfig()
        lib.disc_server_config_default(ctypes.byref(cfg))
        if proj is not None:
            cfg.proj = make_proj(proj)
        else:
            cfg.proj = Proj(None, DISC_BF16, c, e)
        cfg.tok_dtype, cfg.c = tok_dtype, c
        cfg.max_frames, cfg.max_masks, cfg.max_h, cfg.max_w = max_frames, max_masks, max_h, max_w
        cfg.min_patch, cfg.max_slots, cfg.lanes, cfg.mem_budget = min_patch, max_slots, lanes, mem_budget
        cfg.use_graph, cfg.dry_run, cfg.fault_batch = int(use_graph), dry_run, fault_batch
        cfg.admission_timeout_ms = admission_timeout_ms
        cfg.opts = options if options is not None else make_options()
        self._proj = proj
        self._keep = {}
        h = ctypes.c_void_p()
        _check(lib.disc_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.h = h
        self.e = cfg.proj.e

    def submit(self, tokens_struct: Tokens, masks_struct: Masks, out_struct: Out, keep=None) -> int:
        t = ctypes.c_uint64()
        _check(load().disc_server_submit(self.h, ctypes.byref(tokens_struct), ctypes.byref(masks_struct),
                                         ctypes.byref(out_struct), ctypes.byref(t)))
        self._keep[t.value] = keep
        return t.value

    def submit_frame(self, frame: FrameInput, output: Optional[FrameOutput] = None, quality: bool = False):
        """Submit one frame; returns (ticket, FrameOutput)."""
        if output is None:
            output = alloc_outputs([frame], self.e, quality=quality)[0]
        tk = make_tokens(frame.tokens, frame.patch, frame.scale)
        mk = make_masks(frame.bits, frame.h, frame.w)
        o = _out(output)
        return self.submit(tk, mk, o, keep=(frame, output)), output

    def poll(self, ticket: int):
        done, res = ctypes.c_int32(), ctypes.c_int32()
        _check(load().disc_server_poll(self.h, ticket, ctypes.byref(done), ctypes.byref(res)))
        if done.value:
            self._keep.pop(ticket, None)
        return bool(done.value), res.value

    def wait(self, ticket: int) -> int:
        res = ctypes.c_int32()
        _check(load().disc_server_wait(self.h, ticket, ctypes.byref(res)))
        self._keep.pop(ticket, None)
        return res.value

    def drain(self):
        _check(load().disc_server_drain(self.h))
        self._keep.clear()

    def stats(self) -> dict:
        st = ServerStats()
        _check(load().disc_server_get_stats(self.h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def reset_stats(self):
        """Restart counts and latency samples (e.g. after a warm-up)."""
        _check(load().disc_server_reset_stats(self.h))

    def close(self):
        if self.h:
            load().disc_server_destroy(self.h)
            self.h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
