"""Copies of the generator's host arrays into device memory (torch tensors).

Pure data movement: no arithmetic of the method happens here.  Used by the
GPU tests and by the benchmark to hand inputs to the library."""
from __future__ import annotations

import numpy as np


def _torch():
    import torch

    return torch


def dev_bits(bits: np.ndarray):
    """[m][h][wq] uint64 packed masks -> int64 device tensor (same bytes)."""
    t = _torch()
    return t.from_numpy(np.ascontiguousarray(bits).view(np.int64)).cuda()


def dev_tokens(tok):
    """Token map -> (data, scale) device tensors: FP32, BF16 (as bfloat16) or
    e4m3fn codes (uint8) with per-token FP32 scales."""
    t = _torch()
    if tok.dtype == "f32":
        data = t.from_numpy(np.ascontiguousarray(tok.data)).cuda()
    elif tok.dtype == "bf16":
        data = t.from_numpy(np.ascontiguousarray(tok.data).view(np.int16)).cuda().view(t.bfloat16)
    else:
        data = t.from_numpy(np.ascontiguousarray(tok.data)).cuda()
    scale = t.from_numpy(tok.scale).cuda() if tok.scale is not None else None
    return data, scale


def dev_proj(P: np.ndarray, dtype: str):
    """Projection [C][E] -> FP32 or bfloat16 device tensor."""
    t = _torch()
    if dtype == "f32":
        return t.from_numpy(np.ascontiguousarray(P)).cuda()
    return t.from_numpy(np.ascontiguousarray(P).view(np.int16)).cuda().view(t.bfloat16)
