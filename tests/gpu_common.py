"""Helpers shared by the GPU tests: move generator inputs to the device and
compare the library with the oracle."""
from __future__ import annotations

import numpy as np

import disc_inputs as di
import oracle
from disc_inputs.device import dev_bits, dev_proj, dev_tokens  # noqa: F401

# Tolerances of the path against the FP64 oracle (per mask, cosine similarity).
COS_FP32 = 1.0 - 1e-6
COS_LOWP = 0.9995
REL_S = 1e-5  # spatial weights / residual norms (informative bound, FP32)


def torch():
    import torch as t

    return t


def frame_input(fr: di.Frame):
    import paper_2603_03935_amd as disc

    data, scale = dev_tokens(fr.tokens)
    return disc.FrameInput(data, dev_bits(fr.bits), fr.h, fr.w, fr.tokens.patch, scale)


def oracle_frame(fr: di.Frame, P: np.ndarray, pdtype: str, spatial=0, distinct=1, eps=1e-6, idx=None):
    """Oracle result for a frame (optionally only the masks in idx)."""
    tok = fr.tokens
    f64 = oracle.decode_tokens(tok.data, tok.dtype, tok.scale)
    P64 = oracle.proj_to_f64(P, pdtype)
    bits = fr.bits if idx is None else fr.bits[idx]
    return oracle.embed(f64, tok.gh, tok.gw, tok.patch, bits, fr.w, P64, spatial, distinct, eps)


def cosines(got: np.ndarray, want: np.ndarray) -> np.ndarray:
    ng = np.linalg.norm(got, axis=1)
    nw = np.linalg.norm(want, axis=1)
    return (got * want).sum(axis=1) / np.maximum(ng * nw, 1e-300)


def check_embeddings(got, status, ref, bound, what=""):
    """Per-mask cosine against the oracle; statuses must agree; zero rows
    where the oracle has them."""
    got = np.asarray(got, dtype=np.float64)
    st = np.asarray(status)
    assert np.array_equal(st, ref["status"]), f"{what}: status differs {st[:10]} vs {ref['status'][:10]}"
    okm = ref["status"] == 0
    assert not got[~okm].any(), f"{what}: non-zero rows for degenerate masks"
    if okm.any():
        c = cosines(got[okm], ref["out"][okm])
        assert c.min() >= bound, (f"{what}: min cos {c.min():.9f} < {bound} "
                                  f"(median {np.median(c):.9f}, worst masks {np.argsort(c)[:5]})")
        assert np.allclose(np.linalg.norm(got[okm], axis=1), 1.0, atol=1e-5)
        return c
    return np.array([])
