"""A synthetic object scene with known per-object features, for comparing
the weighting modes (crop-free distance/distinctiveness weighting against the
naive average over the mask).

A frame holds overlapping filled ellipses (drawn in order, later ones occlude
earlier ones) on a background.  Every object k and the background own a
feature vector phi_k ~ N(0, I_C).  The token of patch p is the coverage-
weighted mix of the features of the pixels it holds (a patch on an object's
outline mixes that object with its neighbours, as a ViT token does), plus
N(0, noise^2) per channel, plus a few high-norm outlier tokens (gain * N(0, I)
added at random patches).  The instance masks are the visible pixels of each
object; the reference feature of mask k is phi_k.

Only inputs are drawn here (label image, features, tokens); nothing of the
method is computed.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import Frame, pack_masks, tokens_from_values


@dataclass
class Scene:
    frame: Frame
    truth: np.ndarray  # [m][c] reference feature of each mask (FP64)


def object_scene(seed: int, h: int = 480, w: int = 640, patch: int = 16, c: int = 1024, n_obj: int = 40,
                 noise: float = 0.5, outliers: int = 12, gain: float = 6.0, min_area: int = 64,
                 dtype: str = "f32") -> Scene:
    rng = np.random.default_rng(seed)
    label = np.zeros((h, w), dtype=np.int32)
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64) + 0.5
    for k in range(1, n_obj + 1):
        cy, cx = rng.uniform(0, h), rng.uniform(0, w)
        a = float(np.exp(rng.uniform(np.log(12.0), np.log(140.0))))
        b = a * rng.uniform(0.35, 1.0)
        th = rng.uniform(0.0, np.pi)
        dy, dx = yy - cy, xx - cx
        u = dx * np.cos(th) + dy * np.sin(th)
        v = -dx * np.sin(th) + dy * np.cos(th)
        label[(u / a) ** 2 + (v / b) ** 2 <= 1.0] = k
    gh, gw = -(-h // patch), -(-w // patch)
    phi = rng.standard_normal((n_obj + 1, c))  # row 0: background
    # coverage of each patch by each label
    cover = np.zeros((gh * gw, n_obj + 1))
    pid = (np.arange(h)[:, None] // patch) * gw + (np.arange(w)[None, :] // patch)
    np.add.at(cover, (pid.ravel(), label.ravel()), 1.0)
    cover /= cover.sum(axis=1, keepdims=True)
    tok = cover @ phi + noise * rng.standard_normal((gh * gw, c))
    for p in rng.choice(gh * gw, size=outliers, replace=False):
        tok[p] += gain * rng.standard_normal(c)
    keep = [k for k in range(1, n_obj + 1) if int((label == k).sum()) >= min_area]
    u8 = np.stack([(label == k).astype(np.uint8) for k in keep]) if keep else np.zeros((0, h, w), np.uint8)
    frame = Frame(tokens_from_values(tok.reshape(gh, gw, c), dtype, patch), pack_masks(u8), h, w)
    return Scene(frame, phi[keep] if keep else np.zeros((0, c)))
