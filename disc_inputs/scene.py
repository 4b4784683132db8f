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


@dataclass
class DepthScene:
    depth: np.ndarray   # [h][w] float32 metres (0 = no reading)
    bits: np.ndarray    # [m][h][wq] uint64 masks (visible pixels of each object)
    h: int
    w: int
    camera: dict        # fx, fy, cx, cy, R [3][3] camera-to-world, t [3], depth_min, depth_max


def depth_scene(seed: int, h: int = 480, w: int = 640, n_obj: int = 40, noise: float = 0.002,
                outlier_frac: float = 0.003, invalid_frac: float = 0.01, min_area: int = 64) -> DepthScene:
    """An RGB-D frame of the same overlapping-ellipse objects: a tilted
    background plane at 4-5 m, each object a dome (0.8-4 m away, bulging up
    to 30 % of its size towards the camera).  Depth carries range-scaled
    Gaussian noise (noise * z^2), a fraction of outlier pixels (uniform
    0.3-6 m: the isolated points a denoising pass removes) and a fraction of
    missing readings (0).  Pinhole camera with f = 525 px at 640 px width and
    a fixed camera-to-world pose."""
    rng = np.random.default_rng(seed)
    label = np.zeros((h, w), dtype=np.int32)
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64) + 0.5
    depth = 4.5 + 0.5 * (yy / h)  # background plane
    for k in range(1, n_obj + 1):
        cy, cx = rng.uniform(0, h), rng.uniform(0, w)
        a = float(np.exp(rng.uniform(np.log(12.0), np.log(140.0))))
        b = a * rng.uniform(0.35, 1.0)
        th = rng.uniform(0.0, np.pi)
        z0 = rng.uniform(0.8, 4.0)
        bulge = rng.uniform(0.0, 0.3)
        dy, dx = yy - cy, xx - cx
        u = dx * np.cos(th) + dy * np.sin(th)
        v = -dx * np.sin(th) + dy * np.cos(th)
        r2 = (u / a) ** 2 + (v / b) ** 2
        inside = r2 <= 1.0
        label[inside] = k
        size_m = z0 * a / 525.0
        depth[inside] = z0 - bulge * size_m * (1.0 - r2[inside])
    depth = depth + noise * depth ** 2 * rng.standard_normal((h, w))
    out = rng.random((h, w)) < outlier_frac
    depth[out] = rng.uniform(0.3, 6.0, int(out.sum()))
    depth[rng.random((h, w)) < invalid_frac] = 0.0
    keep = [k for k in range(1, n_obj + 1) if int((label == k).sum()) >= min_area]
    u8 = np.stack([(label == k).astype(np.uint8) for k in keep]) if keep else np.zeros((0, h, w), np.uint8)
    f = 525.0 * w / 640.0
    ang = 0.3
    R = np.array([[1.0, 0.0, 0.0], [0.0, np.cos(ang), -np.sin(ang)], [0.0, np.sin(ang), np.cos(ang)]])
    cam = {"fx": f, "fy": f, "cx": w / 2.0 - 0.5, "cy": h / 2.0 - 0.5, "R": R, "t": np.array([1.5, -0.4, 1.2]),
           "depth_min": 0.1, "depth_max": 10.0}
    return DepthScene(depth.astype(np.float32), pack_masks(u8), h, w, cam)
