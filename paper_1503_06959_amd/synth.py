"""Seeded synthetic video scenes standing in for the paper's video sets.

The paper measures on hand-held VGA sequences (Stanford MAR, 640x480,
200 frames), the Rome Landmark queries (480x360 to 640x360, 24 fps) and the
MAR multi-object set (640x480); none of them is available here. These scenes
have the same shape of content for a corner detector: a smooth textured
background, flat objects with sharp corners that translate, global camera
pan, and per-frame sensor noise (Sec. 4, "Dataset").

This module only renders pixels. It holds none of the detection method's
arithmetic, so both the GPU path and the CPU oracle can consume its frames.

Recipe (all draws from one numpy PCG64 generator per scene, in this order):
  * background: U[0,255) i.i.d. float64, separable Gaussian blur sigma=3
    (radius 9, reflect padding), rounded to nearest, clipped to uint8;
  * objects, in index order: rectangle or disk with probability 1/2; a
    rectangle's w and h are drawn independently from U{s_min..s_max}, a disk's
    diameter from the same range; intensity U{0..255}; top-left uniform over
    the canvas. A disk covers the pixels whose centre lies within radius d/2
    of the disk centre;
  * motion: a random subset of round(M * move_frac) objects moves with an
    integer velocity drawn from U{-3..3}^2 per frame; the rest are static;
    objects may leave the frame;
  * pan (optional): on each frame after the first, with probability 1/2, the
    camera steps by U{-1,0,1}^2 px over a canvas with a 160 px margin;
  * noise: N(0, sigma_n^2) added per pixel per frame, rounded, clipped, uint8.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Tuple

import numpy as np
from scipy.ndimage import gaussian_filter1d

PAN_MARGIN = 160


@dataclasses.dataclass(frozen=True)
class Scene:
    width: int
    height: int
    frames: int
    n_objects: int
    size_min: int
    size_max: int
    move_frac: float = 0.5
    noise_sigma: float = 2.0
    pan: bool = False
    seed: int = 0


@dataclasses.dataclass(frozen=True)
class Detector:
    """Detector and mask settings: FAST threshold t, octave count O (levels
    0..O-1), the N_c x N_r cell grid, the intensity-difference threshold T_I
    (mean absolute difference per pixel) and the keypoint-binning threshold
    T_H (UINT32_MAX switches binning off)."""
    fast_t: int
    n_octaves: int
    grid_cols: int
    grid_rows: int
    id_thresh: int = 8
    kb_thresh: int = 0xFFFFFFFF


KB_OFF = 0xFFFFFFFF

# The five workloads. Single-stream scenes use seeds 1001..1003; batched
# streams use 4000 + s; serving clip banks use 5000 + i.
SCENES: Dict[str, Scene] = {
    "c1_320x240": Scene(320, 240, 30, 12, 10, 60, 0.5, 2.0, False, 1001),
    "c2_640x480": Scene(640, 480, 300, 40, 10, 60, 0.5, 2.0, True, 1002),
    "c3_1920x1080": Scene(1920, 1080, 300, 150, 20, 200, 0.5, 3.0, False, 1003),
}
DETECTORS: Dict[str, Detector] = {
    "c1_320x240": Detector(30, 3, 8, 6, 8, KB_OFF),
    "c2_640x480": Detector(20, 4, 16, 12, 8, KB_OFF),
    "c3_1920x1080": Detector(20, 5, 32, 18, 8, KB_OFF),
}

# Per-resolution presets for the multi-stream workloads.
RES_PRESETS: Dict[Tuple[int, int], Tuple[Detector, int, int, int, float]] = {
    # (W, H): (detector, n_objects, size_min, size_max, noise_sigma)
    (320, 240): (Detector(30, 3, 8, 6, 8, KB_OFF), 12, 10, 60, 2.0),
    (640, 480): (Detector(20, 4, 16, 12, 8, KB_OFF), 40, 10, 60, 2.0),
    (1280, 720): (Detector(20, 5, 32, 18, 8, KB_OFF), 150, 20, 200, 3.0),
    (1920, 1080): (Detector(20, 5, 32, 18, 8, KB_OFF), 150, 20, 200, 3.0),
}
MOTION_LEVELS = (0.0, 0.25, 0.75)


def batch_streams(n_frames: int = 120) -> List[Tuple[Scene, Detector]]:
    """The 64-stream mixed-resolution batch: streams 0-23 at 320x240, 24-47 at
    640x480, 48-63 at 1280x720; motion level 0/25/75 % by stream index mod 3."""
    out = []
    for s in range(64):
        res = (320, 240) if s < 24 else (640, 480) if s < 48 else (1280, 720)
        det, m, smin, smax, sig = RES_PRESETS[res]
        sc = Scene(res[0], res[1], n_frames, m, smin, smax, MOTION_LEVELS[s % 3], sig, False, 4000 + s)
        out.append((sc, det))
    return out


def _disk_mask(d: int) -> np.ndarray:
    r = d / 2.0
    c = np.arange(d) + 0.5
    return ((c[None, :] - r) ** 2 + (c[:, None] - r) ** 2) <= r * r


class _Renderer:
    def __init__(self, sc: Scene):
        self.sc = sc
        rng = np.random.Generator(np.random.PCG64(sc.seed))
        self.rng = rng
        margin = PAN_MARGIN if sc.pan else 0
        self.margin = margin
        cw, ch = sc.width + 2 * margin, sc.height + 2 * margin
        bg = rng.uniform(0.0, 255.0, size=(ch, cw))
        bg = gaussian_filter1d(bg, 3.0, axis=0, mode="reflect", truncate=3.0)
        bg = gaussian_filter1d(bg, 3.0, axis=1, mode="reflect", truncate=3.0)
        self.bg = np.clip(np.rint(bg), 0, 255).astype(np.float32)
        objs = []
        for _ in range(sc.n_objects):
            disk = bool(rng.random() < 0.5)
            if disk:
                d = int(rng.integers(sc.size_min, sc.size_max + 1))
                w = h = d
                shape = _disk_mask(d)
            else:
                w = int(rng.integers(sc.size_min, sc.size_max + 1))
                h = int(rng.integers(sc.size_min, sc.size_max + 1))
                shape = None
            val = float(rng.integers(0, 256))
            x0 = int(rng.integers(0, cw))
            y0 = int(rng.integers(0, ch))
            objs.append([x0, y0, w, h, val, shape, 0, 0])
        n_move = int(round(sc.n_objects * sc.move_frac))
        movers = rng.permutation(sc.n_objects)[:n_move]
        for i in movers:
            vx, vy = rng.integers(-3, 4, size=2)
            objs[i][6], objs[i][7] = int(vx), int(vy)
        self.objs = objs
        self.cam = [0, 0]
        self.n = 0

    def next_frame(self) -> np.ndarray:
        sc, rng, m = self.sc, self.rng, self.margin
        if sc.pan and self.n > 0 and rng.random() < 0.5:
            step = rng.integers(-1, 2, size=2)
            self.cam[0] = int(np.clip(self.cam[0] + step[0], -m, m))
            self.cam[1] = int(np.clip(self.cam[1] + step[1], -m, m))
        vx0, vy0 = m + self.cam[0], m + self.cam[1]
        W, H = sc.width, sc.height
        img = self.bg[vy0:vy0 + H, vx0:vx0 + W].copy()
        for (x0, y0, w, h, val, shape, vx, vy) in self.objs:
            # object top-left in view coordinates at this frame
            ox = x0 + vx * self.n - vx0
            oy = y0 + vy * self.n - vy0
            xa, xb = max(ox, 0), min(ox + w, W)
            ya, yb = max(oy, 0), min(oy + h, H)
            if xa >= xb or ya >= yb:
                continue
            if shape is None:
                img[ya:yb, xa:xb] = val
            else:
                sub = shape[ya - oy:yb - oy, xa - ox:xb - ox]
                img[ya:yb, xa:xb][sub] = val
        noise = rng.standard_normal(size=(H, W), dtype=np.float32) * np.float32(sc.noise_sigma)
        img += noise
        self.n += 1
        return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def make_video(sc: Scene, frames: int | None = None) -> np.ndarray:
    """Render the scene: uint8 array [F, H, W], row-major, pitch W."""
    f = sc.frames if frames is None else frames
    r = _Renderer(sc)
    out = np.empty((f, sc.height, sc.width), dtype=np.uint8)
    for i in range(f):
        out[i] = r.next_frame()
    return out


def clip_bank(width: int, height: int, n_clips: int = 4, frames: int = 240) -> np.ndarray:
    """Pre-rendered clips for the serving workload, seeds 5000 + i per
    resolution class: uint8 [n_clips, frames, H, W]."""
    det, m, smin, smax, sig = RES_PRESETS[(width, height)]
    base = {320: 0, 640: 100, 1280: 200, 1920: 300}[width]
    clips = [make_video(Scene(width, height, frames, m, smin, smax, 0.5, sig, False, 5000 + base + i))
             for i in range(n_clips)]
    return np.stack(clips)


def random_image(rng: np.random.Generator, h: int, w: int) -> np.ndarray:
    return rng.integers(0, 256, size=(h, w), dtype=np.uint8)
