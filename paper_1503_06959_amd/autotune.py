"""Autotuner for the batched tick and the full-frame detection pass.

Two tunables, neither of which ever changes results (the GPU tests check
that every choice gives identical keypoints):

- the side of the level-0 tiles of the pyramid/difference pass (32, 64 or
  128 pixels, at least 2^(O-1)): how that pass maps onto workgroups and XCD
  L2s; timed on a short batched run of synthetic streams;
- the cells per workgroup (a rectangle of group_cols x group_rows cells)
  and the workgroup size (256 or 512 threads) of the detection pass when
  every cell is marked (full-frame chunks), the pass that dominates
  full-frame time; timed on a full-frame chunk of synthetic frames.

For each resolution class (W, H, O, grid) the tuner times each candidate
and keeps the fastest; choices are cached per GPU architecture in a JSON
file.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, List, Optional, Tuple

import numpy as np
import torch

from . import kpd, synth

CACHE = os.environ.get("KPD_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "kpd", "tune.json"))
TILES = (32, 64, 128)


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def class_key(width: int, height: int, det: synth.Detector) -> str:
    return f"{width}x{height}/O{det.n_octaves}/{det.grid_cols}x{det.grid_rows}"


def candidates(det: synth.Detector) -> List[int]:
    return [t for t in TILES if t >= (1 << (det.n_octaves - 1))]


def _load() -> Dict[str, Dict[str, int]]:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(cache: Dict[str, Dict[str, int]]) -> None:
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def time_class(width: int, height: int, det: synth.Detector, tile: int, n_streams: int = 8,
               n_ticks: int = 12, frames: Optional[np.ndarray] = None) -> float:
    """Seconds per tick of n_streams streams of one class with this tile."""
    from .batch import Batch
    if frames is None:
        _, m, smin, smax, sig = synth.RES_PRESETS.get((width, height), (det, 20, 10, 60, 2.0))
        frames = synth.make_video(synth.Scene(width, height, 8, m, smin, smax, 0.5, sig, False, 7000), 8)
    dev = torch.from_numpy(frames).cuda()
    b = Batch(max_streams=n_streams)
    p = kpd.make_params(det.fast_t, det.n_octaves, det.grid_cols, det.grid_rows, det.id_thresh, det.kb_thresh,
                        tile)
    streams = [b.open_stream(width, height, p) for _ in range(n_streams)]
    f = len(dev)
    with torch.cuda.stream(b.torch_stream):
        for k in range(3 + n_ticks):
            if k == 3:
                b.synchronize()
                t0 = time.perf_counter()
            i = k % (2 * f - 2) if f > 1 else 0
            i = i if i < f else 2 * f - 2 - i
            for s in streams:
                b.push(s, dev[i], retain=True)
            b.tick()
        b.synchronize()
    dt = (time.perf_counter() - t0) / n_ticks
    for s in streams:
        b.detach(s)
        s.close()
    b.close()
    return dt


def best_tile(width: int, height: int, det: synth.Detector, retune: bool = False) -> Tuple[int, Dict[int, float]]:
    """Fastest tile for this class, from the cache or by timing."""
    cache = _load()
    arch = _arch()
    key = class_key(width, height, det)
    if not retune and key in cache.get(arch, {}):
        return int(cache[arch][key]), {}
    times = {t: time_class(width, height, det, t) for t in candidates(det)}
    best = min(times, key=times.get)
    cache.setdefault(arch, {})[key] = best
    _save(cache)
    return best, times


GROUP_SHAPES = ((1, 1), (2, 1), (4, 1), (8, 1), (2, 2), (4, 2))
GROUP_THREADS = (256, 512)


def group_candidates(width: int, height: int, det: synth.Detector) -> List[Tuple[int, int, int]]:
    """(group_cols, group_rows, threads) that the library accepts for this class."""
    out = []
    for gx, gy in GROUP_SHAPES:
        if gx > det.grid_cols or gy > det.grid_rows:
            continue
        for nt in GROUP_THREADS:
            p = kpd.make_params(det.fast_t, det.n_octaves, det.grid_cols, det.grid_rows, -1, det.kb_thresh, 0, 16,
                                group_cols=gx, group_rows=gy, group_threads=nt)
            if kpd.lib.stream_bytes(width, height, kpd.ctypes.byref(p)) > 0:
                out.append((gx, gy, nt))
    return out


def time_groups(width: int, height: int, det: synth.Detector, groups: Tuple[int, int, int], n_frames: int = 64,
                reps: int = 3, frames: Optional[np.ndarray] = None) -> float:
    """Seconds per full-frame detection pass over n_frames frames in one chunk."""
    if frames is None:
        _, m, smin, smax, sig = synth.RES_PRESETS.get((width, height), (det, 20, 10, 60, 2.0))
        frames = synth.make_video(synth.Scene(width, height, n_frames, m, smin, smax, 0.5, sig, False, 7100))
    dev = torch.from_numpy(frames[:n_frames]).cuda()
    gx, gy, nt = groups
    p = kpd.make_params(det.fast_t, det.n_octaves, det.grid_cols, det.grid_rows, -1, det.kb_thresh, 0, len(dev),
                        group_cols=gx, group_rows=gy, group_threads=nt)
    s = kpd.Stream(width, height, p)
    s.push_chunk(dev)
    torch.cuda.synchronize()
    kpd.profile(s.handle, True)
    for _ in range(reps):
        s.push_chunk(dev)
    ms, n = kpd.profile_read(s.handle)
    s.close()
    return float(ms[1]) / max(1, int(n[1])) * 1e-3


def best_groups(width: int, height: int, det: synth.Detector,
                retune: bool = False) -> Tuple[Tuple[int, int, int], Dict[Tuple[int, int, int], float]]:
    """Fastest (group_cols, group_rows, threads) for this class, from the cache or by timing."""
    cache = _load()
    arch = _arch()
    key = "groups/" + class_key(width, height, det)
    if not retune and key in cache.get(arch, {}):
        return tuple(cache[arch][key]), {}
    times = {g: time_groups(width, height, det, g) for g in group_candidates(width, height, det)}
    best = min(times, key=times.get)
    cache.setdefault(arch, {})[key] = list(best)
    _save(cache)
    return best, times
