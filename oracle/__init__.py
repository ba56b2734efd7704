"""CPU oracle for masked multi-scale FAST detection in video — TEST INFRASTRUCTURE.

A ctypes view of ``kpd_oracle.c`` (plain scalar C written from the paper's
definitions; every reading of the paper it takes is listed at the top of that
file). Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
CPU-baseline leg may import this package. The GPU library never does, and
shares no code with it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kpd_oracle.c")
LIB = os.path.join(HERE, "libkpd_oracle.so")
GCC_CMD = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-Wall", "-Wextra", "-shared", "-fPIC", "-o", LIB, SRC, "-lm"]

KP_DTYPE = np.dtype([("x", "<i4"), ("y", "<i4"), ("octave", "<i4"), ("score", "<i4")])
KB_OFF = 0xFFFFFFFF

_lib: Optional[ctypes.CDLL] = None


def build() -> str:
    subprocess.run(GCC_CMD, check=True)
    return LIB


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    # KPD_ORACLE_LIB names another build of the same source (the sanitizer
    # test loads an address/undefined-behaviour-checked one)
    path = os.environ.get("KPD_ORACLE_LIB")
    if not path:
        path = LIB
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, u32 = ctypes.c_int32, ctypes.c_uint32
    L.orc_level_dims.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P]
    L.orc_level_dims.restype = ctypes.c_long
    L.orc_pyramid.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P]
    L.orc_ring.argtypes = [ctypes.c_int, P, P]
    L.orc_arc9.argtypes = [ctypes.c_uint]
    L.orc_score_level.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P]
    L.orc_detect.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, ctypes.c_int]
    L.orc_cell_of.argtypes = [ctypes.c_int] * 7
    L.orc_open.argtypes = [ctypes.c_int] * 6 + [i32, u32]
    L.orc_open.restype = P
    L.orc_close.argtypes = [P]
    L.orc_close.restype = None
    L.orc_set_thresholds.argtypes = [P, ctypes.c_int, i32, u32]
    L.orc_reset.argtypes = [P]
    L.orc_set_id_mode.argtypes = [P, ctypes.c_int, ctypes.c_int]
    L.orc_push.argtypes = [P, P]
    L.orc_get.argtypes = [P, P, ctypes.c_int, P, P, P]
    L.orc_set_descriptors.argtypes = [P, ctypes.c_int]
    L.orc_get_desc.argtypes = [P, P, P, ctypes.c_int]
    L.orc_describe.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P]
    L.orc_desc_point.argtypes = [ctypes.c_int, ctypes.c_int, P, P]
    L.orc_set_refine.argtypes = [P, ctypes.c_int]
    L.orc_get_refined.argtypes = [P, P, ctypes.c_int]
    L.orc_refine_kp.argtypes = [P, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P]
    L.orc_refine_kp.restype = None
    L.orc_layer_dims.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P]
    L.orc_layer_dims.restype = ctypes.c_long
    L.orc_twothirds.argtypes = [P, ctypes.c_int, ctypes.c_int, P]
    L.orc_layers.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P]
    L.orc_layer_range.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P]
    L.orc_detect_layers.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, ctypes.c_int]
    L.orc_set_layers.argtypes = [P, ctypes.c_int]
    L.orc_set_lazy.argtypes = [P, ctypes.c_int]
    L.orc_refine_layers.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P]
    L.orc_tcd_sample.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.orc_tcd_spiral.argtypes = [ctypes.c_int, P, P]
    L.orc_tcd_track.argtypes = [P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P]
    L.orc_tcd_open.argtypes = [ctypes.c_int] * 9
    L.orc_tcd_open.restype = P
    L.orc_tcd_close.argtypes = [P]
    L.orc_tcd_close.restype = None
    L.orc_tcd_reset.argtypes = [P]
    L.orc_tcd_push.argtypes = [P, P]
    L.orc_tcd_get.argtypes = [P, P, ctypes.c_int]
    _lib = L
    return L


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def level_dims(W: int, H: int, O: int):
    ws = np.zeros(32, np.int32)
    hs = np.zeros(32, np.int32)
    lib().orc_level_dims(W, H, O, _ptr(ws), _ptr(hs))
    return [(int(ws[o]), int(hs[o])) for o in range(O)]


def pyramid(img: np.ndarray, O: int):
    """Levels 0..O-1 as a list of uint8 arrays."""
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = img.shape
    dims = level_dims(W, H, O)
    out = np.zeros(sum(w * h for w, h in dims), np.uint8)
    assert lib().orc_pyramid(_ptr(img), W, H, O, _ptr(out)) == 0
    levels, off = [], 0
    for w, h in dims:
        levels.append(out[off:off + w * h].reshape(h, w))
        off += w * h
    return levels


def ring():
    dx, dy = ctypes.c_int(), ctypes.c_int()
    out = []
    for k in range(16):
        lib().orc_ring(k, ctypes.byref(dx), ctypes.byref(dy))
        out.append((dx.value, dy.value))
    return out


def arc9(mask: int) -> bool:
    return bool(lib().orc_arc9(mask))


def score_level(level: np.ndarray, t: int) -> np.ndarray:
    level = np.ascontiguousarray(level, dtype=np.uint8)
    h, w = level.shape
    V = np.zeros((h, w), np.uint16)
    lib().orc_score_level(_ptr(level), w, h, t, _ptr(V))
    return V


def detect(img: np.ndarray, t: int, O: int) -> np.ndarray:
    """Full-frame detection F(I): structured array (x, y, octave, score),
    ordered by octave, y, x."""
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = img.shape
    cap = W * H + 16
    out = np.zeros(cap, KP_DTYPE)
    n = lib().orc_detect(_ptr(img), W, H, t, O, _ptr(out), cap)
    assert n >= 0, n
    return out[:n].copy()


def describe(level: np.ndarray, x: int, y: int):
    """Orientation sector and 512-bit descriptor (8 uint64 words) of the
    keypoint at (x, y) of a level image (R13-R15)."""
    level = np.ascontiguousarray(level, dtype=np.uint8)
    bits = np.zeros(8, np.uint64)
    b = lib().orc_describe(_ptr(level), level.shape[1], level.shape[0], x, y, _ptr(bits))
    return b, bits


def refine(levels, t: int, x: int, y: int, o: int):
    """Refined (x, y) in level-0 pixels, log2 scale and score of the
    keypoint (x, y) of level o (R17-R19); `levels` is the pyramid."""
    levels = [np.ascontiguousarray(l, dtype=np.uint8) for l in levels]
    O = len(levels)
    ptrs = (ctypes.c_void_p * 32)(*[l.ctypes.data for l in levels])
    ws = np.array([l.shape[1] for l in levels] + [0] * (32 - O), np.int32)
    hs = np.array([l.shape[0] for l in levels] + [0] * (32 - O), np.int32)
    out = np.zeros(4, np.float32)
    lib().orc_refine_kp(ptrs, _ptr(ws), _ptr(hs), O, t, x, y, o, _ptr(out))
    return out


def desc_pattern(b: int):
    """Rounded offsets (dx, dy) and box half-sizes of the 60 pattern points
    turned to sector b."""
    out = np.zeros((60, 3), np.int32)
    dx, dy = ctypes.c_int(), ctypes.c_int()
    for i in range(60):
        out[i, 2] = lib().orc_desc_point(b, i, ctypes.byref(dx), ctypes.byref(dy))
        out[i, 0], out[i, 1] = dx.value, dy.value
    return out


def cell_of(x: int, y: int, o: int, W: int, H: int, Nc: int, Nr: int) -> int:
    return lib().orc_cell_of(x, y, o, W, H, Nc, Nr)


class Stream:
    """The oracle's video stream: push frames, read D_n, the mask M_n, the
    per-cell SAD and the per-cell counts."""

    def __init__(self, W: int, H: int, t: int, O: int, Nc: int, Nr: int, TI: int, TH: int = KB_OFF):
        self.W, self.H, self.Nc, self.Nr = W, H, Nc, Nr
        self.h = lib().orc_open(W, H, t, O, Nc, Nr, TI, TH & 0xFFFFFFFF)
        if not self.h:
            raise ValueError("bad oracle stream parameters")

    def set_thresholds(self, t: int, TI: int, TH: int = KB_OFF):
        lib().orc_set_thresholds(self.h, t, TI, TH & 0xFFFFFFFF)

    def reset(self):
        lib().orc_reset(self.h)

    def set_id_mode(self, mode: int, layer: int = 0):
        """0: per-cell mean difference at level 0; 1: per-pixel difference on
        pyramid layer `layer`, Eq. 1 per feature position; 2: per-pixel
        difference on every level, each octave's features tested on their own
        level (layer 0)."""
        assert lib().orc_set_id_mode(self.h, mode, layer) == 0

    def push(self, frame: np.ndarray) -> int:
        frame = np.ascontiguousarray(frame, dtype=np.uint8)
        assert frame.shape == (self.H, self.W)
        n = lib().orc_push(self.h, _ptr(frame))
        assert n >= 0
        return n

    def get(self):
        nc = self.Nc * self.Nr
        n = lib().orc_get(self.h, None, 0, None, None, None)
        kps = np.zeros(max(n, 1), KP_DTYPE)
        mask = np.zeros(nc, np.uint8)
        sad = np.zeros(nc, np.int64)
        cnt = np.zeros(nc, np.uint32)
        n2 = lib().orc_get(self.h, _ptr(kps), len(kps), _ptr(mask), _ptr(sad), _ptr(cnt))
        assert n2 == n
        return kps[:n].copy(), mask, sad, cnt

    def set_descriptors(self, on: bool = True):
        """Keep a descriptor with every feature of D_n (R13-R16)."""
        lib().orc_set_descriptors(self.h, 1 if on else 0)

    def set_lazy(self, on: bool = True):
        """CPU-masked mode: score only what the marked cells' suppression
        reads (same results as the definitional mode)."""
        assert lib().orc_set_lazy(self.h, 1 if on else 0) == 0

    def set_layers(self, on: bool = True):
        """Detect over octaves and intra-octaves (L5) from the next frame on."""
        assert lib().orc_set_layers(self.h, 1 if on else 0) == 0

    def set_refine(self, on: bool = True):
        """Keep the refined position, log2 scale and score with every feature of D_n (R17-R19)."""
        lib().orc_set_refine(self.h, 1 if on else 0)

    def refined(self):
        """float32 [n, 4]: refined x, y (level-0 pixels), log2 scale and score of D_n."""
        n = lib().orc_get(self.h, None, 0, None, None, None)
        out = np.zeros((max(n, 1), 4), np.float32)
        assert lib().orc_get_refined(self.h, _ptr(out), max(n, 1)) == n
        return out[:n].copy()

    def descriptors(self):
        """(sectors int32 [n], descriptors uint64 [n, 8]) of D_n, in D_n's order."""
        n = lib().orc_get(self.h, None, 0, None, None, None)
        bits = np.zeros((max(n, 1), 8), np.uint64)
        bins = np.zeros(max(n, 1), np.int32)
        assert lib().orc_get_desc(self.h, _ptr(bits), _ptr(bins), max(n, 1)) == n
        return bins[:n].copy(), bits[:n].copy()

    def close(self):
        if self.h:
            lib().orc_close(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------- temporally coherent detector

TRACK_DTYPE = np.dtype([("x4", "<i4"), ("y4", "<i4"), ("octave", "<i4"), ("score", "<i4"), ("sad", "<i4")])


def tcd_sample(frame: np.ndarray, X: int, Y: int) -> int:
    """Bilinear sample of `frame` at quarter-pixel position (X, Y) (T3); -1
    when it needs pixels outside the frame."""
    frame = np.ascontiguousarray(frame, dtype=np.uint8)
    return lib().orc_tcd_sample(_ptr(frame), frame.shape[1], frame.shape[0], X, Y)


def tcd_spiral(k: int):
    """The k-th grid offset (u, v) of the spiral search order (T6)."""
    u, v = ctypes.c_int(), ctypes.c_int()
    assert lib().orc_tcd_spiral(k, ctypes.byref(u), ctypes.byref(v)) == 0
    return u.value, v.value


def tcd_track(prev: np.ndarray, cur: np.ndarray, tracks: np.ndarray, t_bm: int, t_et: int) -> np.ndarray:
    """One propagation step (T5-T7): the tracks of `prev` that match in `cur`."""
    prev = np.ascontiguousarray(prev, dtype=np.uint8)
    cur = np.ascontiguousarray(cur, dtype=np.uint8)
    tracks = np.ascontiguousarray(tracks, dtype=TRACK_DTYPE)
    out = np.zeros(max(len(tracks), 1), TRACK_DTYPE)
    H, W = prev.shape
    m = lib().orc_tcd_track(_ptr(prev), _ptr(cur), W, H, t_bm, t_et, _ptr(tracks), len(tracks), _ptr(out))
    return out[:m].copy()


class Tcd:
    """The oracle's temporally coherent detector (T1-T7): full-frame
    detection on the first frame of every group of `gop`, block-matching
    propagation on the others."""

    def __init__(self, W: int, H: int, t: int, O: int, Nc: int, Nr: int, gop: int = 10, t_bm: int = 1800,
                 t_et: int = 1000):
        self.W, self.H = W, H
        self.h = lib().orc_tcd_open(W, H, t, O, Nc, Nr, gop, t_bm, t_et)
        if not self.h:
            raise ValueError("bad oracle tracker parameters")

    def reset(self):
        lib().orc_tcd_reset(self.h)

    def push(self, frame: np.ndarray) -> int:
        frame = np.ascontiguousarray(frame, dtype=np.uint8)
        assert frame.shape == (self.H, self.W)
        return lib().orc_tcd_push(self.h, _ptr(frame))

    def tracks(self) -> np.ndarray:
        n = lib().orc_tcd_get(self.h, None, 0)
        out = np.zeros(max(n, 1), TRACK_DTYPE)
        assert lib().orc_tcd_get(self.h, _ptr(out), len(out)) == n
        return out[:n].copy()

    def close(self):
        if self.h:
            lib().orc_tcd_close(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------ intra-octave layers

def layer_dims(W: int, H: int, O: int):
    """[(w, h, pixel size in half level-0 pixels)] of the 2O layers c_0, d_0,
    c_1, d_1, ... (L1)."""
    ws, hs, S = (np.zeros(64, np.int32) for _ in range(3))
    lib().orc_layer_dims(W, H, O, _ptr(ws), _ptr(hs), _ptr(S))
    return [(int(ws[l]), int(hs[l]), int(S[l])) for l in range(2 * O)]


def twothirds(img: np.ndarray) -> np.ndarray:
    img = np.ascontiguousarray(img, dtype=np.uint8)
    h, w = img.shape
    out = np.zeros(((h // 3) * 2, (w // 3) * 2), np.uint8)
    lib().orc_twothirds(_ptr(img), w, h, _ptr(out))
    return out


def layers(img: np.ndarray, O: int):
    """The 2O layers (L1) as arrays, in scale order."""
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = img.shape
    dims = layer_dims(W, H, O)
    buf = np.zeros(sum(w * h for w, h, _ in dims) + 1, np.uint8)
    assert lib().orc_layers(_ptr(img), W, H, O, _ptr(buf)) == 0
    out, off = [], 0
    for w, h, _ in dims:
        out.append(buf[off:off + w * h].reshape(h, w).copy())
        off += w * h
    return out


def layer_range(S1: int, S2: int, x: int):
    lo, hi = ctypes.c_int(), ctypes.c_int()
    lib().orc_layer_range(S1, S2, x, ctypes.byref(lo), ctypes.byref(hi))
    return lo.value, hi.value


def detect_layers(img: np.ndarray, t: int, O: int) -> np.ndarray:
    """Full-frame detection over octaves and intra-octaves (L1-L3); the
    `octave` field holds the layer index (2i: c_i, 2i+1: d_i)."""
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = img.shape
    cap = W * H + 16
    out = np.zeros(cap, KP_DTYPE)
    n = lib().orc_detect_layers(_ptr(img), W, H, t, O, _ptr(out), cap)
    assert n >= 0
    return out[:n].copy()


def refine_layers(img: np.ndarray, t: int, O: int, kps: np.ndarray) -> np.ndarray:
    """float32 [n, 4]: refined x, y (level-0 pixels), log2 scale and score of
    keypoints of detect_layers (L4)."""
    img = np.ascontiguousarray(img, dtype=np.uint8)
    kps = np.ascontiguousarray(kps, dtype=KP_DTYPE)
    H, W = img.shape
    out = np.zeros((max(len(kps), 1), 4), np.float32)
    assert lib().orc_refine_layers(_ptr(img), W, H, t, O, _ptr(kps), len(kps), _ptr(out)) == 0
    return out[:len(kps)].copy()
