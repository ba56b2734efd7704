"""Python binding of the gfx950 keypoint-detection library (include/kpd.h).

Argument marshalling only: every step of the detection path runs in the HIP
kernels of ``libkpd.so``. PyTorch supplies device memory (one uint8 arena
tensor per stream) and HIP streams. ``torch`` is imported before the library
is loaded so that both use the same HIP runtime.

The functions carry the C names: ``stream_bytes``, ``open_stream``,
``set_thresholds``, ``push_frame``, ``push_frames`` (a chunk of consecutive
frames), ``get_keypoints``, ``get_chunk_keypoints``, ``close_stream``,
``reset_stream``, the batch calls (``open_batch``, ``batch_attach``,
``batch_push``, ``batch_tick``, ``batch_gather``, ...), plus the inspection
calls ``cell_stats``, ``pyramid_level``, ``device_result``,
``chunk_result`` and ``profile``/``profile_read``. ``Stream`` wraps them for
one video stream.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np
import torch  # noqa: F401  (must precede loading libkpd.so: one HIP runtime)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkpd.so")

KPD_OK, KPD_EINVAL, KPD_ENOMEM, KPD_EDEVICE, KPD_ETRUNC, KPD_ESTATE = 0, -1, -2, -3, -4, -5
KPD_KB_OFF = 0xFFFFFFFF
FRAME_HOST, FRAME_DEVICE, FRAME_DEVICE_RETAIN = 0, 1, 2

KEYPOINT_DTYPE = np.dtype([("x", "<u2"), ("y", "<u2"), ("octave", "u1"), ("pad", "u1"), ("score", "<u2")])
EXPORTED = ("stream_bytes", "open_stream", "set_thresholds", "push_frame", "get_keypoints",
            "close_stream", "reset_stream", "kpd_last_error", "kpd_device_result", "kpd_cell_stats",
            "kpd_pyramid_level", "kpd_profile", "kpd_profile_read", "batch_bytes", "open_batch",
            "batch_attach", "batch_detach", "batch_push", "batch_push_many", "batch_tick", "batch_gather",
            "close_batch",
            "push_frames", "kpd_chunk_result", "get_chunk_keypoints", "set_mask_mode", "get_descriptors",
            "kpd_desc_point", "get_refined", "get_chunk_descriptors", "get_chunk_refined", "tcd_bytes", "tcd_open", "tcd_push", "tcd_get",
            "tcd_device_result", "tcd_reset", "tcd_close", "kpd_layers_bytes", "kpd_detect_layers",
            "kpd_detect_layers_static", "batch_set_single_launch",
            "kpd_layer_plane", "kpd_refine_layers", "kpd_lstream_bytes", "kpd_lstream_open", "kpd_lstream_push",
            "kpd_lstream_get", "kpd_lstream_reset", "kpd_lstream_close", "kpd_lstream_push_frames",
            "kpd_lstream_get_chunk", "kpd_lbatch_bytes", "kpd_lbatch_open", "kpd_lbatch_push", "kpd_lbatch_tick",
            "kpd_lbatch_get", "kpd_lbatch_reset", "kpd_lbatch_close")
DESCRIPTOR_DTYPE = np.dtype([("sector", "<u4"), ("pad", "<u4"), ("bits", "<u8", (8,))])
TRACK_DTYPE = np.dtype([("x4", "<i4"), ("y4", "<i4"), ("octave", "u1"), ("pad", "u1"), ("score", "<u2"),
                        ("sad", "<u4")])
REFINED_DTYPE = np.dtype([("x", "<f4"), ("y", "<f4"), ("log2_scale", "<f4"), ("score", "<f4")])
FEAT_DESCRIPTOR, FEAT_REFINE = 1, 2
STATIC_WORKSPACE = 16 << 20   # KPD_STATIC_WORKSPACE: bytes of kpd_detect_layers_static's workspace
KERNEL_NAMES = ("k_frame", "k_detect", "k_compact", "k_mark", "k_describe")


class KpdParams(ctypes.Structure):
    _fields_ = [("fast_t", ctypes.c_int32), ("n_octaves", ctypes.c_int32),
                ("grid_cols", ctypes.c_int32), ("grid_rows", ctypes.c_int32),
                ("id_thresh", ctypes.c_int32), ("kb_thresh", ctypes.c_uint32),
                ("tile", ctypes.c_int32), ("chunk_frames", ctypes.c_int32),
                ("layer_mask", ctypes.c_int32), ("features", ctypes.c_int32),
                ("group_cols", ctypes.c_int32), ("group_rows", ctypes.c_int32),
                ("group_threads", ctypes.c_int32)]


class KpdTcdParams(ctypes.Structure):
    _fields_ = [("gop", ctypes.c_int32), ("t_bm", ctypes.c_int32), ("t_et", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class KpdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"kpd error {code}: {msg}")
        self.code = code


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1503_06959_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, sz = ctypes.c_void_p, ctypes.c_size_t
    i32, u32 = ctypes.c_int32, ctypes.c_uint32
    L.stream_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(KpdParams)]
    L.stream_bytes.restype = sz
    L.open_stream.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(KpdParams), P, sz, P,
                              ctypes.POINTER(P)]
    L.set_thresholds.argtypes = [P, i32, i32, u32]
    L.push_frame.argtypes = [P, P, sz, ctypes.c_int]
    L.get_keypoints.argtypes = [P, P, sz, ctypes.POINTER(sz), P]
    L.close_stream.argtypes = [P]
    L.kpd_last_error.argtypes = []
    L.kpd_last_error.restype = ctypes.c_char_p
    L.kpd_device_result.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P)]
    L.kpd_cell_stats.argtypes = [P, P, P]
    L.kpd_pyramid_level.argtypes = [P, ctypes.c_int, P]
    L.reset_stream.argtypes = [P]
    L.kpd_profile.argtypes = [P, ctypes.c_int]
    L.kpd_profile_read.argtypes = [P, P, P]
    L.batch_bytes.argtypes = [ctypes.c_int, ctypes.c_int]
    L.batch_bytes.restype = sz
    L.open_batch.argtypes = [ctypes.c_int, ctypes.c_int, P, sz, P, ctypes.c_int, ctypes.POINTER(P)]
    L.batch_attach.argtypes = [P, P]
    L.batch_detach.argtypes = [P, P]
    L.batch_push.argtypes = [P, P, P, sz, ctypes.c_int]
    L.batch_push_many.argtypes = [P, ctypes.c_int, P, P, P, ctypes.c_int]
    L.batch_tick.argtypes = [P]
    L.batch_set_single_launch.argtypes = [P, ctypes.c_int]
    L.batch_gather.argtypes = [P, P, sz, P]
    L.close_batch.argtypes = [P]
    L.push_frames.argtypes = [P, P, sz, sz, ctypes.c_int]
    L.kpd_chunk_result.argtypes = [P, ctypes.c_int, ctypes.POINTER(P), ctypes.POINTER(P)]
    L.get_chunk_keypoints.argtypes = [P, ctypes.c_int, P, sz, ctypes.POINTER(sz)]
    L.set_mask_mode.argtypes = [P, ctypes.c_int, ctypes.c_int]
    L.get_descriptors.argtypes = [P, P, sz, ctypes.POINTER(sz)]
    L.get_refined.argtypes = [P, P, sz, ctypes.POINTER(sz)]
    L.get_chunk_descriptors.argtypes = [P, ctypes.c_int, P, sz, ctypes.POINTER(sz)]
    L.get_chunk_refined.argtypes = [P, ctypes.c_int, P, sz, ctypes.POINTER(sz)]
    L.kpd_layers_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.kpd_layers_bytes.restype = sz
    L.kpd_detect_layers.argtypes = [P, sz, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, sz, P, u32, P, P]
    L.kpd_detect_layers_static.argtypes = [P, sz, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, u32, P,
                                           P]
    L.kpd_refine_layers.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, sz, P, P, u32, P, P]
    L.kpd_lstream_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(KpdParams)]
    L.kpd_lstream_bytes.restype = sz
    L.kpd_lstream_open.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(KpdParams), P, sz, P, ctypes.POINTER(P)]
    L.kpd_lstream_push.argtypes = [P, P, sz, ctypes.c_int]
    L.kpd_lstream_get.argtypes = [P, P, sz, ctypes.POINTER(sz), P]
    L.kpd_lstream_push_frames.argtypes = [P, P, sz, sz, ctypes.c_int]
    L.kpd_lbatch_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(KpdParams), ctypes.c_int]
    L.kpd_lbatch_bytes.restype = sz
    L.kpd_lbatch_open.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(KpdParams), ctypes.c_int, P, sz, P,
                                  ctypes.POINTER(P)]
    L.kpd_lbatch_push.argtypes = [P, ctypes.c_int, P, sz]
    L.kpd_lbatch_tick.argtypes = [P]
    L.kpd_lbatch_get.argtypes = [P, ctypes.c_int, P, sz, ctypes.POINTER(sz), P]
    L.kpd_lbatch_reset.argtypes = [P, ctypes.c_int]
    L.kpd_lbatch_close.argtypes = [P]
    L.kpd_lstream_get_chunk.argtypes = [P, ctypes.c_int, P, sz, ctypes.POINTER(sz)]
    L.kpd_lstream_reset.argtypes = [P]
    L.kpd_lstream_close.argtypes = [P]
    L.kpd_layer_plane.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(sz),
                                  ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    TP = ctypes.POINTER(KpdTcdParams)
    L.tcd_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(KpdParams), TP]
    L.tcd_bytes.restype = sz
    L.tcd_open.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(KpdParams), TP, P, sz, P, ctypes.POINTER(P)]
    L.tcd_push.argtypes = [P, P, sz, ctypes.c_int]
    L.tcd_get.argtypes = [P, P, sz, ctypes.POINTER(sz)]
    L.tcd_device_result.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P)]
    L.tcd_reset.argtypes = [P]
    L.tcd_close.argtypes = [P]
    L.kpd_desc_point.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                 ctypes.POINTER(ctypes.c_int)]
    return L


lib = _load()


def _check(rc: int) -> int:
    if rc != KPD_OK:
        raise KpdError(rc, lib.kpd_last_error().decode())
    return rc


def make_params(fast_t: int, n_octaves: int, grid_cols: int, grid_rows: int,
                id_thresh: int = 8, kb_thresh: int = KPD_KB_OFF, tile: int = 0, chunk_frames: int = 0,
                layer_mask: int = 0, features: int = 0, group_cols: int = 0, group_rows: int = 0,
                group_threads: int = 0) -> KpdParams:
    """features: FEAT_DESCRIPTOR | FEAT_REFINE bits; group_cols x group_rows:
    cells per workgroup of full-frame chunk detection and group_threads its
    threads (0: defaults)."""
    return KpdParams(fast_t, n_octaves, grid_cols, grid_rows, id_thresh, kb_thresh & 0xFFFFFFFF, tile, chunk_frames,
                     layer_mask, features, group_cols, group_rows, group_threads)


def stream_bytes(width: int, height: int, params: KpdParams) -> int:
    n = lib.stream_bytes(width, height, ctypes.byref(params))
    if n == 0:
        raise KpdError(KPD_EINVAL, lib.kpd_last_error().decode())
    return n


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def open_stream(width: int, height: int, params: KpdParams, arena: torch.Tensor, stream=None) -> int:
    if arena.device.type != "cuda" or arena.dtype != torch.uint8 or not arena.is_contiguous():
        raise ValueError("arena must be a contiguous uint8 CUDA tensor")
    h = ctypes.c_void_p()
    _check(lib.open_stream(width, height, ctypes.byref(params), arena.data_ptr(), arena.numel(),
                           _stream_ptr(stream), ctypes.byref(h)))
    return h.value


def set_thresholds(handle: int, fast_t: int, id_thresh: int, kb_thresh: int = KPD_KB_OFF) -> None:
    _check(lib.set_thresholds(handle, fast_t, id_thresh, kb_thresh & 0xFFFFFFFF))


def push_frame(handle: int, frame, retain: bool = False) -> None:
    """frame: numpy uint8 [H, W] (host, copied) or a CUDA uint8 tensor
    [H, W] with unit column stride (copied, or read in place when `retain`)."""
    if isinstance(frame, np.ndarray):
        if frame.dtype != np.uint8 or frame.ndim != 2 or frame.strides[1] != 1:
            raise ValueError("host frame must be a uint8 [H, W] array with unit column stride")
        _check(lib.push_frame(handle, frame.ctypes.data, frame.strides[0], FRAME_HOST))
        return
    if not (isinstance(frame, torch.Tensor) and frame.device.type == "cuda" and frame.dtype == torch.uint8
            and frame.dim() == 2 and frame.stride(1) == 1):
        raise ValueError("device frame must be a CUDA uint8 [H, W] tensor with unit column stride")
    _check(lib.push_frame(handle, frame.data_ptr(), frame.stride(0),
                          FRAME_DEVICE_RETAIN if retain else FRAME_DEVICE))


def get_keypoints(handle: int, n_cells: int, capacity: int = 4096) -> Tuple[np.ndarray, np.ndarray]:
    """D_n as a structured array (x, y, octave, pad, score), and M_n."""
    mask = np.zeros(n_cells, np.uint8)
    out = np.zeros(max(capacity, 1), KEYPOINT_DTYPE)
    cnt = ctypes.c_size_t()
    rc = lib.get_keypoints(handle, out.ctypes.data, len(out), ctypes.byref(cnt), mask.ctypes.data)
    if rc == KPD_ETRUNC:
        out = np.zeros(cnt.value, KEYPOINT_DTYPE)
        rc = lib.get_keypoints(handle, out.ctypes.data, len(out), ctypes.byref(cnt), mask.ctypes.data)
    _check(rc)
    return out[:cnt.value].copy(), mask


def push_frames(handle: int, frames: torch.Tensor) -> None:
    """frames: CUDA uint8 tensor [n, H, W] with unit column stride, read in
    place (the caller keeps it alive until the next push)."""
    if not (isinstance(frames, torch.Tensor) and frames.device.type == "cuda" and frames.dtype == torch.uint8
            and frames.dim() == 3 and frames.stride(2) == 1):
        raise ValueError("frames must be a CUDA uint8 [n, H, W] tensor with unit column stride")
    _check(lib.push_frames(handle, frames.data_ptr(), frames.stride(0), frames.stride(1), frames.shape[0]))


def get_chunk_keypoints(handle: int, i: int, capacity: int = 4096) -> np.ndarray:
    out = np.zeros(max(capacity, 1), KEYPOINT_DTYPE)
    cnt = ctypes.c_size_t()
    rc = lib.get_chunk_keypoints(handle, i, out.ctypes.data, len(out), ctypes.byref(cnt))
    if rc == KPD_ETRUNC:
        out = np.zeros(cnt.value, KEYPOINT_DTYPE)
        rc = lib.get_chunk_keypoints(handle, i, out.ctypes.data, len(out), ctypes.byref(cnt))
    _check(rc)
    return out[:cnt.value].copy()


def chunk_result(handle: int, i: int) -> Tuple[int, int]:
    lst, cnt = ctypes.c_void_p(), ctypes.c_void_p()
    _check(lib.kpd_chunk_result(handle, i, ctypes.byref(lst), ctypes.byref(cnt)))
    return lst.value, cnt.value


def set_mask_mode(handle: int, mode: int, layer: int = 0) -> None:
    """0: per-cell mean difference at level 0; 1: per-pixel difference on
    pyramid layer `layer`, Eq. 1 per feature position; 2: per-pixel
    difference on every level, each octave's features tested on their own
    level (layer 0). Modes 1 and 2 run on single-frame pushes."""
    _check(lib.set_mask_mode(handle, mode, layer))


def _get_features(fn, dtype, handle: int, capacity: int) -> np.ndarray:
    out = np.zeros(max(capacity, 1), dtype)
    cnt = ctypes.c_size_t()
    rc = fn(handle, out.ctypes.data, len(out), ctypes.byref(cnt))
    if rc == KPD_ETRUNC:
        out = np.zeros(cnt.value, dtype)
        rc = fn(handle, out.ctypes.data, len(out), ctypes.byref(cnt))
    _check(rc)
    return out[:cnt.value].copy()


def get_descriptors(handle: int, capacity: int = 4096) -> np.ndarray:
    """Descriptors of D_n (DESCRIPTOR_DTYPE), in get_keypoints' order."""
    return _get_features(lib.get_descriptors, DESCRIPTOR_DTYPE, handle, capacity)


def get_refined(handle: int, capacity: int = 4096) -> np.ndarray:
    """Refined position, log2 scale and score of D_n's features
    (REFINED_DTYPE), in get_keypoints' order."""
    return _get_features(lib.get_refined, REFINED_DTYPE, handle, capacity)


def get_chunk_descriptors(handle: int, i: int, capacity: int = 4096) -> np.ndarray:
    """Descriptors of frame i of the last chunk, in get_chunk_keypoints' order."""
    return _get_features(lambda h, o, n, c: lib.get_chunk_descriptors(h, i, o, n, c), DESCRIPTOR_DTYPE, handle,
                         capacity)


def get_chunk_refined(handle: int, i: int, capacity: int = 4096) -> np.ndarray:
    """Refined values of frame i of the last chunk, in get_chunk_keypoints' order."""
    return _get_features(lambda h, o, n, c: lib.get_chunk_refined(h, i, o, n, c), REFINED_DTYPE, handle, capacity)


def desc_point(sector: int, i: int) -> Tuple[int, int, int]:
    """(dx, dy, box half-size) of the library's descriptor pattern point i
    turned to `sector`."""
    dx, dy = ctypes.c_int(), ctypes.c_int()
    h = lib.kpd_desc_point(sector, i, ctypes.byref(dx), ctypes.byref(dy))
    if h < 0:
        raise KpdError(KPD_EINVAL, "sector or point out of range")
    return dx.value, dy.value, h


def close_stream(handle: int) -> None:
    _check(lib.close_stream(handle))


def reset_stream(handle: int) -> None:
    _check(lib.reset_stream(handle))


def profile(handle: int, enable: bool) -> None:
    _check(lib.kpd_profile(handle, 1 if enable else 0))


def profile_read(handle: int) -> Tuple[np.ndarray, np.ndarray]:
    """Summed event-timed milliseconds and launch counts per kernel
    (KERNEL_NAMES order) since the last read."""
    ms = np.zeros(len(KERNEL_NAMES), np.float64)
    n = np.zeros(len(KERNEL_NAMES), np.uint64)
    _check(lib.kpd_profile_read(handle, ms.ctypes.data, n.ctypes.data))
    return ms, n


def cell_stats(handle: int, n_cells: int) -> Tuple[np.ndarray, np.ndarray]:
    sad = np.zeros(n_cells, np.uint32)
    cnt = np.zeros(n_cells, np.uint32)
    _check(lib.kpd_cell_stats(handle, sad.ctypes.data, cnt.ctypes.data))
    return sad, cnt


def pyramid_level(handle: int, octave: int, width: int, height: int) -> np.ndarray:
    out = np.zeros((height >> octave, width >> octave), np.uint8)
    _check(lib.kpd_pyramid_level(handle, octave, out.ctypes.data))
    return out


def device_result(handle: int) -> Tuple[int, int]:
    lst, cnt = ctypes.c_void_p(), ctypes.c_void_p()
    _check(lib.kpd_device_result(handle, ctypes.byref(lst), ctypes.byref(cnt)))
    return lst.value, cnt.value


def _frame_args(frame, retain: bool):
    if isinstance(frame, np.ndarray):
        if frame.dtype != np.uint8 or frame.ndim != 2 or frame.strides[1] != 1:
            raise ValueError("host frame must be a uint8 [H, W] array with unit column stride")
        return frame.ctypes.data, frame.strides[0], FRAME_HOST
    if not (isinstance(frame, torch.Tensor) and frame.device.type == "cuda" and frame.dtype == torch.uint8
            and frame.dim() == 2 and frame.stride(1) == 1):
        raise ValueError("device frame must be a CUDA uint8 [H, W] tensor with unit column stride")
    return frame.data_ptr(), frame.stride(0), FRAME_DEVICE_RETAIN if retain else FRAME_DEVICE


def batch_bytes(max_streams: int, max_blocks: int) -> int:
    return lib.batch_bytes(max_streams, max_blocks)


def open_batch(max_streams: int, max_blocks: int, scratch: torch.Tensor, stream, use_graph: bool = True) -> int:
    h = ctypes.c_void_p()
    _check(lib.open_batch(max_streams, max_blocks, scratch.data_ptr(), scratch.numel(), _stream_ptr(stream),
                          1 if use_graph else 0, ctypes.byref(h)))
    return h.value


def batch_attach(batch: int, handle: int) -> None:
    _check(lib.batch_attach(batch, handle))


def batch_detach(batch: int, handle: int) -> None:
    _check(lib.batch_detach(batch, handle))


def batch_push(batch: int, handle: int, frame, retain: bool = False) -> None:
    ptr, pitch, flags = _frame_args(frame, retain)
    _check(lib.batch_push(batch, handle, ptr, pitch, flags))


def batch_push_many(batch: int, handles, frame_ptrs, pitches, retain: bool = False) -> None:
    """Stage one device frame for each of several streams in one call:
    handles, frame_ptrs (device addresses of uint8 frames) and pitches
    (bytes) are equal-length sequences of ints."""
    n = len(handles)
    if len(frame_ptrs) != n or len(pitches) != n:
        raise ValueError("handles, frame_ptrs and pitches differ in length")
    h = np.asarray(handles, dtype=np.uint64)
    f = np.asarray(frame_ptrs, dtype=np.uint64)
    p = np.asarray(pitches, dtype=np.uint64)
    _check(lib.batch_push_many(batch, n, h.ctypes.data, f.ctypes.data, p.ctypes.data,
                               FRAME_DEVICE_RETAIN if retain else FRAME_DEVICE))


def batch_set_single_launch(batch: int, on: bool) -> None:
    _check(lib.batch_set_single_launch(batch, int(bool(on))))


def batch_tick(batch: int) -> None:
    _check(lib.batch_tick(batch))


def batch_gather(batch: int, out: torch.Tensor, counts: torch.Tensor) -> None:
    """out: CUDA uint8 tensor viewed as keypoint records (8 bytes each);
    counts: CUDA int32/uint32 tensor with one entry per attached stream."""
    _check(lib.batch_gather(batch, out.data_ptr(), out.numel() // 8, counts.data_ptr()))


def close_batch(batch: int) -> None:
    _check(lib.close_batch(batch))


class Stream:
    """One video stream: owns its device arena and keeps retained frames alive."""

    def __init__(self, width: int, height: int, params: KpdParams, stream=None, device="cuda"):
        self.width, self.height, self.params = width, height, params
        self.n_cells = params.grid_cols * params.grid_rows
        self.nbytes = stream_bytes(width, height, params)
        self.arena = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.stream = stream
        self.handle = open_stream(width, height, params, self.arena, stream)
        self._held = [None, None]
        self._out = None

    def push(self, frame, retain: bool = False) -> None:
        push_frame(self.handle, frame, retain)
        if retain:
            self._held = [self._held[1], frame]

    def push_chunk(self, frames: torch.Tensor) -> None:
        """Several consecutive frames [n, H, W] in one call (n <= chunk_frames)."""
        push_frames(self.handle, frames)
        self._held = [self._held[1], frames]

    def chunk_keypoints(self, i: int) -> np.ndarray:
        return get_chunk_keypoints(self.handle, i)

    def chunk_descriptors(self, i: int) -> np.ndarray:
        return get_chunk_descriptors(self.handle, i)

    def chunk_refined(self, i: int) -> np.ndarray:
        return get_chunk_refined(self.handle, i)

    def set_thresholds(self, fast_t: int, id_thresh: int, kb_thresh: int = KPD_KB_OFF) -> None:
        set_thresholds(self.handle, fast_t, id_thresh, kb_thresh)

    def set_mask_mode(self, mode: int, layer: int = 0) -> None:
        set_mask_mode(self.handle, mode, layer)

    def keypoints(self) -> Tuple[np.ndarray, np.ndarray]:
        """D_n (a copy) and M_n of the last push."""
        if self._out is None:
            self._out = np.zeros(4096, KEYPOINT_DTYPE)
        mask = np.zeros(self.n_cells, np.uint8)
        cnt = ctypes.c_size_t()
        rc = lib.get_keypoints(self.handle, self._out.ctypes.data, len(self._out), ctypes.byref(cnt),
                               mask.ctypes.data)
        if rc == KPD_ETRUNC:
            self._out = np.zeros(cnt.value, KEYPOINT_DTYPE)
            rc = lib.get_keypoints(self.handle, self._out.ctypes.data, len(self._out), ctypes.byref(cnt),
                                   mask.ctypes.data)
        _check(rc)
        return self._out[:cnt.value].copy(), mask

    def descriptors(self) -> np.ndarray:
        """Descriptors of D_n (streams opened with FEAT_DESCRIPTOR)."""
        return get_descriptors(self.handle)

    def refined(self) -> np.ndarray:
        """Refined values of D_n (streams opened with FEAT_REFINE)."""
        return get_refined(self.handle)

    def cell_stats(self):
        return cell_stats(self.handle, self.n_cells)

    def reset(self) -> None:
        reset_stream(self.handle)

    def level(self, octave: int) -> np.ndarray:
        return pyramid_level(self.handle, octave, self.width, self.height)

    def close(self) -> None:
        if self.handle:
            close_stream(self.handle)
            self.handle = None
            self._held = [None, None]

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------- temporally coherent detector

def tcd_bytes(width: int, height: int, params: KpdParams, tp: KpdTcdParams) -> int:
    n = lib.tcd_bytes(width, height, ctypes.byref(params), ctypes.byref(tp))
    if n == 0:
        raise KpdError(KPD_EINVAL, lib.kpd_last_error().decode())
    return n


class Tcd:
    """The temporally coherent detector (the comparison system of Sec. 4):
    full-frame detection on the first frame of every group of `gop` frames,
    block-matching propagation of the keypoints on the others."""

    def __init__(self, width: int, height: int, params: KpdParams, gop: int = 10, t_bm: int = 1800,
                 t_et: int = 1000, stream=None, device="cuda"):
        self.width, self.height = width, height
        self.tp = KpdTcdParams(gop, t_bm, t_et, 0)
        self.params = params
        self.nbytes = tcd_bytes(width, height, params, self.tp)
        self.arena = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        if self.arena.data_ptr() % 256:
            raise ValueError("arena not 256-byte aligned")
        h = ctypes.c_void_p()
        _check(lib.tcd_open(width, height, ctypes.byref(params), ctypes.byref(self.tp), self.arena.data_ptr(),
                            self.arena.numel(), _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h.value
        self._held = [None, None]

    def push(self, frame, retain: bool = False) -> None:
        """frame: as push_frame (host array, or CUDA tensor copied or read in
        place when `retain`; a retained frame is kept alive until the next
        push, which matches against it)."""
        if isinstance(frame, np.ndarray):
            if frame.dtype != np.uint8 or frame.ndim != 2 or frame.strides[1] != 1:
                raise ValueError("host frame must be a uint8 [H, W] array with unit column stride")
            _check(lib.tcd_push(self.handle, frame.ctypes.data, frame.strides[0], FRAME_HOST))
            return
        if not (isinstance(frame, torch.Tensor) and frame.device.type == "cuda" and frame.dtype == torch.uint8
                and frame.dim() == 2 and frame.stride(1) == 1):
            raise ValueError("device frame must be a CUDA uint8 [H, W] tensor with unit column stride")
        _check(lib.tcd_push(self.handle, frame.data_ptr(), frame.stride(0),
                            FRAME_DEVICE_RETAIN if retain else FRAME_DEVICE))
        if retain:
            self._held = [self._held[1], frame]

    def tracks(self, capacity: int = 4096) -> np.ndarray:
        out = np.zeros(max(capacity, 1), TRACK_DTYPE)
        cnt = ctypes.c_size_t()
        rc = lib.tcd_get(self.handle, out.ctypes.data, len(out), ctypes.byref(cnt))
        if rc == KPD_ETRUNC:
            out = np.zeros(cnt.value, TRACK_DTYPE)
            rc = lib.tcd_get(self.handle, out.ctypes.data, len(out), ctypes.byref(cnt))
        _check(rc)
        return out[:cnt.value].copy()

    def device_result(self):
        """(device pointer to the tracks, device pointer to their uint32 count)."""
        t, c = ctypes.c_void_p(), ctypes.c_void_p()
        _check(lib.tcd_device_result(self.handle, ctypes.byref(t), ctypes.byref(c)))
        return t.value, c.value

    def reset(self) -> None:
        _check(lib.tcd_reset(self.handle))

    def close(self) -> None:
        if self.handle:
            _check(lib.tcd_close(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------ octaves and intra-octaves

def layers_bytes(width: int, height: int, n_octaves: int) -> int:
    n = lib.kpd_layers_bytes(width, height, n_octaves)
    if n == 0:
        raise KpdError(KPD_EINVAL, lib.kpd_last_error().decode())
    return n


def layer_plane(width: int, height: int, n_octaves: int, layer: int) -> Tuple[int, int, int]:
    """(byte offset in the workspace, width, height) of layer `layer` >= 1."""
    off, w, h = ctypes.c_size_t(), ctypes.c_int(), ctypes.c_int()
    _check(lib.kpd_layer_plane(width, height, n_octaves, layer, ctypes.byref(off), ctypes.byref(w), ctypes.byref(h)))
    return off.value, w.value, h.value


class LayerDetector:
    """Full-frame detection over octaves and intra-octaves (Sec. 2) for
    frames of one size: owns the workspace, the output list and its count
    on the device."""

    def __init__(self, width: int, height: int, fast_t: int, n_octaves: int, capacity: int = 0,
                 stream=None, device="cuda"):
        self.width, self.height, self.fast_t, self.n_octaves = width, height, fast_t, n_octaves
        self.workspace = torch.empty(layers_bytes(width, height, n_octaves), dtype=torch.uint8, device=device)
        if capacity <= 0:   # at most one keypoint per 2 x 2 block of every layer
            capacity = 16
            for l in range(2 * n_octaves):
                w = (width >> (l // 2)) if l % 2 == 0 else (((width // 3) * 2) >> (l // 2))
                h = (height >> (l // 2)) if l % 2 == 0 else (((height // 3) * 2) >> (l // 2))
                capacity += ((w + 1) // 2) * ((h + 1) // 2)
        self.capacity = capacity
        self.out = torch.empty(capacity * KEYPOINT_DTYPE.itemsize, dtype=torch.uint8, device=device)
        self.count = torch.zeros(1, dtype=torch.int32, device=device)
        self.stream = stream

    def detect_async(self, frame: torch.Tensor) -> None:
        """Queue detection of a CUDA uint8 [H, W] frame (unit column stride)."""
        if not (isinstance(frame, torch.Tensor) and frame.device.type == "cuda" and frame.dtype == torch.uint8
                and frame.dim() == 2 and frame.stride(1) == 1
                and tuple(frame.shape) == (self.height, self.width)):
            raise ValueError("frame must be a CUDA uint8 [H, W] tensor with unit column stride")
        _check(lib.kpd_detect_layers(frame.data_ptr(), frame.stride(0), self.width, self.height, self.fast_t,
                                     self.n_octaves, self.workspace.data_ptr(), self.workspace.numel(),
                                     self.out.data_ptr(), self.capacity, self.count.data_ptr(),
                                     _stream_ptr(self.stream)))

    def detect_static_async(self, frame: torch.Tensor) -> None:
        """detect_async through kpd_detect_layers_static: the library's static
        workspace instead of this detector's."""
        if not (isinstance(frame, torch.Tensor) and frame.device.type == "cuda" and frame.dtype == torch.uint8
                and frame.dim() == 2 and frame.stride(1) == 1
                and tuple(frame.shape) == (self.height, self.width)):
            raise ValueError("frame must be a CUDA uint8 [H, W] tensor with unit column stride")
        _check(lib.kpd_detect_layers_static(frame.data_ptr(), frame.stride(0), self.width, self.height, self.fast_t,
                                            self.n_octaves, self.out.data_ptr(), self.capacity,
                                            self.count.data_ptr(), _stream_ptr(self.stream)))

    def detect(self, frame) -> np.ndarray:
        """Keypoints (KEYPOINT_DTYPE, `octave` = layer index) of one frame."""
        if isinstance(frame, np.ndarray):
            frame = torch.from_numpy(np.ascontiguousarray(frame)).cuda()
        self.detect_async(frame)
        n = min(int(self.count.item()), self.capacity)
        raw = self.out[:n * KEYPOINT_DTYPE.itemsize].cpu().numpy()
        return raw.view(KEYPOINT_DTYPE).copy()

    def refine(self) -> np.ndarray:
        """Refined values (REFINED_DTYPE) of the last detection's keypoints,
        in their order."""
        if not hasattr(self, "refined_dev"):
            self.refined_dev = torch.empty(self.capacity * REFINED_DTYPE.itemsize, dtype=torch.uint8,
                                           device=self.out.device)
        _check(lib.kpd_refine_layers(self.width, self.height, self.n_octaves, self.workspace.data_ptr(),
                                     self.workspace.numel(), self.out.data_ptr(), self.count.data_ptr(),
                                     self.capacity, self.refined_dev.data_ptr(), _stream_ptr(self.stream)))
        n = min(int(self.count.item()), self.capacity)
        return self.refined_dev[:n * REFINED_DTYPE.itemsize].cpu().numpy().view(REFINED_DTYPE).copy()

    def layer(self, l: int) -> np.ndarray:
        """Layer l >= 1 of the last frame, as computed on the device."""
        off, w, h = layer_plane(self.width, self.height, self.n_octaves, l)
        return self.workspace[off:off + w * h].cpu().numpy().reshape(h, w)


class LayerStream:
    """The masked stream over octaves and intra-octaves (per-cell mask,
    Eq. 1; D_n's `octave` field holds the layer index)."""

    def __init__(self, width: int, height: int, params: KpdParams, stream=None, device="cuda"):
        self.width, self.height, self.params = width, height, params
        self.n_cells = params.grid_cols * params.grid_rows
        n = lib.kpd_lstream_bytes(width, height, ctypes.byref(params))
        if n == 0:
            raise KpdError(KPD_EINVAL, lib.kpd_last_error().decode())
        self.arena = torch.empty(n, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        _check(lib.kpd_lstream_open(width, height, ctypes.byref(params), self.arena.data_ptr(), n,
                                    _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h.value
        self._held = [None, None]

    def push(self, frame, retain: bool = False) -> None:
        if isinstance(frame, np.ndarray):
            if frame.dtype != np.uint8 or frame.ndim != 2 or frame.strides[1] != 1:
                raise ValueError("host frame must be a uint8 [H, W] array with unit column stride")
            _check(lib.kpd_lstream_push(self.handle, frame.ctypes.data, frame.strides[0], FRAME_HOST))
            return
        if not (isinstance(frame, torch.Tensor) and frame.device.type == "cuda" and frame.dtype == torch.uint8
                and frame.dim() == 2 and frame.stride(1) == 1):
            raise ValueError("device frame must be a CUDA uint8 [H, W] tensor with unit column stride")
        _check(lib.kpd_lstream_push(self.handle, frame.data_ptr(), frame.stride(0),
                                    FRAME_DEVICE_RETAIN if retain else FRAME_DEVICE))
        if retain:
            self._held = [self._held[1], frame]

    def push_chunk(self, frames: torch.Tensor) -> None:
        """Consecutive frames [n, H, W] (a CUDA uint8 tensor with unit column
        stride, n <= chunk_frames) in one call, read in place."""
        if not (isinstance(frames, torch.Tensor) and frames.device.type == "cuda" and frames.dtype == torch.uint8
                and frames.dim() == 3 and frames.stride(2) == 1):
            raise ValueError("frames must be a CUDA uint8 [n, H, W] tensor with unit column stride")
        _check(lib.kpd_lstream_push_frames(self.handle, frames.data_ptr(), frames.stride(0), frames.stride(1),
                                           frames.shape[0]))
        self._held = [self._held[1], frames]

    def chunk_keypoints(self, i: int, capacity: int = 4096) -> np.ndarray:
        """D of frame i of the last push_chunk."""
        out = np.zeros(max(capacity, 1), KEYPOINT_DTYPE)
        cnt = ctypes.c_size_t()
        rc = lib.kpd_lstream_get_chunk(self.handle, i, out.ctypes.data, len(out), ctypes.byref(cnt))
        if rc == KPD_ETRUNC:
            out = np.zeros(cnt.value, KEYPOINT_DTYPE)
            rc = lib.kpd_lstream_get_chunk(self.handle, i, out.ctypes.data, len(out), ctypes.byref(cnt))
        _check(rc)
        return out[:cnt.value].copy()

    def keypoints(self, capacity: int = 4096) -> Tuple[np.ndarray, np.ndarray]:
        out = np.zeros(max(capacity, 1), KEYPOINT_DTYPE)
        mask = np.zeros(self.n_cells, np.uint8)
        cnt = ctypes.c_size_t()
        rc = lib.kpd_lstream_get(self.handle, out.ctypes.data, len(out), ctypes.byref(cnt), mask.ctypes.data)
        if rc == KPD_ETRUNC:
            out = np.zeros(cnt.value, KEYPOINT_DTYPE)
            rc = lib.kpd_lstream_get(self.handle, out.ctypes.data, len(out), ctypes.byref(cnt), mask.ctypes.data)
        _check(rc)
        return out[:cnt.value].copy(), mask

    def reset(self) -> None:
        _check(lib.kpd_lstream_reset(self.handle))

    def close(self) -> None:
        if self.handle:
            _check(lib.kpd_lstream_close(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class LayerBatch:
    """A batch of masked streams over octaves and intra-octaves sharing one
    frame size and one set of parameters: `n_slots` streams advanced
    together, one tick at a time (frames read in place from the device)."""

    def __init__(self, width: int, height: int, params: KpdParams, n_slots: int, stream=None, device="cuda"):
        self.width, self.height, self.params, self.n_slots = width, height, params, n_slots
        self.n_cells = params.grid_cols * params.grid_rows
        n = lib.kpd_lbatch_bytes(width, height, ctypes.byref(params), n_slots)
        if n == 0:
            raise KpdError(KPD_EINVAL, lib.kpd_last_error().decode())
        self.arena = torch.empty(n, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        _check(lib.kpd_lbatch_open(width, height, ctypes.byref(params), n_slots, self.arena.data_ptr(), n,
                                   _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h.value
        self._held = [[None, None] for _ in range(n_slots)]

    def push(self, slot: int, frame: torch.Tensor) -> None:
        if not (isinstance(frame, torch.Tensor) and frame.device.type == "cuda" and frame.dtype == torch.uint8
                and frame.dim() == 2 and frame.stride(1) == 1):
            raise ValueError("frame must be a CUDA uint8 [H, W] tensor with unit column stride")
        _check(lib.kpd_lbatch_push(self.handle, slot, frame.data_ptr(), frame.stride(0)))
        self._held[slot] = [self._held[slot][1], frame]

    def tick(self) -> None:
        _check(lib.kpd_lbatch_tick(self.handle))

    def keypoints(self, slot: int, capacity: int = 4096) -> Tuple[np.ndarray, np.ndarray]:
        out = np.zeros(max(capacity, 1), KEYPOINT_DTYPE)
        mask = np.zeros(self.n_cells, np.uint8)
        cnt = ctypes.c_size_t()
        rc = lib.kpd_lbatch_get(self.handle, slot, out.ctypes.data, len(out), ctypes.byref(cnt), mask.ctypes.data)
        if rc == KPD_ETRUNC:
            out = np.zeros(cnt.value, KEYPOINT_DTYPE)
            rc = lib.kpd_lbatch_get(self.handle, slot, out.ctypes.data, len(out), ctypes.byref(cnt), mask.ctypes.data)
        _check(rc)
        return out[:cnt.value].copy(), mask

    def reset(self, slot: int) -> None:
        _check(lib.kpd_lbatch_reset(self.handle, slot))

    def close(self) -> None:
        if self.handle:
            _check(lib.kpd_lbatch_close(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
