#!/usr/bin/env python3
"""Throughput and latency of masked vs full-frame keypoint detection on one GPU.

One step = one pass of the whole detection path (cell mask, pyramid,
segment test + score + scale-space suppression, compaction, Eq. (1) output)
over every frame of one synthetic video, frames already resident in HBM and
pushed through the C ABI in place (no copy). The headline workload is the
640x480, 300-frame single stream (FAST-9 t=20, 4 octaves, 16x12 cells,
T_I = 8), pushed up to 256 consecutive frames per push_frames call
(results are identical to one push per frame). The same line also carries the
full-frame rate of that workload, the streaming mode (one push_frame per
frame) with its per-frame latency percentiles, the 1920x1080 rates, the
batched 64-stream and serving sections, the dominant kernel's roofline and
the CPU oracle's rate on a bounded sample.

Prints one JSON line on stdout. Usage:
  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-hd]
  python bench.py --copy-calibration MiB   (plain device copy, for counter scaling)
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "masked-detect Mpixel/s & frames/s vs full-frame at 1 GPU; p50/p99 frame latency"


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2_640x480")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-hd", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MiB")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the 64-stream batched ticks (both forms) and print their line (for profiling)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-horizon", type=float, default=48.0)
    ap.add_argument("--serve-speedup", type=float, default=4.0)
    ap.add_argument("--serve-budget-mib", type=int, default=1024)
    ap.add_argument("--saturation-seconds", type=float, default=4.0)
    ap.add_argument("--saturation-budget-mib", type=int, default=4096)
    ap.add_argument("--batch-ticks", type=int, default=120)
    ap.add_argument("--batch-clip", type=int, default=40)
    ap.add_argument("--chunk", type=int, default=0,
                    help="frames per push_frames call (at most 512; 0: the whole video in one call)")
    ap.add_argument("--mode", choices=("both", "masked", "full"), default="both",
                    help="masked or full: run only that pass of --workload and print its line (for profiling)")
    ap.add_argument("--chunked", action="store_true", help="with --mode: push --chunk frames per call")
    ap.add_argument("--layer", type=int, default=None,
                    help="with --mode masked: the per-pixel mask on this pyramid layer (single-frame pushes)")
    ap.add_argument("--tile", type=int, default=0, help="level-0 tile of the tile pass (0: the library default)")
    ap.add_argument("--groups", default="0x0x0", metavar="CxRxT",
                    help="cells per workgroup (columns x rows) and threads of full-frame chunk detection "
                         "(0x0x0: the library default)")
    ap.add_argument("--profile-script", metavar="OUTDIR", help="print the rocprofv3 script for the profiles")
    ap.add_argument("--summarize-profiles", metavar="OUTDIR", help="write profiles/ from that script's output")
    return ap.parse_args()


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def level_sizes(W, H, O):
    return [(W >> o) * (H >> o) for o in range(O)]


class Workload:
    def __init__(self, name: str):
        import torch
        from paper_1503_06959_amd import synth
        self.name = name
        self.sc = synth.SCENES[name]
        self.det = synth.DETECTORS[name]
        t0 = time.time()
        self.frames = synth.make_video(self.sc)
        log(f"[bench] generated {name}: {self.frames.shape} in {time.time() - t0:.1f}s")
        self.dev = torch.from_numpy(self.frames).cuda()
        self.F, self.H, self.W = self.frames.shape
        self.ncell = self.det.grid_cols * self.det.grid_rows

    def describe(self, id_thresh):
        d = self.det
        return (f"{self.name}: 1 stream, {self.F} frames {self.W}x{self.H} u8, FAST-9/16 t={d.fast_t}, "
                f"{d.n_octaves} octaves, {d.grid_cols}x{d.grid_rows} cells, "
                + ("full-frame (T_I<0)" if id_thresh < 0 else f"T_I={id_thresh}, T_H off"))


TILE = 0
GROUPS = (0, 0, 0)   # cells per workgroup of full-frame chunk detection (cols, rows) and its threads; 0: default


def open_stream(wl: Workload, id_thresh: int, chunk: int = 0, layer_mask: bool = False, kb_thresh=None,
                features: int = 0):
    from paper_1503_06959_amd import kpd
    d = wl.det
    kb = d.kb_thresh if kb_thresh is None else kb_thresh
    params = kpd.make_params(d.fast_t, d.n_octaves, d.grid_cols, d.grid_rows, id_thresh, kb, TILE, chunk,
                             int(layer_mask), features, *GROUPS)
    s = kpd.Stream(wl.W, wl.H, params)
    s.chunk = chunk
    return s


def one_pass(kpd, s, wl: Workload) -> None:
    """Push every frame of the video in place (one frame per call, or
    chunks of s.chunk consecutive frames); results stay on the device."""
    kpd.reset_stream(s.handle)
    h, dev, pitch = s.handle, wl.dev, wl.W
    if s.chunk > 1:
        push = kpd.lib.push_frames
        base, stride = dev.data_ptr(), wl.W * wl.H
        for i in range(0, wl.F, s.chunk):
            rc = push(h, base + i * stride, stride, pitch, min(s.chunk, wl.F - i))
            if rc:
                raise kpd.KpdError(rc, kpd.lib.kpd_last_error().decode())
        return
    push = kpd.lib.push_frame
    for i in range(wl.F):
        rc = push(h, dev[i].data_ptr(), pitch, kpd.FRAME_DEVICE_RETAIN)
        if rc:
            raise kpd.KpdError(rc, kpd.lib.kpd_last_error().decode())


def timed_passes(kpd, s, wl: Workload, steps: int, warmup: int) -> float:
    import torch
    for _ in range(warmup):
        one_pass(kpd, s, wl)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one_pass(kpd, s, wl)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def chunk_latency(kpd, s, wl: Workload, reps: int = 3):
    """Milliseconds from push_frames of one chunk to the last frame's
    keypoints on the host (the first frame of a chunk waits for the whole
    chunk to arrive before this starts)."""
    import numpy as np
    lat = []
    base, stride = wl.dev.data_ptr(), wl.W * wl.H
    for _ in range(reps):
        kpd.reset_stream(s.handle)
        for i in range(0, wl.F, s.chunk):
            t0 = time.perf_counter()
            kpd._check(kpd.lib.push_frames(s.handle, base + i * stride, stride, wl.W, min(s.chunk, wl.F - i)))
            s.keypoints()
            lat.append((time.perf_counter() - t0) * 1e3)
    lat = np.array(lat)
    return float(np.percentile(lat, 50)), float(np.percentile(lat, 99))


def host_frames_pass(kpd, wl: Workload, steps: int) -> dict:
    """Streaming from host memory: every push copies the frame over PCIe
    into the stream's arena slot (pageable numpy frames)."""
    import torch
    s = open_stream(wl, wl.det.id_thresh)
    frames = [wl.frames[i] for i in range(wl.F)]
    for i in range(min(wl.F, 20)):
        kpd.push_frame(s.handle, frames[i])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        kpd.reset_stream(s.handle)
        for f in frames:
            kpd.push_frame(s.handle, f)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    s.close()
    return {"value": round(wl.F * wl.W * wl.H / dt / 1e6, 2), "unit": "Mpixel/s",
            "frames_per_s": round(wl.F / dt, 1),
            "what": "push_frame from pageable host memory (copy included), masked, one frame per call"}


def latency_pass(kpd, s, wl: Workload):
    """Per-frame latency push -> keypoints on the host; also collects what
    the algorithmic byte counts need (marked cells, keypoints in them)."""
    import numpy as np
    d = wl.det
    kpd.reset_stream(s.handle)
    lat, marked, new_kp, total_kp = [], [], [], []
    for i in range(wl.F):
        t0 = time.perf_counter()
        kpd.push_frame(s.handle, wl.dev[i], retain=True)
        k, m = s.keypoints()
        lat.append((time.perf_counter() - t0) * 1e3)
        cell = ((k["y"].astype(np.int64) << k["octave"]) * d.grid_rows // wl.H) * d.grid_cols + \
               ((k["x"].astype(np.int64) << k["octave"]) * d.grid_cols // wl.W)
        marked.append(int(m.sum()))
        new_kp.append(int(m[cell].sum()) if len(k) else 0)
        total_kp.append(len(k))
    lat = np.array(lat)
    return {
        "lat_p50": float(np.percentile(lat, 50)), "lat_p99": float(np.percentile(lat, 99)),
        "marked": marked, "new_kp": new_kp, "total_kp": total_kp,
    }


def device_time_pass(kpd, s, wl: Workload):
    """Per-frame device time of streaming pushes: HIP events recorded on the
    stream's HIP stream before and after each push_frame, read after the
    pass (no host wait between frames); p50 and p99 in ms."""
    import numpy as np
    import torch
    kpd.reset_stream(s.handle)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(wl.F + 1)]
    ev[0].record()
    for i in range(wl.F):
        kpd._check(kpd.lib.push_frame(s.handle, wl.dev[i].data_ptr(), wl.W, kpd.FRAME_DEVICE_RETAIN))
        ev[i + 1].record()
    torch.cuda.synchronize()
    ms = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(wl.F)])
    return float(np.percentile(ms, 50)), float(np.percentile(ms, 99))


def kernel_profile(kpd, s, wl: Workload, steps: int):
    """Event-timed milliseconds and launch counts per kernel over `steps`
    passes (events on the stream the kernels are launched on)."""
    kpd.profile(s.handle, True)
    kpd.profile_read(s.handle)
    for _ in range(steps):
        one_pass(kpd, s, wl)
    ms, n = kpd.profile_read(s.handle)
    kpd.profile(s.handle, False)
    out = {name: (float(ms[k]), int(n[k])) for k, name in enumerate(kpd.KERNEL_NAMES) if n[k]}
    out["passes"] = steps
    return out


def algorithmic_bytes(wl: Workload, st, masked: bool, chunked: bool = False) -> dict:
    """Bytes the method must move per pass over the video, per kernel.
    The tile pass reads I_n (and I_{n-1} for the intensity-difference test)
    and writes the coarser octaves: all of them in full-frame mode, the
    marked cells' share f * P of them in masked mode (2N + f P per streamed
    frame; in a chunk I_{n-1} is the frame just read, so N + f P per frame
    plus the frame before the chunk; what a pass writes beyond that is
    waste, not method). The cell pass reads the octave pixels of
    the marked cells, writes their keypoints, and carries the others' (Eq. 1)
    with a 16-byte read+write per entry; 24 bytes per cell and frame cover
    the per-cell counts, offsets and SAD. In chunks the cell pass writes
    only the marked cells' keypoints (plus 16 bytes of mark, count and SAD
    per cell and frame) and the compaction pass reads and writes every
    frame's whole D_n (16 bytes per entry) plus the per-cell metadata.
    Score maps are an LDS intermediate and count nothing. Frame 0 of a pass
    marks every cell."""
    d = wl.det
    N = wl.W * wl.H
    lv = level_sizes(wl.W, wl.H, d.n_octaves)
    P = sum(lv[1:])
    F = wl.F
    layer = st.get("layer")
    sad_frames = (F - 1) if masked and layer is None else 0
    frac = [m / wl.ncell for m in st["marked"]]
    carried = sum(t - n for t, n in zip(st["total_kp"], st["new_kp"]))
    meta = 24 * wl.ncell * F
    scan = sum(f * sum(lv) for f in frac) + 8 * sum(st["new_kp"])
    pyr = P * (sum(frac) if masked and layer is None else F)
    # a single frame's pass reads I_{n-1} beside I_n (2N + f P); in a chunk
    # every frame is I_n of its frame and I_{n-1} of the next, so the method
    # reads each frame once plus the frame before the chunk (N + f P)
    prev_reads = (1 if sad_frames else 0) if chunked else sad_frames
    out = {"k_frame": F * N + pyr + N * prev_reads}
    if chunked:
        out["k_detect"] = scan + 16 * wl.ncell * F
        out["k_compact"] = 16 * sum(st["total_kp"]) + meta
        out["k_mark"] = 8 * wl.ncell * F
    else:
        out["k_detect"] = scan + 16 * carried + meta
        if layer is not None:   # the per-pixel test reads layer `layer` of I_n and I_{n-1}
            out["k_detect"] += 2 * lv[layer] * (F - 1)
    return out


FEATURE_PASSES = {
    "descriptors": (1, "descriptors (60-point pattern, 32 sectors, 512 bits)"),
    "refinement": (2, "sub-pixel and sub-scale refinement (3x3 score fits on three layers)"),
}


def feature_workload(kpd, wl: Workload, args, which: str) -> dict:
    """Per-feature values of D_n (streaming, one push_frame per frame):
    masked frames compute them only for the features of marked cells and
    carry the rest (Eq. 1), full-frame ones for every feature."""
    features, label = FEATURE_PASSES[which]
    out = {}
    for name, ti in (("masked", wl.det.id_thresh), ("full_frame", -1)):
        s = open_stream(wl, ti, features=features)
        sec = timed_passes(kpd, s, wl, max(1, args.steps // 5), 1)
        prof = kernel_profile(kpd, s, wl, 2)
        st = latency_pass(kpd, s, wl)
        s.close()
        out[name] = {"value": round(wl.F * wl.W * wl.H / sec / 1e6, 2), "unit": "Mpixel/s",
                     "frames_per_s": round(wl.F / sec, 1),
                     "latency_ms": {"p50": round(st["lat_p50"], 4), "p99": round(st["lat_p99"], 4)},
                     "computed_per_frame": round(sum(st["new_kp"]) / wl.F, 1),
                     "features_per_frame": round(sum(st["total_kp"]) / wl.F, 1),
                     "k_describe_avg_us": round(prof["k_describe"][0] * 1e3 / max(prof["k_describe"][1], 1), 3)
                     if "k_describe" in prof else None}
    K = chunk_of(args, wl)
    for name, ti in (("chunked_masked", wl.det.id_thresh), ("chunked_full_frame", -1)):
        s = open_stream(wl, ti, K, features=features)
        sec = timed_passes(kpd, s, wl, max(1, args.steps // 5), 1)
        prof = kernel_profile(kpd, s, wl, 2)
        s.close()
        out[name] = {"value": round(wl.F * wl.W * wl.H / sec / 1e6, 2), "unit": "Mpixel/s",
                     "frames_per_s": round(wl.F / sec, 1), "chunk": K,
                     "k_describe_us_per_pass": round(prof["k_describe"][0] * 1e3 / prof["passes"], 3)
                     if "k_describe" in prof else None}
    out["what"] = (f"{wl.name}, {label}: one push_frame per frame (masked, full_frame) or chunks of {K} frames "
                   "(chunked_*); masked frames compute them for the new features only, carried ones keep theirs")
    out["computed_masked_over_full"] = round(out["masked"]["computed_per_frame"] /
                                             max(out["full_frame"]["computed_per_frame"], 1e-9), 4)
    return out


def tcd_workload(kpd, wl: Workload, args) -> dict:
    """The comparison system of Sec. 4 on the same video: full-frame
    detection on the first frame of every group of 10, quarter-pixel block
    matching of the keypoints' 16 x 16 patches on the others (T_BM = 1800,
    T_ET = 1000). Whole-video throughput, per-frame GPU time of detected and
    propagated frames (events on the tracker's stream), tracks per frame."""
    import numpy as np
    import torch
    d = wl.det
    gop = 10
    g = kpd.Tcd(wl.W, wl.H, kpd.make_params(d.fast_t, d.n_octaves, d.grid_cols, d.grid_rows), gop, 1800, 1000)
    ptrs = [wl.dev[i].data_ptr() for i in range(wl.F)]

    def one_pass():
        g.reset()
        for p in ptrs:
            kpd._check(kpd.lib.tcd_push(g.handle, p, wl.W, kpd.FRAME_DEVICE_RETAIN))

    one_pass()
    torch.cuda.synchronize()
    steps = max(1, args.steps // 5)
    t0 = time.perf_counter()
    for _ in range(steps):
        one_pass()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(wl.F + 1)]
    g.reset()
    ev[0].record()
    for i, p in enumerate(ptrs):
        kpd._check(kpd.lib.tcd_push(g.handle, p, wl.W, kpd.FRAME_DEVICE_RETAIN))
        ev[i + 1].record()
    torch.cuda.synchronize()
    ms = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(wl.F)])
    first = np.arange(wl.F) % gop == 0
    g.reset()
    counts = []
    for p in ptrs:
        kpd._check(kpd.lib.tcd_push(g.handle, p, wl.W, kpd.FRAME_DEVICE_RETAIN))
        counts.append(len(g.tracks()))
    g.close()
    counts = np.array(counts)
    return {"value": round(wl.F * wl.W * wl.H / dt / 1e6, 2), "unit": "Mpixel/s", "frames_per_s": round(wl.F / dt, 1),
            "gpu_ms_per_frame": {"detected": round(float(ms[first].mean()), 4),
                                 "propagated": round(float(ms[~first].mean()), 4)},
            "tracks_per_frame": {"detected": round(float(counts[first].mean()), 1),
                                 "propagated": round(float(counts[~first].mean()), 1)},
            "what": f"{wl.name}, temporally coherent detector: groups of {gop}, 16x16 patches, coarse spiral "
                    "search (2-pixel steps, 24-pixel window), quarter-pixel refinement within 1.75 pixels, "
                    "T_BM=1800, T_ET=1000; one tcd_push per frame"}


def layer_launches(O: int) -> int:
    """Launches of one kpd_detect_layers call: the octaves two halvings per
    launch, the 1.5x pass with d_1, the intra-octaves two per launch, then
    score, suppression, scan and write."""
    return O // 2 + 1 + (max(O - 2, 0) + 1) // 2 + 4


def intra_octave_workload(kpd, wl: Workload, args) -> dict:
    """Full-frame detection over octaves and intra-octaves (Sec. 2's BRISK
    scale space, 2O layers), one call per frame of the video, frames in
    place; keypoints per frame on octave and intra-octave layers."""
    import numpy as np
    import torch
    d = wl.det
    det = kpd.LayerDetector(wl.W, wl.H, d.fast_t, d.n_octaves)

    def one_pass():
        for i in range(wl.F):
            det.detect_async(wl.dev[i])

    one_pass()
    torch.cuda.synchronize()
    steps = max(1, args.steps // 10)
    t0 = time.perf_counter()
    for _ in range(steps):
        one_pass()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    one_pass()
    e1.record()
    torch.cuda.synchronize()
    oct_kp, intra_kp = [], []
    for i in range(0, wl.F, max(1, wl.F // 30)):
        k = det.detect(wl.dev[i])
        oct_kp.append(int((k["octave"] % 2 == 0).sum()))
        intra_kp.append(int((k["octave"] % 2 == 1).sum()))
    # detection followed by refinement of every keypoint, frame by frame
    det.refine()
    r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    r0.record()
    for i in range(wl.F):
        det.detect_async(wl.dev[i])
        kpd._check(kpd.lib.kpd_refine_layers(det.width, det.height, det.n_octaves, det.workspace.data_ptr(),
                                             det.workspace.numel(), det.out.data_ptr(), det.count.data_ptr(),
                                             det.capacity, det.refined_dev.data_ptr(), kpd._stream_ptr(None)))
    r1.record()
    torch.cuda.synchronize()
    # the masked stream over the same layers (per-cell mask, Eq. 1)
    streams = {}
    for name, ti in (("masked", d.id_thresh), ("full_frame", -1)):
        ls = kpd.LayerStream(wl.W, wl.H, kpd.make_params(d.fast_t, d.n_octaves, d.grid_cols, d.grid_rows, ti,
                                                         d.kb_thresh))

        def ls_pass():
            kpd._check(kpd.lib.kpd_lstream_reset(ls.handle))
            for i in range(wl.F):
                kpd._check(kpd.lib.kpd_lstream_push(ls.handle, wl.dev[i].data_ptr(), wl.W, kpd.FRAME_DEVICE_RETAIN))

        ls_pass()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ls_pass()
        torch.cuda.synchronize()
        lt = (time.perf_counter() - t0) / steps
        marked, kps = [], []
        kpd._check(kpd.lib.kpd_lstream_reset(ls.handle))
        for i in range(wl.F):
            kpd._check(kpd.lib.kpd_lstream_push(ls.handle, wl.dev[i].data_ptr(), wl.W, kpd.FRAME_DEVICE_RETAIN))
            if i % max(1, wl.F // 30) == 0:
                k, m = ls.keypoints()
                marked.append(float(m.mean()))
                kps.append(len(k))
        ls.close()
        streams[name] = {"value": round(wl.F * wl.W * wl.H / lt / 1e6, 2), "unit": "Mpixel/s",
                         "frames_per_s": round(wl.F / lt, 1), "marked_cell_frac": round(float(np.mean(marked)), 4),
                         "keypoints_per_frame": round(float(np.mean(kps)), 1)}
        # the same stream in chunks of consecutive frames (kpd_lstream_push_frames)
        K = chunk_of(args, wl)
        lc = kpd.LayerStream(wl.W, wl.H, kpd.make_params(d.fast_t, d.n_octaves, d.grid_cols, d.grid_rows, ti,
                                                         d.kb_thresh, 0, K))

        def lc_pass():
            kpd._check(kpd.lib.kpd_lstream_reset(lc.handle))
            base, stride = wl.dev.data_ptr(), wl.W * wl.H
            for i in range(0, wl.F, K):
                kpd._check(kpd.lib.kpd_lstream_push_frames(lc.handle, base + i * stride, stride, wl.W,
                                                           min(K, wl.F - i)))

        lc_pass()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            lc_pass()
        torch.cuda.synchronize()
        ct = (time.perf_counter() - t0) / steps
        lc.close()
        streams[name + "_chunked"] = {"value": round(wl.F * wl.W * wl.H / ct / 1e6, 2), "unit": "Mpixel/s",
                                      "frames_per_s": round(wl.F / ct, 1), "chunk": K,
                                      "over_per_frame_push": round(lt / ct, 2)}
    return {"value": round(wl.F * wl.W * wl.H / dt / 1e6, 2), "unit": "Mpixel/s", "frames_per_s": round(wl.F / dt, 1),
            "stream": streams,
            "gpu_us_per_frame": round(e0.elapsed_time(e1) * 1e3 / wl.F, 3),
            "gpu_us_per_frame_with_refinement": round(r0.elapsed_time(r1) * 1e3 / wl.F, 3),
            "keypoints_per_frame": {"octave_layers": round(float(np.mean(oct_kp)), 1),
                                    "intra_octave_layers": round(float(np.mean(intra_kp)), 1)},
            "what": f"{wl.name}, full-frame detection over {2 * d.n_octaves} layers (octaves and intra-octaves), "
                    f"one kpd_detect_layers call per frame ({layer_launches(d.n_octaves)} launches); with refinement, "
                    "one kpd_refine_layers call after it; `stream`: the masked stream over the same layers "
                    "(per-cell mask, Eq. 1), one kpd_lstream_push per frame, masked and full-frame, and "
                    "kpd_lstream_push_frames chunks of the whole video (*_chunked)"}


def layered_batch_workload(kpd, wl: Workload, args, n_slots: int = 64, n_ticks: int = 60) -> dict:
    """64 masked streams over octaves and intra-octaves of one shape advanced
    together: kpd_lbatch ticks against one kpd_lstream per stream pushed one
    frame per tick. Slot s plays the video from frame 5 s on (wrapping)."""
    import torch
    d = wl.det
    params = kpd.make_params(d.fast_t, d.n_octaves, d.grid_cols, d.grid_rows, d.id_thresh, d.kb_thresh)
    frame_of = lambda s, t: wl.dev[(5 * s + t) % wl.F]
    b = kpd.LayerBatch(wl.W, wl.H, params, n_slots)

    def batched(t0):
        for t in range(t0, t0 + n_ticks):
            for s in range(n_slots):
                kpd._check(kpd.lib.kpd_lbatch_push(b.handle, s, frame_of(s, t).data_ptr(), wl.W))
            kpd._check(kpd.lib.kpd_lbatch_tick(b.handle))

    batched(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batched(n_ticks)
    torch.cuda.synchronize()
    bt = (time.perf_counter() - t0) / n_ticks
    b.close()
    streams = [kpd.LayerStream(wl.W, wl.H, params) for _ in range(n_slots)]

    def plain(t0):
        for t in range(t0, t0 + n_ticks):
            for s, ls in enumerate(streams):
                kpd._check(kpd.lib.kpd_lstream_push(ls.handle, frame_of(s, t).data_ptr(), wl.W,
                                                    kpd.FRAME_DEVICE_RETAIN))

    plain(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain(n_ticks)
    torch.cuda.synchronize()
    pt = (time.perf_counter() - t0) / n_ticks
    for ls in streams:
        ls.close()
    px = n_slots * wl.W * wl.H
    return {"what": f"{n_slots} masked streams over octaves and intra-octaves of {wl.name} (slot s plays the video "
                    f"from frame 5 s), {n_ticks} timed ticks: one kpd_lbatch tick against {n_slots} kpd_lstream_push "
                    "calls per tick",
            "batched": {"mpix_per_s": round(px / bt / 1e6, 2), "ms_per_tick": round(bt * 1e3, 4)},
            "plain_per_stream": {"mpix_per_s": round(px / pt / 1e6, 2), "ms_per_tick": round(pt * 1e3, 4)},
            "batched_over_plain": round(pt / bt, 3)}


def layer_study(kpd, wl: Workload, args) -> dict:
    """The mask variants side by side on one workload (the paper tries every
    layer and keeps the top one since results are alike): per-frame push
    throughput, the share of cells whose mask is set, and how much of each
    frame's full detection F(I_n) the carried set D_n reproduces exactly
    (same position, octave and score)."""
    import numpy as np
    import torch
    full = open_stream(wl, -1)
    ref = []
    for i in range(wl.F):
        kpd.push_frame(full.handle, wl.dev[i], retain=True)
        ref.append(np.sort(full.keypoints()[0].view(np.uint64)))
    full.close()
    variants = [("cell_mean_level0", None)] + [(f"layer{l}", (1, l)) for l in range(wl.det.n_octaves)] + \
               [("per_octave", (2, 0))]
    out = {}
    for name, mode in variants:
        s = open_stream(wl, wl.det.id_thresh, layer_mask=mode is not None)
        if mode is not None:
            s.set_mask_mode(*mode)
        sec = timed_passes(kpd, s, wl, max(1, args.steps // 5), 1)
        kpd.reset_stream(s.handle)
        hit = tot_ref = tot_d = marked = 0
        for i in range(wl.F):
            kpd.push_frame(s.handle, wl.dev[i], retain=True)
            k, m = s.keypoints()
            d = np.sort(k.view(np.uint64))
            hit += len(np.intersect1d(d, ref[i], assume_unique=True))
            tot_ref += len(ref[i])
            tot_d += len(d)
            if i:
                marked += int(m.sum())
        s.close()
        out[name] = {"mpix_per_s": round(wl.F * wl.W * wl.H / sec / 1e6, 1),
                     "marked_cell_frac": round(marked / max(1, (wl.F - 1) * wl.ncell), 4),
                     "recall_of_full_detection": round(hit / max(1, tot_ref), 4),
                     "precision_vs_full_detection": round(hit / max(1, tot_d), 4),
                     "keypoints_per_frame": round(tot_d / wl.F, 1)}
    torch.cuda.synchronize()
    return {"what": f"{wl.name}, T_I={wl.det.id_thresh}, T_H off, one push_frame per frame; recall = share of "
                    "F(I_n) found unchanged in D_n, precision = share of D_n that is in F(I_n)",
            "full_detection_keypoints_per_frame": round(sum(len(r) for r in ref) / wl.F, 1), "variants": out}


def chunk_of(args, wl: Workload) -> int:
    """Frames per push_frames call: --chunk, or the whole video (at most 512)."""
    return args.chunk if args.chunk > 0 else min(wl.F, 512)


def run_workload(kpd, wl: Workload, id_thresh: int, args, want_latency=True, want_profile=True, chunk=0,
                 layer=None, kb_thresh=None, mask_mode=1):
    """layer: None for the per-cell mean-difference mask, else the pyramid
    layer of the per-pixel mask (mask_mode 1; mask_mode 2 masks each octave
    on its own level). kb_thresh: T_H (default: the workload's)."""
    s = open_stream(wl, id_thresh, chunk, layer_mask=layer is not None, kb_thresh=kb_thresh)
    if layer is not None:
        s.set_mask_mode(mask_mode, layer if mask_mode == 1 else 0)
    sec = timed_passes(kpd, s, wl, args.steps, args.warmup)
    res = {"sec_per_pass": sec, "frames": wl.F, "chunk": chunk, "layer": layer,
           "mpix_per_s": wl.F * wl.W * wl.H / sec / 1e6, "frames_per_s": wl.F / sec}
    if want_latency:
        if chunk > 1:
            res["lat_p50"], res["lat_p99"] = chunk_latency(kpd, s, wl)
        else:
            res.update(latency_pass(kpd, s, wl))
            res["dev_p50"], res["dev_p99"] = device_time_pass(kpd, s, wl)
    if want_profile:
        res["kernels"] = kernel_profile(kpd, s, wl, max(1, args.steps // 2))
    s.close()
    return res


def roofline_of(wl: Workload, res, masked: bool, traffic=None, stats=None, kernel=None):
    """Dominant kernel by summed event-timed duration (or `kernel`);
    achieved = algorithmic bytes per launch / average launch duration.
    `stats` (marked cells and keypoint counts per frame) default to the
    run's own."""
    st = dict(stats or res)
    st["chunk"] = res.get("chunk", 0)
    st["layer"] = res.get("layer")
    ab = algorithmic_bytes(wl, st, masked, chunked=res.get("chunk", 0) > 1)
    kern = {k: v for k, v in res["kernels"].items() if k != "passes"}
    passes = res["kernels"]["passes"]
    dom = kernel if kernel in kern else max(kern, key=lambda k: kern[k][0])
    ms, n = kern[dom]
    per_launch = ab[dom] * passes / max(n, 1)
    avg_s = ms / 1e3 / max(n, 1)
    achieved = per_launch / avg_s / 1e9 if avg_s > 0 else 0.0
    if traffic is None:
        traffic = traffic_for(wl.name, masked, res.get("chunk", 0), dom, res.get("layer"))
    measured = None
    if traffic:
        # the counters' bytes over the same launch time: what the kernel moved
        mt = traffic / avg_s / 1e9 if avg_s > 0 else 0.0
        measured = {"GBs": round(mt, 2), "frac": round(mt / HBM_PEAK_GBS, 5),
                    "over_algorithmic": round(traffic / per_launch, 3) if per_launch else None}
    return {
        "kernel": dom, "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic, "traffic_rate": measured,
        "algorithmic_bytes_per_launch": int(per_launch), "avg_launch_us": round(avg_s * 1e6, 3),
        "launches": n,
        "per_kernel_avg_us": {k: round(v[0] * 1e3 / max(v[1], 1), 3) for k, v in kern.items()},
    }


def _time_oracle(wl: Workload, id_thresh: int, lazy: bool, seconds: float, min_frames: int = 10):
    """Frames of the workload through one oracle stream for about `seconds`
    (at least min_frames); returns (frames, seconds)."""
    import oracle
    d = wl.det
    s = oracle.Stream(wl.W, wl.H, d.fast_t, d.n_octaves, d.grid_cols, d.grid_rows, id_thresh, d.kb_thresh)
    s.set_lazy(lazy)
    n = 0
    t0 = time.perf_counter()
    while True:
        for i in range(wl.F):
            s.push(wl.frames[i])
            n += 1
            if time.perf_counter() - t0 >= seconds and n >= min_frames:
                break
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    s.close()
    return n, dt


def cpu_baseline(wl: Workload, seconds: float):
    """The oracle on one host core on the masked workload: its definitional
    mode (full-frame detection, then the mask and Eq. 1) as `value`; beside
    it the CPU-masked mode (the same results, scoring only what the marked
    cells' suppression reads: the method on a CPU) and full-frame detection
    (T_I < 0)."""
    px = wl.W * wl.H
    n, dt = _time_oracle(wl, wl.det.id_thresh, False, seconds * 0.5)
    nm, dtm = _time_oracle(wl, wl.det.id_thresh, True, seconds * 0.25)
    nf, dtf = _time_oracle(wl, -1, False, seconds * 0.25)
    return {
        "value": round(n * px / dt / 1e6, 3), "unit": "Mpixel/s", "cores": 1, "kind": "oracle",
        "sample": f"{n} frames of {wl.name} through the oracle stream (mask + full-frame detection + Eq. 1), "
                  f"{dt:.1f}s, single thread, {cpu_model()}, {os.cpu_count()} host cores visible; beside it "
                  f"{nm} frames in the oracle's CPU-masked mode and {nf} full-frame (T_I < 0)",
        "frames_per_s": round(n / dt, 2),
        "cpu_masked_mode": {"value": round(nm * px / dtm / 1e6, 3), "unit": "Mpixel/s",
                            "frames_per_s": round(nm / dtm, 2)},
        "full_frame": {"value": round(nf * px / dtf / 1e6, 3), "unit": "Mpixel/s", "frames_per_s": round(nf / dtf, 2)},
    }


def _gen_clip(args):
    from paper_1503_06959_amd import synth
    sc, n = args
    return synth.make_video(sc, n)


def _oracle_streams(args):
    """One host worker of the all-cores oracle baseline: its share of the
    batched streams, each through its own oracle stream, one frame per stream
    per tick until `seconds` have passed. Returns (level-0 pixels, seconds)."""
    import oracle
    from paper_1503_06959_amd import synth
    idx, clip, seconds = args
    specs = synth.batch_streams(clip)
    mine = [(specs[i][0], specs[i][1], synth.make_video(specs[i][0], clip)) for i in idx]
    streams = [oracle.Stream(sc.width, sc.height, d.fast_t, d.n_octaves, d.grid_cols, d.grid_rows, d.id_thresh,
                             d.kb_thresh) for sc, d, _ in mine]
    px, k = 0, 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        i = pingpong(k, clip)
        for s, (sc, _, frames) in zip(streams, mine):
            s.push(frames[i])
            px += sc.width * sc.height
        k += 1
    dt = time.perf_counter() - t0
    for s in streams:
        s.close()
    return px, dt


def oracle_all_cores(clip: int, seconds: float) -> dict:
    """The oracle on every host core for the 64-stream batched workload:
    streams dealt round-robin to one worker process per core."""
    from concurrent.futures import ProcessPoolExecutor
    n = min(16, os.cpu_count() or 1)
    parts = [(list(range(w, 64, n)), clip, seconds) for w in range(n)]
    with ProcessPoolExecutor(max_workers=n) as ex:
        res = list(ex.map(_oracle_streams, parts))
    px = sum(p for p, _ in res)
    dt = max(d for _, d in res)
    return {"value": round(px / dt / 1e6, 3), "unit": "Mpixel/s", "cores": n, "kind": "oracle",
            "sample": f"the 64 batched streams dealt to {n} worker processes, one oracle stream per video stream, "
                      f"about {seconds:.0f}s each, {cpu_model()}"}


def pingpong(k: int, n: int) -> int:
    """Index of tick k when an n-frame clip plays forward and back."""
    if n == 1:
        return 0
    m = k % (2 * n - 2)
    return m if m < n else 2 * n - 2 - m


def batched_workload(kpd, n_ticks: int, clip: int, warmup: int, cpu: bool = True) -> dict:
    """64 mixed-resolution streams (24 x 320x240, 24 x 640x480, 16 x 1280x720),
    one frame each per tick: batched ticks (four graph-replayed launches per
    tick, and the single-launch form beside them) against plain per-stream
    pushes (three launches per stream and frame) over the same frames."""
    import torch
    from concurrent.futures import ProcessPoolExecutor
    from paper_1503_06959_amd import autotune, synth
    from paper_1503_06959_amd.batch import Batch
    specs = synth.batch_streams(clip)
    t0 = time.time()
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        clips = list(ex.map(_gen_clip, [(sc, clip) for sc, _ in specs]))
    log(f"[bench] generated 64 clips of {clip} frames in {time.time() - t0:.1f}s")
    devs = [torch.from_numpy(c).cuda() for c in clips]
    tiles = {}
    for sc, det in specs:
        key = autotune.class_key(sc.width, sc.height, det)
        if key not in tiles:
            tiles[key] = autotune.best_tile(sc.width, sc.height, det)[0]
    px_per_tick = sum(sc.width * sc.height for sc, _ in specs)

    b = Batch(max_streams=len(specs))
    bs = [b.open_stream(sc.width, sc.height,
                        kpd.make_params(d.fast_t, d.n_octaves, d.grid_cols, d.grid_rows, d.id_thresh, d.kb_thresh,
                                        tiles[autotune.class_key(sc.width, sc.height, d)]))
          for sc, d in specs]
    push = kpd.lib.batch_push
    def tick(k):
        i = pingpong(k, clip)
        for s, dev in zip(bs, devs):
            rc = push(b.handle, s.handle, dev[i].data_ptr(), dev.shape[2], kpd.FRAME_DEVICE_RETAIN)
            if rc:
                raise kpd.KpdError(rc, kpd.lib.kpd_last_error().decode())
        kpd.batch_tick(b.handle)
    def timed_ticks():
        for k in range(warmup):
            tick(k)
        b.synchronize()
        t0 = time.perf_counter()
        for k in range(warmup, warmup + n_ticks):
            tick(k)
        b.synchronize()
        return (time.perf_counter() - t0) / n_ticks
    sec_b = timed_ticks()
    b.set_single_launch(True)
    sec_1 = timed_ticks()
    b.set_single_launch(False)
    for s in bs:
        b.detach(s)
        s.close()
    b.close()

    ts = torch.cuda.Stream()
    ps = [kpd.Stream(sc.width, sc.height,
                     kpd.make_params(d.fast_t, d.n_octaves, d.grid_cols, d.grid_rows, d.id_thresh, d.kb_thresh),
                     stream=ts) for sc, d in specs]
    pf = kpd.lib.push_frame
    def plain(k):
        i = pingpong(k, clip)
        for s, dev in zip(ps, devs):
            rc = pf(s.handle, dev[i].data_ptr(), dev.shape[2], kpd.FRAME_DEVICE_RETAIN)
            if rc:
                raise kpd.KpdError(rc, kpd.lib.kpd_last_error().decode())
    for k in range(warmup):
        plain(k)
    ts.synchronize()
    t0 = time.perf_counter()
    for k in range(warmup, warmup + n_ticks):
        plain(k)
    ts.synchronize()
    sec_p = (time.perf_counter() - t0) / n_ticks
    for s in ps:
        s.close()
    return {
        "workload": f"64 streams (24 x 320x240, 24 x 640x480, 16 x 1280x720), {clip}-frame clips played "
                    f"forward and back, {n_ticks} timed ticks, T_I=8, per-resolution presets",
        "batched": {"mpix_per_s": round(px_per_tick / sec_b / 1e6, 2), "frames_per_s": round(64 / sec_b, 1),
                    "ms_per_tick": round(sec_b * 1e3, 4), "launches_per_tick": 4, "hip_graph": True,
                    "tiles": tiles},
        "batched_single_launch": {"mpix_per_s": round(px_per_tick / sec_1 / 1e6, 2),
                                  "ms_per_tick": round(sec_1 * 1e3, 4), "launches_per_tick": 1,
                                  "hip_graph": True},
        "plain_per_stream": {"mpix_per_s": round(px_per_tick / sec_p / 1e6, 2),
                             "frames_per_s": round(64 / sec_p, 1), "ms_per_tick": round(sec_p * 1e3, 4),
                             "launches_per_tick": 192},
        "batched_over_plain": round(sec_p / sec_b, 3),
        **({"cpu_all_cores": oracle_all_cores(clip, 10.0)} if cpu else {}),
    }


def serving_workload(horizon: float, speedup: float, budget_mib: int) -> dict:
    """Poisson arrivals (8 streams/s, 200-2000 frames at 30 fps, resolutions
    uniform over 320x240 .. 1920x1080), at most 256 concurrent streams,
    admitted against an HBM budget; batched ticks against plain per-stream
    pushes on the same request trace."""
    import torch
    from paper_1503_06959_amd import autotune, kpd, serve, synth
    t0 = time.time()
    bank = serve.ClipBank(n_clips=2, clip_len=48, workers=min(16, os.cpu_count() or 1))
    log(f"[bench] serving clip bank ready in {time.time() - t0:.1f}s")
    tiles = {}
    for res in serve.RESOLUTIONS:
        tiles[res] = autotune.best_tile(res[0], res[1], synth.RES_PRESETS[res][0])[0]
    reqs = serve.poisson_requests(8.0, horizon, 5000, clip_len=48)
    out = {"workload": f"Poisson arrivals 8 streams/s for {horizon:.0f}s of stream time (x{speedup:g} wall speed), "
                       f"200-2000 frames at 30 fps, resolutions uniform over "
                       f"{'/'.join(f'{w}x{h}' for w, h in serve.RESOLUTIONS)}, <= 256 concurrent, "
                       f"HBM budget {budget_mib} MiB, {len(reqs)} requests"}
    for cls in (serve.BatchedBackend, serve.PlainBackend):
        be = cls(max_streams=256, tiles=tiles)
        srv = serve.Server(be, bank, reqs, budget_bytes=budget_mib << 20, max_streams=256, speedup=speedup)
        st = srv.run(horizon)
        be.shutdown()
        torch.cuda.synchronize()
        out[be.name] = st.summary()
        log(f"[bench] serving {be.name}: {out[be.name]}")
    out["batched_over_plain_mpix"] = round(out["batched"]["mpix_per_s"] / max(out["plain"]["mpix_per_s"], 1e-9), 3)
    return out


def serving_saturation(duration: float, budget_mib: int) -> dict:
    """Serving at saturation: 2000 requests (200-2000 frames, resolutions
    uniform over 320x240 .. 1920x1080) all waiting at the start, at most 256
    concurrent streams under the HBM budget; every admitted stream has a
    frame ready at every tick, and ended streams give their slot to waiting
    ones. Batched ticks against plain per-stream pushes, `duration` wall
    seconds each: throughput is the GPU's and the host loop's, not the
    arrival rate's."""
    import torch
    from paper_1503_06959_amd import autotune, serve, synth
    bank = serve.ClipBank(n_clips=2, clip_len=48, workers=min(16, os.cpu_count() or 1))
    tiles = {res: autotune.best_tile(res[0], res[1], synth.RES_PRESETS[res][0])[0] for res in serve.RESOLUTIONS}
    reqs = serve.poisson_requests(8.0, 250.0, 5001, clip_len=48)[:2000]
    out = {"workload": f"{len(reqs)} requests waiting at the start (200-2000 frames each, resolutions uniform over "
                       f"{'/'.join(f'{w}x{h}' for w, h in serve.RESOLUTIONS)}), <= 256 concurrent, HBM budget "
                       f"{budget_mib} MiB, every active stream has a frame ready at every tick, {duration:g}s per "
                       "backend"}
    for cls in (serve.BatchedBackend, serve.PlainBackend):
        be = cls(max_streams=256, tiles=tiles)
        srv = serve.Server(be, bank, reqs, budget_bytes=budget_mib << 20, max_streams=256, saturate=True)
        st = srv.run(duration)
        be.shutdown()
        torch.cuda.synchronize()
        out[be.name] = st.summary()
        log(f"[bench] saturated serving {be.name}: {out[be.name]}")
    out["batched_over_plain_mpix"] = round(out["batched"]["mpix_per_s"] / max(out["plain"]["mpix_per_s"], 1e-9), 3)
    return out


# rocprofv3 runs whose summaries live under profiles/: kernel traces of the
# bench itself, and HBM byte counters (FETCH_SIZE, WRITE_SIZE, one counter
# per run) of single-mode passes and of a plain copy that scales them.
PROFILE_CASES = {
    "kt_c2_640x480_bench": ("trace", "--no-hd --no-batch --no-serve --no-cpu-baseline --steps 10 --warmup 2"),
    "kt_c2_640x480_masked_chunked": ("trace", "--workload c2_640x480 --mode masked --chunked --steps 20 --warmup 2"),
    "kt_c3_1920x1080_full_chunked": ("trace", "--workload c3_1920x1080 --mode full --chunked --steps 10 --warmup 2"),
    "kt_c3_1920x1080_masked_chunked": ("trace",
                                       "--workload c3_1920x1080 --mode masked --chunked --steps 10 --warmup 2"),
    "kt_c3_1920x1080_masked_frame": ("trace", "--workload c3_1920x1080 --mode masked --steps 4 --warmup 1"),
    "kt_c3_1920x1080_full_frame": ("trace", "--workload c3_1920x1080 --mode full --steps 4 --warmup 1"),
    "kt_c2_640x480_layer3_frame": ("trace", "--workload c2_640x480 --mode masked --layer 3 --steps 10 --warmup 2"),
    "kt_batch_64_streams_tick": ("trace", "--batch-only --batch-ticks 60 --warmup 5"),
    "pmc_c2_640x480_masked_chunked": ("pmc", "--workload c2_640x480 --mode masked --chunked --steps 2 --warmup 0"),
    "pmc_c2_640x480_full_chunked": ("pmc", "--workload c2_640x480 --mode full --chunked --steps 2 --warmup 0"),
    "pmc_c3_1920x1080_full_chunked": ("pmc", "--workload c3_1920x1080 --mode full --chunked --steps 2 --warmup 0"),
    "pmc_c3_1920x1080_masked_chunked": ("pmc",
                                        "--workload c3_1920x1080 --mode masked --chunked --steps 2 --warmup 0"),
    "pmc_c2_640x480_layer3_frame": ("pmc", "--workload c2_640x480 --mode masked --layer 3 --steps 2 --warmup 0"),
    "pmc_copy_256MiB": ("pmc", "--copy-calibration 256"),
    "valu_c3_1920x1080_full_chunked": ("valu", "--workload c3_1920x1080 --mode full --chunked --steps 2 --warmup 0"),
}
PMC_COUNTERS = ("FETCH_SIZE", "WRITE_SIZE")
# counter sets of the VALU study, one rocprofv3 run each
VALU_SETS = (("VALUBusy",), ("SQ_INSTS_VALU", "SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_ANY",
                             "SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT", "GRBM_GUI_ACTIVE"))
# kernel -> (push path, the timed kernel id its launches count under)
KERNEL_IDS = {"k_frame1": ("frame", "k_frame"), "k_detect1": ("frame", "k_detect"),
              "k_det1_groups": ("frame", "k_detect"), "k_compact1": ("frame", "k_compact"),
              "k_frame_chunk": ("chunk", "k_frame"), "k_frame_chunk_seq": ("chunk", "k_frame"),
              "k_detect_chunk": ("chunk", "k_detect"), "k_detect_chunk_groups": ("chunk", "k_detect"),
              "k_detect_list_groups": ("chunk", "k_detect"),
              "k_detect_list": ("chunk", "k_detect"), "k_mark_chunk": ("chunk", "k_mark"),
              "k_compact_chunk": ("chunk", "k_compact")}
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = ("kpd_kernels.hip", "kpd_kernels.h", "kpd_geom.h", "kpd_group.h", "kpd_group.hip")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1503_06959_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profile_command(case: str, out: str, counter: str = "", root: str = "$R") -> str:
    kind, args = PROFILE_CASES[case]
    if kind == "trace":
        return (f"rocprofv3 --kernel-trace --stats --output-format csv -d {out}/{case} -o kt -- "
                f"python3 {root}/bench.py {args}")
    tag = counter.split()[0]
    return (f"rocprofv3 --pmc {counter} --output-format csv -d {out}/{case}_{tag} -o p -- "
            f"python3 {root}/bench.py {args}")


def profile_script(out: str) -> str:
    """Shell script that runs every profiling case (started from the
    repository root, R; the profiler runs from /tmp; one counter per --pmc
    run, each under its own time limit). `out` is relative to R."""
    out = "$R/" + out
    lines = ["set -o pipefail", "R=$(pwd)", f"mkdir -p {out}", "cd /tmp && export TMPDIR=/tmp"]
    for case, (kind, _) in PROFILE_CASES.items():
        if kind == "trace":
            lines.append(f"timeout -k 10 300 {profile_command(case, out)} > {out}/{case}.out 2> {out}/{case}.log "
                         f"|| exit $?")
        else:
            sets = PMC_COUNTERS if kind == "pmc" else [" ".join(v) for v in VALU_SETS]
            for c in sets:
                tag = c.split()[0]
                lines.append(f"timeout -s KILL 90 {profile_command(case, out, c)} > {out}/{case}_{tag}.out "
                             f"2> {out}/{case}_{tag}.log || exit $?")
        lines.append(f"echo {case} done")
    return "\n".join(lines) + "\n"


def summarize_profiles(out: str) -> None:
    """Write profiles/*.txt and profiles/traffic.json from the csv files of
    profile_script's runs."""
    import csv
    from collections import defaultdict
    pdir = os.path.join(ROOT, "profiles")
    os.makedirs(pdir, exist_ok=True)
    def short(n):
        n = n.replace("(anonymous namespace)::", "").split("(")[0].replace("kpd::", "")
        if n.startswith("void "):
            n = n[5:]
        return n.split("<")[0]
    for case, (kind, _) in PROFILE_CASES.items():
        if kind != "trace":
            continue
        path = os.path.join(out, case, "kt_kernel_stats.csv")
        if not os.path.exists(path):
            log(f"[bench] no kernel trace of {case} under {out}: its summary is left as it is")
            continue
        rows = list(csv.DictReader(open(path)))
        lines = [f"# kernel durations, {case}", "", "command (R = the repository root, OUT = the output folder given to --profile-script, run from /tmp):",
                 "  " + profile_command(case, "$OUT"), "",
                 f"{'kernel':40s} {'calls':>7s} {'avg_us':>10s} {'min_us':>9s} {'max_us':>9s} {'share':>7s}"]
        for r in rows:
            lines.append(f"{short(r['Name']):40s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:10.3f} "
                         f"{float(r['MinNs']) / 1e3:9.3f} {float(r['MaxNs']) / 1e3:9.3f} "
                         f"{float(r['Percentage']):6.2f}%")
        open(os.path.join(pdir, f"kernel_trace_{case[3:]}.txt"), "w").write("\n".join(lines) + "\n")

    def pmc(case, counter, name=None):
        path = os.path.join(out, f"{case}_{counter}", "p_counter_collection.csv")
        agg = defaultdict(list)
        for r in csv.DictReader(open(path)):
            if name is None or r["Counter_Name"] == name:
                agg[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
        return {k: (sum(v) / len(v), len(v)) for k, v in agg.items()}

    if not os.path.exists(os.path.join(out, "pmc_copy_256MiB_FETCH_SIZE", "p_counter_collection.csv")):
        log(f"[bench] no counter runs under {out}: traffic and VALU summaries are left as they are")
        return
    copy_bytes = 256 << 20
    fc, wc = pmc("pmc_copy_256MiB", "FETCH_SIZE"), pmc("pmc_copy_256MiB", "WRITE_SIZE")
    f_scale = copy_bytes / (fc["__amd_rocclr_copyBuffer"][0] * 1024)
    w_scale = copy_bytes / (wc["__amd_rocclr_copyBuffer"][0] * 1024)
    traffic = {"kernel_source_sha256": kernel_source_hash(), "fetch_scale": round(f_scale, 4),
               "write_scale": round(w_scale, 4), "per_launch_bytes": {}}
    lines = ["# HBM bytes per launch from FETCH_SIZE and WRITE_SIZE (KiB per dispatch, one counter per run)", "",
             f"scale: a plain copy of {copy_bytes} bytes reads FETCH_SIZE {fc['__amd_rocclr_copyBuffer'][0]:.1f} KiB "
             f"and WRITE_SIZE {wc['__amd_rocclr_copyBuffer'][0]:.1f} KiB per dispatch, so bytes = "
             f"FETCH_SIZE x 1024 x {f_scale:.3f} + WRITE_SIZE x 1024 x {w_scale:.3f}", "",
             "commands (R = the repository root, OUT = the output folder given to --profile-script, run from /tmp):"]
    for case in PROFILE_CASES:
        if PROFILE_CASES[case][0] == "pmc":
            for c in PMC_COUNTERS:
                lines.append("  " + profile_command(case, "$OUT", c))
    lines += ["", f"{'case':34s} {'kernel':22s} {'dispatches':>10s} {'FETCH_KiB':>11s} {'WRITE_KiB':>11s} "
                  f"{'bytes/launch':>13s}"]
    for case, (kind, _) in PROFILE_CASES.items():
        if kind != "pmc" or case == "pmc_copy_256MiB":
            continue
        f, w = pmc(case, "FETCH_SIZE"), pmc(case, "WRITE_SIZE")
        wl, mode = case[4:].rsplit("_", 2)[0], case[4:].rsplit("_", 2)[1]
        acc = defaultdict(lambda: [0.0, 0])   # timed kernel id -> summed bytes, dispatches
        for k in sorted(f):
            if k not in KERNEL_IDS or k not in w:
                continue
            b = f[k][0] * 1024 * f_scale + w[k][0] * 1024 * w_scale
            key = f"{wl}/{mode}/{KERNEL_IDS[k][0]}/{KERNEL_IDS[k][1]}"
            acc[key][0] += b * f[k][1]
            acc[key][1] += f[k][1]
            lines.append(f"{case[4:]:34s} {k:22s} {f[k][1]:10d} {f[k][0]:11.2f} {w[k][0]:11.2f} {int(b):13d}")
        for key, (b, n) in acc.items():
            traffic["per_launch_bytes"][key] = int(b / n)
    open(os.path.join(pdir, "hbm_traffic_chunked_and_single.txt"), "w").write("\n".join(lines) + "\n")

    # VALU study of the full-frame 1920x1080 chunk passes
    case = "valu_c3_1920x1080_full_chunked"
    busy = pmc(case, "VALUBusy", "VALUBusy")
    cnt = {c: pmc(case, "SQ_INSTS_VALU", c) for c in VALU_SETS[1]}
    lv = level_sizes(1920, 1080, 5)
    px_oct = 300 * sum(lv)   # pixel-octaves one chunk launch covers (the whole video)
    lines = ["# VALU study, 1920x1080 full-frame chunks (300 frames per launch), one counter set per run", "",
             "commands (R = the repository root, OUT = the output folder given to --profile-script, run from /tmp):"]
    for c in VALU_SETS:
        lines.append("  " + profile_command(case, "$OUT", " ".join(c)))
    lines += ["", f"{'kernel':22s} {'dispatches':>10s} {'VALUBusy%':>10s} {'VALU insts':>14s} {'waves':>10s} "
                  f"{'wait/wave cyc':>13s} {'lane-ops/px-oct':>16s} {'LDS insts':>12s} {'LDS conflict cyc':>17s}"]
    for k in ("k_frame_chunk", "k_detect_chunk_groups", "k_compact_chunk"):
        if k not in busy or k not in cnt["SQ_INSTS_VALU"]:
            continue
        insts, n = cnt["SQ_INSTS_VALU"][k]
        waves = cnt["SQ_WAVES"][k][0]
        wait = cnt["SQ_WAIT_ANY"][k][0] / max(cnt["SQ_WAVE_CYCLES"][k][0], 1)
        per = insts * 64 / px_oct if k == "k_detect_chunk_groups" else float("nan")
        lds = cnt["SQ_INSTS_LDS"].get(k, (float("nan"), 0))[0]
        conf = cnt["SQ_LDS_BANK_CONFLICT"].get(k, (float("nan"), 0))[0]
        lines.append(f"{k:22s} {n:10d} {busy[k][0]:10.1f} {insts:14.0f} {waves:10.0f} {wait:13.3f} {per:16.1f} "
                     f"{lds:12.0f} {conf:17.0f}")
    lines += ["", "lane-ops/px-oct: VALU instructions x 64 lanes per pixel-octave of the launch "
                  f"({px_oct} = 300 frames x {sum(lv)}); wait/wave cyc: SQ_WAIT_ANY over SQ_WAVE_CYCLES; "
                  "LDS conflict cyc: SQ_LDS_BANK_CONFLICT (cycles stalled on LDS bank conflicts)"]
    open(os.path.join(pdir, "valu_c3_1920x1080_full_chunked.txt"), "w").write("\n".join(lines) + "\n")
    with open(TRAFFIC_JSON, "w") as fh:
        json.dump(traffic, fh, indent=1, sort_keys=True)


def traffic_for(wl_name: str, masked: bool, chunk: int, kernel: str, layer=None):
    """Counter-measured HBM bytes per launch of this kernel on this workload,
    or None when not measured or when the kernels changed since."""
    try:
        with open(TRAFFIC_JSON) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_hash():
        return None
    mode = f"layer{layer}" if layer is not None else ("masked" if masked else "full")
    key = f"{wl_name}/{mode}/{'chunk' if chunk > 1 else 'frame'}/{kernel}"
    return t["per_launch_bytes"].get(key)


def copy_calibration(mib: int) -> None:
    """A plain device-to-device copy of known size, for scaling the HBM byte
    counters read on the detection kernels."""
    import torch
    n = mib << 20
    a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "launches": 3}), flush=True)


def main():
    args = parse()
    if args.profile_script:
        sys.stdout.write(profile_script(args.profile_script))
        return
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); streams shard across GPUs "
              f"without communication, see the design notes", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    from paper_1503_06959_amd import kpd
    global TILE, GROUPS
    TILE = args.tile
    GROUPS = tuple(int(v) for v in args.groups.split("x"))
    if args.batch_only:
        print(json.dumps(batched_workload(kpd, args.batch_ticks, args.batch_clip, args.warmup, cpu=False)), flush=True)
        return

    wl = Workload(args.workload)
    if args.mode != "both":
        masked = args.mode == "masked"
        chunk = chunk_of(args, wl) if args.chunked else 0
        layer = args.layer if masked else None
        if layer is not None and chunk:
            sys.exit("--layer runs on single-frame pushes: leave out --chunked")
        log(f"[bench] {args.mode} pass only, chunk {chunk}, layer {layer}")
        r = run_workload(kpd, wl, wl.det.id_thresh if masked else -1, args, chunk=chunk, layer=layer)
        stats = r if chunk <= 1 else run_workload(kpd, wl, wl.det.id_thresh if masked else -1, args,
                                                  want_profile=False)
        print(json.dumps({"workload": wl.describe(wl.det.id_thresh if masked else -1), "chunk": chunk,
                          "layer": layer,
                          "value": round(r["mpix_per_s"], 2), "unit": "Mpixel/s",
                          "frames_per_s": round(r["frames_per_s"], 1),
                          "latency_ms": {"p50": round(r["lat_p50"], 4), "p99": round(r["lat_p99"], 4)},
                          **({"device_ms_per_frame": {"p50": round(r["dev_p50"], 4), "p99": round(r["dev_p99"], 4)}}
                             if "dev_p50" in r else {}),
                          "roofline": roofline_of(wl, r, masked, stats=stats)}), flush=True)
        return
    K = chunk_of(args, wl)
    log(f"[bench] masked pass, chunks of {K}")
    masked_c = run_workload(kpd, wl, wl.det.id_thresh, args, chunk=K)
    log(f"[bench] masked {masked_c['mpix_per_s']:.1f} Mpx/s; full-frame pass")
    full_c = run_workload(kpd, wl, -1, args, chunk=K)
    log(f"[bench] full-frame {full_c['mpix_per_s']:.1f} Mpx/s; per-frame pushes")
    masked = run_workload(kpd, wl, wl.det.id_thresh, args)
    full = run_workload(kpd, wl, -1, args)
    log(f"[bench] per-frame masked {masked['mpix_per_s']:.1f}, full {full['mpix_per_s']:.1f} Mpx/s")
    skipped = 1.0 - sum(masked["marked"][1:]) / max(1, (wl.F - 1) * wl.ncell)

    out = {
        "metric": METRIC,
        "value": round(masked_c["mpix_per_s"], 2),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(masked_c["sec_per_pass"] * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": wl.describe(wl.det.id_thresh), "frames_per_step": wl.F,
                   "frame": f"{wl.W}x{wl.H}", "push": f"push_frames, {K} consecutive frames per call",
                   "parallelism": "1 stream, 1 GPU"},
        "frames_per_s": round(masked_c["frames_per_s"], 1),
        "latency_ms": {"p50": round(masked["lat_p50"], 4), "p99": round(masked["lat_p99"], 4),
                       "what": "streaming: push_frame -> get_keypoints on the host, one frame in flight"},
        "chunk_latency_ms": {"p50": round(masked_c["lat_p50"], 4), "p99": round(masked_c["lat_p99"], 4),
                             "what": f"push_frames of {K} frames -> last frame's keypoints on the host"},
        "skipped_cell_frac": round(skipped, 4),
        "full_frame": {"value": round(full_c["mpix_per_s"], 2), "unit": "Mpixel/s",
                       "frames_per_s": round(full_c["frames_per_s"], 1),
                       "ms_per_step": round(full_c["sec_per_pass"] * 1e3, 4),
                       "chunk_latency_ms": {"p50": round(full_c["lat_p50"], 4),
                                            "p99": round(full_c["lat_p99"], 4)},
                       "roofline": roofline_of(wl, full_c, False, stats=full)},
        "masked_over_full": round(masked_c["mpix_per_s"] / full_c["mpix_per_s"], 3),
        "roofline": roofline_of(wl, masked_c, True, stats=masked),
        "per_frame_push": {
            "what": "streaming mode: one push_frame call per frame",
            "masked": {"value": round(masked["mpix_per_s"], 2), "unit": "Mpixel/s",
                       "frames_per_s": round(masked["frames_per_s"], 1),
                       "ms_per_step": round(masked["sec_per_pass"] * 1e3, 4),
                       "latency_ms": {"p50": round(masked["lat_p50"], 4), "p99": round(masked["lat_p99"], 4)},
                       "device_ms_per_frame": {"p50": round(masked["dev_p50"], 4), "p99": round(masked["dev_p99"], 4)},
                       "roofline": roofline_of(wl, masked, True)},
            "full_frame": {"value": round(full["mpix_per_s"], 2), "unit": "Mpixel/s",
                           "frames_per_s": round(full["frames_per_s"], 1),
                           "ms_per_step": round(full["sec_per_pass"] * 1e3, 4),
                           "latency_ms": {"p50": round(full["lat_p50"], 4), "p99": round(full["lat_p99"], 4)},
                           "device_ms_per_frame": {"p50": round(full["dev_p50"], 4), "p99": round(full["dev_p99"], 4)},
                           "roofline": roofline_of(wl, full, False)},
            "masked_over_full": round(masked["mpix_per_s"] / full["mpix_per_s"], 3),
        },
    }
    top = wl.det.n_octaves - 1
    log(f"[bench] per-pixel mask on layer {top}")
    lm = run_workload(kpd, wl, wl.det.id_thresh, args, layer=top)
    out["layer_mask"] = {
        "what": f"per-pixel |I_n - I_(n-1)| > T_I on pyramid layer {top} (the top octave), Eq. 1 per feature "
                "position, one push_frame per frame",
        "value": round(lm["mpix_per_s"], 2), "unit": "Mpixel/s", "frames_per_s": round(lm["frames_per_s"], 1),
        "ms_per_step": round(lm["sec_per_pass"] * 1e3, 4),
        "latency_ms": {"p50": round(lm["lat_p50"], 4), "p99": round(lm["lat_p99"], 4)},
        "touched_cell_frac": round(sum(lm["marked"][1:]) / max(1, (wl.F - 1) * wl.ncell), 4),
        "roofline": roofline_of(wl, lm, True),
    }
    for key, mode in (("chunked", 1), ("octave_masks_chunked", 2)):
        log(f"[bench] per-pixel mask mode {mode} in chunks of {K}")
        lc = run_workload(kpd, wl, wl.det.id_thresh, args, chunk=K, layer=top, mask_mode=mode)
        kern = {k: round(v[0] * 1e3 / lc["kernels"]["passes"], 2) for k, v in lc["kernels"].items() if k != "passes"}
        out["layer_mask"][key] = {
            "what": (f"mode {mode} ({'layer ' + str(top) + ' for every octave' if mode == 1 else 'each octave on its own level'})"
                     f", push_frames chunks of {K}: diff, mark, listed detection, per-cell merge of Eq. 1 per "
                     "feature along the chunk, compaction"),
            "value": round(lc["mpix_per_s"], 2), "unit": "Mpixel/s", "frames_per_s": round(lc["frames_per_s"], 1),
            "ms_per_step": round(lc["sec_per_pass"] * 1e3, 4),
            "chunk_latency_ms": {"p50": round(lc["lat_p50"], 4), "p99": round(lc["lat_p99"], 4)},
            "kernel_us_per_pass": kern,
        }
    log("[bench] keypoint-binning mask only (T_I off, T_H = 2)")
    kbc = run_workload(kpd, wl, 255, args, chunk=K, kb_thresh=2, want_profile=False)
    kbf = run_workload(kpd, wl, 255, args, kb_thresh=2, want_profile=False)
    out["kb_only"] = {
        "what": "the keypoint-binning mask alone (Sec. 3.2, Eqs. 3-4): T_I off (255), T_H = 2; marks need the "
                "previous frame's counts, so chunks run the chained detection pass",
        "chunked": {"value": round(kbc["mpix_per_s"], 2), "unit": "Mpixel/s", "frames_per_s": round(kbc["frames_per_s"], 1),
                    "ms_per_step": round(kbc["sec_per_pass"] * 1e3, 4)},
        "per_frame_push": {"value": round(kbf["mpix_per_s"], 2), "unit": "Mpixel/s",
                           "frames_per_s": round(kbf["frames_per_s"], 1),
                           "latency_ms": {"p50": round(kbf["lat_p50"], 4), "p99": round(kbf["lat_p99"], 4)}},
        "marked_cell_frac": round(sum(kbf["marked"][1:]) / max(1, (wl.F - 1) * wl.ncell), 4),
    }
    log("[bench] layer study")
    out["layer_study"] = layer_study(kpd, wl, args)
    for which in FEATURE_PASSES:
        log(f"[bench] {which}")
        out[which] = feature_workload(kpd, wl, args, which)
    log("[bench] temporally coherent detector")
    out["tcd"] = tcd_workload(kpd, wl, args)
    log("[bench] intra-octave layers")
    out["intra_octaves"] = intra_octave_workload(kpd, wl, args)
    log("[bench] batch of layered streams")
    out["intra_octaves"]["batched_64_streams"] = layered_batch_workload(kpd, wl, args)
    out["host_frames"] = host_frames_pass(kpd, wl, max(1, args.steps // 10))
    if not args.no_hd:
        del wl
        torch.cuda.empty_cache()
        hd = Workload("c3_1920x1080")
        log("[bench] 1080p passes")
        hmc = run_workload(kpd, hd, hd.det.id_thresh, args, chunk=K)
        hfc = run_workload(kpd, hd, -1, args, chunk=K)
        hm = run_workload(kpd, hd, hd.det.id_thresh, args)
        hf = run_workload(kpd, hd, -1, args)
        lv = level_sizes(hd.W, hd.H, hd.det.n_octaves)
        N, P = lv[0], sum(lv[1:])
        kps = sum(hf["total_kp"]) / hd.F
        b_full = N + 2 * P + 8 * kps

        def eff(r):
            e = b_full * hd.F / r["sec_per_pass"] / 1e9
            return {"effective_hbm_GBs": round(e, 2), "effective_hbm_frac": round(e / HBM_PEAK_GBS, 5),
                    "algorithmic_bytes_per_frame": int(b_full)}

        out["hd_1080p"] = {
            "workload": hd.describe(hd.det.id_thresh),
            "push": f"push_frames, {K} consecutive frames per call",
            "masked": {"value": round(hmc["mpix_per_s"], 2), "unit": "Mpixel/s",
                       "frames_per_s": round(hmc["frames_per_s"], 1),
                       "chunk_latency_ms": {"p50": round(hmc["lat_p50"], 4), "p99": round(hmc["lat_p99"], 4)},
                       "roofline": roofline_of(hd, hmc, True, stats=hm)},
            "full_frame": dict({"value": round(hfc["mpix_per_s"], 2), "unit": "Mpixel/s",
                                "frames_per_s": round(hfc["frames_per_s"], 1),
                                "chunk_latency_ms": {"p50": round(hfc["lat_p50"], 4),
                                                     "p99": round(hfc["lat_p99"], 4)},
                                "roofline": roofline_of(hd, hfc, False, stats=hf)}, **eff(hfc)),
            "per_frame_push": {
                "masked": {"value": round(hm["mpix_per_s"], 2), "unit": "Mpixel/s",
                           "frames_per_s": round(hm["frames_per_s"], 1),
                           "latency_ms": {"p50": round(hm["lat_p50"], 4), "p99": round(hm["lat_p99"], 4)},
                           "device_ms_per_frame": {"p50": round(hm["dev_p50"], 4), "p99": round(hm["dev_p99"], 4)},
                           "roofline": roofline_of(hd, hm, True)},
                "full_frame": dict({"value": round(hf["mpix_per_s"], 2), "unit": "Mpixel/s",
                                    "frames_per_s": round(hf["frames_per_s"], 1),
                                    "latency_ms": {"p50": round(hf["lat_p50"], 4), "p99": round(hf["lat_p99"], 4)},
                                    "device_ms_per_frame": {"p50": round(hf["dev_p50"], 4),
                                                            "p99": round(hf["dev_p99"], 4)},
                                    "roofline": roofline_of(hd, hf, False)}, **eff(hf)),
                "masked_over_full_device_p50": round(hm["dev_p50"] / hf["dev_p50"], 3),
                "masked_over_full_device_p99": round(hm["dev_p99"] / hf["dev_p99"], 3),
            },
            "skipped_cell_frac": round(1.0 - sum(hm["marked"][1:]) / max(1, (hd.F - 1) * hd.ncell), 4),
        }
        # The headline roofline: the 1080p masked chunk pass, whose 300 frames
        # (622 MB) exceed the 256 MB Infinity Cache, so its bytes come from HBM.
        out["roofline_c2_640x480"] = dict(out["roofline"], note="the 300 C2 frames (92 MB) and their pyramid fit "
                                          "in the 256 MB Infinity Cache across steps: not HBM evidence")
        out["roofline"] = dict(out["hd_1080p"]["masked"]["roofline"],
                               workload=f"{hd.name} masked (T_I={hd.det.id_thresh}), push_frames of {K} frames")
        # the pass's HBM-bound kernel beside it (when the detection of the
        # marked cells, latency-bound, takes longer than the tile pass)
        out["roofline_tile_pass"] = dict(roofline_of(hd, hmc, True, stats=hm, kernel="k_frame"),
                                         workload=out["roofline"]["workload"])
        if not args.no_cpu_baseline:
            log("[bench] 1080p cpu baseline (oracle)")
            out["hd_1080p"]["cpu_baseline"] = cpu_baseline(hd, args.cpu_seconds)
        wl = hd
    if not args.no_batch:
        del wl
        torch.cuda.empty_cache()
        log("[bench] batched 64-stream ticks")
        out["batched_64_streams"] = batched_workload(kpd, args.batch_ticks, args.batch_clip, args.warmup)
        wl = None
    if not args.no_serve:
        wl = None
        torch.cuda.empty_cache()
        log("[bench] serving")
        out["serving"] = serving_workload(args.serve_horizon, args.serve_speedup, args.serve_budget_mib)
        torch.cuda.empty_cache()
        log("[bench] serving at saturation")
        out["serving_saturated"] = serving_saturation(args.saturation_seconds, args.saturation_budget_mib)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        from paper_1503_06959_amd import synth
        base = Workload(args.workload) if wl is None or wl.name != args.workload else wl
        out["cpu_baseline"] = cpu_baseline(base, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
