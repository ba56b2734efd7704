"""Serving loop: video streams arrive, are admitted against an HBM budget,
and share batched ticks as their frames arrive (continuous batching).

Pieces:
  * ``poisson_requests``: arrival process of streams (rate per second,
    durations in frames at a frame rate, resolutions drawn from a set);
  * ``Admission``: host-side admission control. A stream is admitted when a
    slot is free and its device footprint (``stream_bytes``) fits in the
    budget, in arrival order; the rest wait. Pure host logic, testable with a
    fake clock and fake footprints;
  * ``ClipBank``: pre-rendered synthetic clips per resolution, resident in
    HBM; a stream plays one clip forward and back from its own offset;
  * ``BatchedBackend`` / ``PlainBackend``: run a set of due frames as one
    batched tick, or as one push per stream;
  * ``Server``: the loop. Every iteration it admits waiting streams, stages
    the frame of every active stream whose arrival time has passed, runs one
    tick, gathers the keypoints of all of them to the host in one copy, and
    records each frame's latency from its arrival to its keypoints on the
    host. Streams that have delivered all their frames release their slot
    and budget.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

RESOLUTIONS = ((320, 240), (640, 480), (1280, 720), (1920, 1080))


@dataclasses.dataclass
class Request:
    sid: int
    arrival: float          # seconds since the start of the run
    n_frames: int
    res: Tuple[int, int]
    clip: int
    offset: int


def poisson_requests(rate: float, horizon: float, seed: int, frames: Tuple[int, int] = (200, 2000),
                     resolutions: Sequence[Tuple[int, int]] = RESOLUTIONS, n_clips: int = 2,
                     clip_len: int = 48) -> List[Request]:
    rng = np.random.Generator(np.random.PCG64(seed))
    out, t, sid = [], 0.0, 0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= horizon:
            return out
        res = resolutions[int(rng.integers(0, len(resolutions)))]
        out.append(Request(sid, t, int(rng.integers(frames[0], frames[1] + 1)), res,
                           int(rng.integers(0, n_clips)), int(rng.integers(0, 2 * clip_len - 2))))
        sid += 1


class Admission:
    """First-come-first-served admission under a slot cap and a byte budget."""

    def __init__(self, budget_bytes: int, max_streams: int, bytes_of: Callable[[Request], int]):
        self.budget, self.max_streams, self.bytes_of = budget_bytes, max_streams, bytes_of
        self.waiting: collections.deque = collections.deque()
        self.active: Dict[int, int] = {}   # sid -> bytes
        self.used = 0
        self.deferred = 0                  # requests that had to wait at least once
        self._seen_wait = set()

    def offer(self, req: Request) -> None:
        if self.bytes_of(req) > self.budget:
            raise ValueError(f"stream {req.sid} can never fit the budget")
        self.waiting.append(req)

    def admit(self) -> List[Request]:
        out = []
        while self.waiting:
            req = self.waiting[0]
            need = self.bytes_of(req)
            if len(self.active) >= self.max_streams or self.used + need > self.budget:
                if req.sid not in self._seen_wait:
                    self._seen_wait.add(req.sid)
                    self.deferred += 1
                break
            self.waiting.popleft()
            self.active[req.sid] = need
            self.used += need
            out.append(req)
        return out

    def release(self, sid: int) -> None:
        self.used -= self.active.pop(sid)


def pingpong(k: int, n: int) -> int:
    if n == 1:
        return 0
    m = k % (2 * n - 2)
    return m if m < n else 2 * n - 2 - m


def _gen_bank(args):
    from . import synth
    w, h, n_clips, clip_len = args
    return synth.clip_bank(w, h, n_clips, clip_len)


class ClipBank:
    """Pre-rendered clips per resolution, on the device: [clips, frames, H, W]."""

    def __init__(self, resolutions=RESOLUTIONS, n_clips: int = 2, clip_len: int = 48, workers: int = 8):
        import torch
        from concurrent.futures import ProcessPoolExecutor
        self.clip_len = clip_len
        with ProcessPoolExecutor(max_workers=workers) as ex:
            banks = list(ex.map(_gen_bank, [(w, h, n_clips, clip_len) for (w, h) in resolutions]))
        self.host = {res: b for res, b in zip(resolutions, banks)}
        self.dev = {res: torch.from_numpy(b).cuda() for res, b in self.host.items()}
        # one view per frame, made once: a tick looks frames up by index
        self.views = {res: [[d[c, f] for f in range(d.shape[1])] for c in range(d.shape[0])]
                      for res, d in self.dev.items()}

    def frame(self, req: Request, k: int):
        return self.views[req.res][req.clip][pingpong(req.offset + k, self.clip_len)]

    def host_frame(self, req: Request, k: int) -> np.ndarray:
        return self.host[req.res][req.clip, pingpong(req.offset + k, self.clip_len)]


def preset_params(kpd, res: Tuple[int, int], tile: int = 0):
    from . import synth
    d = synth.RES_PRESETS[res][0]
    return kpd.make_params(d.fast_t, d.n_octaves, d.grid_cols, d.grid_rows, d.id_thresh, d.kb_thresh, tile)


class BatchedBackend:
    """All admitted streams attached to one batch; one tick per loop turn;
    results of every ticked stream gathered to the host in one copy."""

    name = "batched"

    def __init__(self, max_streams: int, tiles: Optional[Dict[Tuple[int, int], int]] = None,
                 gather_cap: int = 1 << 21, use_graph: bool = True):
        import torch
        from . import kpd
        from .batch import Batch
        self.kpd, self.torch = kpd, torch
        self.batch = Batch(max_streams=max_streams, use_graph=use_graph)
        self.tiles = tiles or {}
        self.streams: Dict[int, object] = {}
        self.order: List[int] = []
        self.out = torch.empty(gather_cap * 8, dtype=torch.uint8, device="cuda")
        self.counts = torch.empty(max_streams, dtype=torch.int32, device="cuda")
        self.staged: List[int] = []
        self.frames: List[object] = []

    def bytes_of(self, req: Request) -> int:
        return self.kpd.stream_bytes(req.res[0], req.res[1], preset_params(self.kpd, req.res))

    def open(self, req: Request) -> None:
        s = self.batch.open_stream(req.res[0], req.res[1],
                                   preset_params(self.kpd, req.res, self.tiles.get(req.res, 0)))
        self.streams[req.sid] = s
        self.order.append(req.sid)

    def push(self, sid: int, frame) -> None:
        self.staged.append(sid)
        self.frames.append(frame)

    def run(self) -> Dict[int, np.ndarray]:
        kpd = self.kpd
        # every staged frame in one library call, then the tick
        with self.torch.cuda.stream(self.batch.torch_stream):
            self.batch.push_many([self.streams[sid] for sid in self.staged], self.frames, retain=True)
        self.frames = []
        self.batch.tick()
        kpd.batch_gather(self.batch.handle, self.out, self.counts)
        with self.torch.cuda.stream(self.batch.torch_stream):
            counts = self.counts[:len(self.order)].cpu().numpy()
            total = int(counts.sum())
            blob = self.out[:8 * total].cpu().numpy()
        kps = blob.view(kpd.KEYPOINT_DTYPE)
        res, off = {}, 0
        staged = set(self.staged)
        for sid, c in zip(self.order, counts):
            if sid in staged:
                res[sid] = kps[off:off + c]
            off += int(c)
        self.staged = []
        return res

    def close(self, sid: int) -> None:
        s = self.streams.pop(sid)
        self.batch.detach(s)
        self.order.remove(sid)
        s.close()

    def shutdown(self) -> None:
        for sid in list(self.streams):
            self.close(sid)
        self.batch.close()


class PlainBackend:
    """The same streams pushed one by one (two launches per stream and
    frame), each stream's keypoints fetched on its own."""

    name = "plain"

    def __init__(self, max_streams: int, tiles=None):
        import torch
        from . import kpd
        self.kpd, self.torch = kpd, torch
        self.stream = torch.cuda.Stream()
        self.streams: Dict[int, object] = {}
        self.staged: List[int] = []

    def bytes_of(self, req: Request) -> int:
        return self.kpd.stream_bytes(req.res[0], req.res[1], preset_params(self.kpd, req.res))

    def open(self, req: Request) -> None:
        self.streams[req.sid] = self.kpd.Stream(req.res[0], req.res[1], preset_params(self.kpd, req.res),
                                                stream=self.stream)

    def push(self, sid: int, frame) -> None:
        self.streams[sid].push(frame, retain=True)
        self.staged.append(sid)

    def run(self) -> Dict[int, np.ndarray]:
        res = {sid: self.streams[sid].keypoints()[0] for sid in self.staged}
        self.staged = []
        return res

    def close(self, sid: int) -> None:
        self.streams.pop(sid).close()

    def shutdown(self) -> None:
        for sid in list(self.streams):
            self.close(sid)


@dataclasses.dataclass
class ServeStats:
    backend: str
    wall_s: float
    frames: int
    pixels: int
    latencies_ms: List[float]
    admitted: int
    deferred: int
    max_active: int
    ticks: int

    def summary(self) -> dict:
        lat = np.array(self.latencies_ms) if self.latencies_ms else np.zeros(1)
        return {
            "backend": self.backend, "wall_s": round(self.wall_s, 3), "frames": self.frames,
            "mpix_per_s": round(self.pixels / self.wall_s / 1e6, 2),
            "frames_per_s": round(self.frames / self.wall_s, 1),
            "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                           "p99": round(float(np.percentile(lat, 99)), 3),
                           "max": round(float(lat.max()), 3)},
            "streams_admitted": self.admitted, "streams_deferred": self.deferred,
            "max_concurrent": self.max_active, "ticks": self.ticks,
        }


class Server:
    """Runs requests against a backend. Simulated time runs `speedup` times
    faster than the wall clock: frame k of a stream admitted at simulated
    time a arrives at a + k / fps. Latencies are wall-clock milliseconds from
    a frame's arrival to its keypoints on the host.

    saturate: every request has arrived at the start and every admitted
    stream has its next frame waiting at every tick (the GPU never waits for
    a frame rate): each tick takes one frame of every active stream, streams
    that end give their slot and budget to waiting ones, and the run lasts
    `horizon` wall-clock seconds. A frame's latency runs from its tick's
    start to its keypoints on the host."""

    def __init__(self, backend, bank, requests: List[Request], budget_bytes: int, max_streams: int = 256,
                 fps: float = 30.0, speedup: float = 1.0, clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep, record: Sequence[int] = (), saturate: bool = False):
        self.backend, self.bank, self.requests = backend, bank, sorted(requests, key=lambda r: r.arrival)
        self.adm = Admission(budget_bytes, max_streams, backend.bytes_of)
        self.fps, self.speedup, self.clock, self.sleep = fps, speedup, clock, sleep
        self.saturate = saturate
        self.record = set(record)
        self.recorded: Dict[int, List[np.ndarray]] = {sid: [] for sid in self.record}
        self.req_of: Dict[int, Request] = {r.sid: r for r in self.requests}

    def run(self, horizon: float) -> ServeStats:
        if self.saturate:
            return self._run_saturated(horizon)
        t0 = self.clock()
        sim = lambda: (self.clock() - t0) * self.speedup
        nxt = 0
        active: Dict[int, List] = {}     # sid -> [start_sim, next_frame]
        lat, frames, pixels, ticks, admitted, max_active = [], 0, 0, 0, 0, 0
        while True:
            now = sim()
            if now >= horizon:
                break
            while nxt < len(self.requests) and self.requests[nxt].arrival <= now:
                self.adm.offer(self.requests[nxt])
                nxt += 1
            for req in self.adm.admit():
                self.backend.open(req)
                active[req.sid] = [now, 0]
                admitted += 1
            max_active = max(max_active, len(active))
            due = []
            for sid, st in active.items():
                req = self.req_of[sid]
                k = st[1]
                if k < req.n_frames:
                    arr = st[0] + k / self.fps
                    if arr <= now:
                        self.backend.push(sid, self.bank.frame(req, k))
                        due.append((sid, arr))
                        st[1] += 1
            if due:
                results = self.backend.run()
                done = sim()
                ticks += 1
                for sid, arr in due:
                    lat.append((done - arr) / self.speedup * 1e3)
                    req = self.req_of[sid]
                    pixels += req.res[0] * req.res[1]
                    frames += 1
                    if sid in self.record:
                        self.recorded[sid].append(results[sid].copy())
                for sid in [s for s, st in active.items() if st[1] >= self.req_of[s].n_frames]:
                    self.backend.close(sid)
                    self.adm.release(sid)
                    del active[sid]
            else:
                # nothing due: wait for the next frame or arrival
                wake = [st[0] + st[1] / self.fps for sid, st in active.items()
                        if st[1] < self.req_of[sid].n_frames]
                if nxt < len(self.requests):
                    wake.append(self.requests[nxt].arrival)
                gap = (min(wake) - now) / self.speedup if wake else 1e-3
                self.sleep(min(max(gap, 0.0), 1e-3))
        wall = self.clock() - t0
        for sid in list(active):
            self.backend.close(sid)
            self.adm.release(sid)
        return ServeStats(self.backend.name, wall, frames, pixels, lat, admitted, self.adm.deferred, max_active,
                          ticks)

    def _run_saturated(self, duration: float) -> ServeStats:
        for req in self.requests:
            self.adm.offer(req)
        t0 = self.clock()
        active: Dict[int, int] = {}      # sid -> next frame
        lat, frames, pixels, ticks, admitted, max_active = [], 0, 0, 0, 0, 0
        while self.clock() - t0 < duration:
            for req in self.adm.admit():
                self.backend.open(req)
                active[req.sid] = 0
                admitted += 1
            if not active:
                break
            max_active = max(max_active, len(active))
            start = self.clock()
            for sid, k in active.items():
                self.backend.push(sid, self.bank.frame(self.req_of[sid], k))
            results = self.backend.run()
            done = self.clock()
            ticks += 1
            for sid in active:
                lat.append((done - start) * 1e3)
                req = self.req_of[sid]
                pixels += req.res[0] * req.res[1]
                frames += 1
                active[sid] += 1
                if sid in self.record:
                    self.recorded[sid].append(results[sid].copy())
            for sid in [s for s, k in active.items() if k >= self.req_of[s].n_frames]:
                self.backend.close(sid)
                self.adm.release(sid)
                del active[sid]
        wall = self.clock() - t0
        for sid in list(active):
            self.backend.close(sid)
            self.adm.release(sid)
        return ServeStats(self.backend.name, wall, frames, pixels, lat, admitted, self.adm.deferred, max_active,
                          ticks)
