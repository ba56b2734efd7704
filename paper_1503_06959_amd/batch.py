"""Batched ticks over many video streams (binding of the batch calls in
include/kpd.h).

A Batch owns a HIP stream (a torch stream) and a device scratch tensor for
its tick tables. Streams are opened on that HIP stream and attached; each
tick runs the next frame of every stream that staged one, in four launches
(or, after set_single_launch(True), one launch of co-resident workgroups
whose phases are separated by device-wide barriers), captured once as a HIP
graph and replayed while the set of attached streams stays the same.
Streams that compute descriptors or refined values add one launch per tick.
"""
from __future__ import annotations

from typing import Dict, Optional

import torch

from . import kpd


class Batch:
    def __init__(self, max_streams: int = 256, max_blocks: int = 1 << 18, use_graph: bool = True,
                 stream: Optional[torch.cuda.Stream] = None):
        self.torch_stream = stream if stream is not None else torch.cuda.Stream()
        self.max_streams, self.max_blocks = max_streams, max_blocks
        nbytes = kpd.batch_bytes(max_streams, max_blocks)
        if nbytes == 0:
            raise ValueError("bad batch capacity")
        self.scratch = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.handle = kpd.open_batch(max_streams, max_blocks, self.scratch, self.torch_stream, use_graph)
        self.streams: Dict[int, kpd.Stream] = {}
        self._held: Dict[int, list] = {}

    def open_stream(self, width: int, height: int, params: kpd.KpdParams) -> kpd.Stream:
        s = kpd.Stream(width, height, params, stream=self.torch_stream)
        kpd.batch_attach(self.handle, s.handle)
        self.streams[s.handle] = s
        self._held[s.handle] = [None, None]
        return s

    def attach(self, s: kpd.Stream) -> None:
        kpd.batch_attach(self.handle, s.handle)
        self.streams[s.handle] = s
        self._held[s.handle] = [None, None]

    def detach(self, s: kpd.Stream) -> None:
        kpd.batch_detach(self.handle, s.handle)
        self.streams.pop(s.handle, None)
        self._held.pop(s.handle, None)

    def push(self, s: kpd.Stream, frame, retain: bool = False) -> None:
        kpd.batch_push(self.handle, s.handle, frame, retain)
        if retain:
            h = self._held[s.handle]
            self._held[s.handle] = [h[1], frame]

    def push_many(self, streams, frames, retain: bool = False) -> None:
        """Stage one device frame for each stream in one library call (the
        same as push() for each pair, in order)."""
        kpd.batch_push_many(self.handle, [s.handle for s in streams], [f.data_ptr() for f in frames],
                            [f.stride(0) for f in frames], retain)
        if retain:
            for s, f in zip(streams, frames):
                h = self._held[s.handle]
                self._held[s.handle] = [h[1], f]

    def set_single_launch(self, on: bool) -> None:
        kpd.batch_set_single_launch(self.handle, on)

    def tick(self) -> None:
        kpd.batch_tick(self.handle)

    def synchronize(self) -> None:
        self.torch_stream.synchronize()

    def close(self) -> None:
        if self.handle:
            kpd.close_batch(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
