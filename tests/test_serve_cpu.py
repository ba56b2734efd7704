"""Host logic of the serving loop (admission and continuous batching), run
on the CPU with a fake clock and a fake backend. The fake backend only
records what it was asked to run; it is a test double for timing and
admission, not a second compute path."""
import numpy as np
import pytest

from paper_1503_06959_amd.serve import Admission, Request, Server, poisson_requests, pingpong


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-4)


class FakeBackend:
    name = "fake"

    def __init__(self, clock, cost=0.002, size=100):
        self.clock, self.cost, self.size = clock, cost, size
        self.open_sids, self.closed, self.staged, self.ticks = set(), [], [], []

    def bytes_of(self, req):
        return self.size if isinstance(self.size, int) else self.size[req.res]

    def open(self, req):
        assert req.sid not in self.open_sids
        self.open_sids.add(req.sid)

    def push(self, sid, frame):
        assert sid in self.open_sids
        assert sid not in self.staged, "two frames of one stream in a tick"
        self.staged.append(sid)

    def run(self):
        self.clock.t += self.cost
        self.ticks.append(list(self.staged))
        out = {sid: np.zeros(0) for sid in self.staged}
        self.staged = []
        return out

    def close(self, sid):
        self.open_sids.remove(sid)
        self.closed.append(sid)


class FakeBank:
    def frame(self, req, k):
        return (req.sid, k)


def req(sid, arrival, n=10, res=(320, 240)):
    return Request(sid, arrival, n, res, 0, 0)


def test_admission_defers_until_budget_frees():
    a = Admission(250, 10, lambda r: 100)
    for i in range(3):
        a.offer(req(i, 0.0))
    assert [r.sid for r in a.admit()] == [0, 1]
    assert a.deferred == 1 and a.used == 200
    assert a.admit() == []
    a.release(0)
    assert [r.sid for r in a.admit()] == [2]
    assert a.used == 200


def test_admission_slot_cap_and_fifo_order():
    a = Admission(10_000, 2, lambda r: 1)
    for i in range(4):
        a.offer(req(i, 0.0))
    assert [r.sid for r in a.admit()] == [0, 1]
    a.release(1)
    assert [r.sid for r in a.admit()] == [2]
    with pytest.raises(ValueError):
        Admission(10, 2, lambda r: 11).offer(req(9, 0.0))


def test_poisson_requests_reproducible_and_rate():
    a = poisson_requests(8.0, 100.0, 5)
    b = poisson_requests(8.0, 100.0, 5)
    assert [(r.arrival, r.n_frames, r.res) for r in a] == [(r.arrival, r.n_frames, r.res) for r in b]
    assert 650 < len(a) < 950
    assert all(200 <= r.n_frames <= 2000 for r in a)
    assert {r.res for r in a} == {(320, 240), (640, 480), (1280, 720), (1920, 1080)}


def test_pingpong_playback():
    assert [pingpong(k, 4) for k in range(8)] == [0, 1, 2, 3, 2, 1, 0, 1]


def test_server_continuous_batching_delivers_every_frame_once():
    clock = FakeClock()
    be = FakeBackend(clock, cost=0.02)   # a tick long enough for frames to pile up
    reqs = [req(0, 0.0, 6), req(1, 0.05, 6), req(2, 0.12, 3)]
    srv = Server(be, FakeBank(), reqs, budget_bytes=1000, fps=30.0, clock=clock, sleep=clock.sleep)
    st = srv.run(horizon=1.0)
    assert st.frames == 15 and st.admitted == 3
    assert sorted(be.closed) == [0, 1, 2]
    # a stream that arrives later joins ticks already running for the others
    assert [t for t in be.ticks if 0 in t and 1 in t]
    assert [t for t in be.ticks if 1 in t and 2 in t]
    # every frame of a stream goes through exactly one tick, in order
    for sid, n in ((0, 6), (1, 6), (2, 3)):
        assert sum(1 for t in be.ticks if sid in t) == n
    # a frame waits at most for the tick in flight plus its own tick
    assert max(st.latencies_ms) <= 2 * 20.0 + 1.0


def test_server_admission_binds_under_small_budget():
    clock = FakeClock()
    be = FakeBackend(clock, size=400)
    reqs = [req(i, 0.01 * i, 5) for i in range(5)]
    srv = Server(be, FakeBank(), reqs, budget_bytes=1000, fps=30.0, clock=clock, sleep=clock.sleep)
    st = srv.run(horizon=2.0)
    assert st.deferred >= 1            # the third stream had to wait
    assert st.max_active == 2          # 2 x 400 fits in 1000, 3 x 400 does not
    assert st.admitted == 5 and st.frames == 25


def test_server_speedup_scales_arrivals():
    clock = FakeClock()
    be = FakeBackend(clock, cost=0.0001)
    reqs = [req(0, 0.0, 30)]
    srv = Server(be, FakeBank(), reqs, budget_bytes=1000, fps=30.0, speedup=10.0, clock=clock, sleep=clock.sleep)
    st = srv.run(horizon=2.0)
    assert st.frames == 30
    # 30 frames at 30 fps of simulated time take about 0.1 s of wall time at 10x
    assert 0.09 < clock.t < 0.25


def test_server_saturated_keeps_every_slot_busy():
    # every admitted stream gives a frame to every tick; ended streams hand
    # their slot to waiting ones in arrival order
    clock = FakeClock()
    be = FakeBackend(clock, cost=0.001)
    reqs = [req(i, 5.0 * i, 3 + i % 4) for i in range(12)]   # arrival times are ignored
    srv = Server(be, FakeBank(), reqs, budget_bytes=10_000, max_streams=4, clock=clock, sleep=clock.sleep,
                 saturate=True)
    st = srv.run(horizon=1.0)
    assert st.admitted == 12 and st.frames == sum(3 + i % 4 for i in range(12))
    assert st.max_active == 4
    assert all(len(t) == 4 for t in be.ticks[:2])            # full ticks while requests wait
    for i in range(12):
        assert sum(1 for t in be.ticks if i in t) == 3 + i % 4
    assert sorted(be.closed) == list(range(12))
    assert max(st.latencies_ms) <= 1.0 + 1e-9                  # one tick each


def test_server_saturated_stops_at_its_duration():
    clock = FakeClock()
    be = FakeBackend(clock, cost=0.01)
    reqs = [req(i, 0.0, 10_000) for i in range(3)]
    st = Server(be, FakeBank(), reqs, budget_bytes=10_000, clock=clock, sleep=clock.sleep,
                saturate=True).run(horizon=0.5)
    assert 0.5 <= st.wall_s < 0.52 and st.frames == 3 * st.ticks
