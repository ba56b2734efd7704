"""GPU serving: streams arrive (Poisson), are admitted against a small HBM
budget, and share batched ticks as their frames arrive. Sampled streams are
re-run alone through push_frame on the same frames; every frame's keypoints
must be identical alone and in the mix."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1503_06959_amd import kpd, serve
    bank = serve.ClipBank(n_clips=2, clip_len=12, workers=8)
    return kpd, serve, bank


def run(env, backend_cls, budget, seed, record=(0, 1, 2, 3, 5, 8)):
    kpd, serve, bank = env
    reqs = serve.poisson_requests(20.0, 1.2, seed, frames=(8, 30), clip_len=12)
    be = backend_cls(max_streams=64)
    srv = serve.Server(be, bank, reqs, budget_bytes=budget, max_streams=64, speedup=4.0, record=record)
    st = srv.run(horizon=1.2)
    be.shutdown()
    return srv, st


def check_alone(env, srv):
    kpd, serve, bank = env
    checked = 0
    for sid, results in srv.recorded.items():
        if not results:
            continue
        req = srv.req_of[sid]
        g = kpd.Stream(req.res[0], req.res[1], serve.preset_params(kpd, req.res))
        for k, got in enumerate(results):
            g.push(bank.frame(req, k), retain=True)
            alone, _ = g.keypoints()
            assert alone.tobytes() == got.tobytes(), f"stream {sid} frame {k}"
        g.close()
        checked += 1
    return checked


def test_batched_serving_matches_streams_run_alone(env):
    kpd, serve, bank = env
    srv, st = run(env, serve.BatchedBackend, budget=48 << 20, seed=11)
    assert st.frames > 0 and st.ticks > 0
    assert st.deferred >= 1, "the budget should have made streams wait"
    assert check_alone(env, srv) >= 3
    s = st.summary()
    assert s["latency_ms"]["p99"] >= s["latency_ms"]["p50"] > 0


def test_plain_serving_matches_streams_run_alone(env):
    kpd, serve, bank = env
    srv, st = run(env, serve.PlainBackend, budget=1 << 30, seed=12, record=(0, 1, 2))
    assert st.frames > 0
    assert check_alone(env, srv) >= 2


def test_gather_matches_per_stream_results(env):
    import torch
    kpd, serve, bank = env
    from paper_1503_06959_amd.batch import Batch
    reqs = serve.poisson_requests(50.0, 1.0, 3, frames=(5, 5), clip_len=12)[:6]
    b = Batch(max_streams=8)
    ss = [b.open_stream(r.res[0], r.res[1], serve.preset_params(kpd, r.res)) for r in reqs]
    out = torch.empty(8 << 20, dtype=torch.uint8, device="cuda")
    counts = torch.empty(8, dtype=torch.int32, device="cuda")
    for k in range(3):
        for i, (r, s) in enumerate(zip(reqs, ss)):
            if (i + k) % 4:                       # some streams sit out some ticks
                with torch.cuda.stream(b.torch_stream):
                    b.push(s, bank.frame(r, k), retain=True)
        b.tick()
        kpd.batch_gather(b.handle, out, counts)
        b.synchronize()
        c = counts[:len(ss)].cpu().numpy()
        blob = out[:8 * int(c.sum())].cpu().numpy().view(kpd.KEYPOINT_DTYPE)
        off = 0
        for i, s in enumerate(ss):
            if (i + k) % 4:
                kp, _ = s.keypoints()
                assert blob[off:off + c[i]].tobytes() == kp.tobytes()
            else:
                assert c[i] == 0
            off += int(c[i])
    b.close()
