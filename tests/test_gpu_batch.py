"""GPU parity of batched ticks: many streams of mixed resolutions and
parameters advance one frame per tick through two table-driven launches
(replayed from a captured HIP graph), and every stream's keypoints and mask
must equal its own oracle run, bit for bit."""
import numpy as np
import pytest

import oracle
from paper_1503_06959_amd import synth

pytestmark = pytest.mark.gpu

KB_OFF = 0xFFFFFFFF


@pytest.fixture(scope="module")
def kpd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1503_06959_amd import kpd as k
    return k


def tuples(arr):
    return [(int(k["x"]), int(k["y"]), int(k["octave"]), int(k["score"])) for k in arr]


def run_batch(kpd, specs, n_ticks, use_graph=True, skip=lambda s, t: False, mode="retain", single=True,
              lazy=False, feats=lambda s: 0, masks=lambda s: None):
    """specs: list of (Scene, (t, O, Nc, Nr, TI, TH, tile)). Every tick each
    stream not skipped pushes its next frame; after the tick every stream's
    D_n and mask are compared with its oracle. single: one launch per tick
    (else four); lazy: the oracle's CPU-masked mode (equal to its
    definitional mode, pinned on the CPU); feats(s): stream s's features
    (FEAT_* bits), compared with its oracle's after every tick; masks(s):
    stream s's per-pixel mask (mode, layer), None for the per-cell one."""
    import torch
    from paper_1503_06959_amd.batch import Batch
    b = Batch(max_streams=len(specs) + 2, use_graph=use_graph)
    b.set_single_launch(single)
    streams = []
    for si, (sc, det) in enumerate(specs):
        t, O, Nc, Nr, TI, TH, tile = det
        frames = synth.make_video(sc, n_ticks)
        g = b.open_stream(sc.width, sc.height, kpd.make_params(t, O, Nc, Nr, TI, TH, tile, features=feats(si),
                                                               layer_mask=int(masks(si) is not None)))
        o = oracle.Stream(sc.width, sc.height, t, O, Nc, Nr, TI, TH)
        if masks(si) is not None:
            g.set_mask_mode(*masks(si))
            o.set_id_mode(*masks(si))
        if lazy:
            o.set_lazy(True)
        o.set_descriptors(bool(feats(si) & kpd.FEAT_DESCRIPTOR))
        o.set_refine(bool(feats(si) & kpd.FEAT_REFINE))
        dev = torch.from_numpy(frames).cuda() if mode != "host" else None
        streams.append(dict(g=g, o=o, frames=frames, dev=dev, next=0))
    torch.cuda.synchronize()
    for tick in range(n_ticks):
        pushed = []
        for si, st in enumerate(streams):
            if skip(si, tick) or st["next"] >= n_ticks:
                continue
            i = st["next"]
            if mode == "host":
                b.push(st["g"], st["frames"][i])
            elif mode != "many":
                with torch.cuda.stream(b.torch_stream):
                    b.push(st["g"], st["dev"][i], retain=(mode == "retain"))
            st["o"].push(st["frames"][i])
            st["next"] += 1
            pushed.append(si)
        if mode == "many":
            # every stream's frame staged in one library call, reversed order
            # (each stream is looked up, not taken by position)
            with torch.cuda.stream(b.torch_stream):
                b.push_many([streams[si]["g"] for si in reversed(pushed)],
                            [streams[si]["dev"][streams[si]["next"] - 1] for si in reversed(pushed)], retain=True)
        b.tick()
        for si in pushed:
            st = streams[si]
            gk, gm = st["g"].keypoints()
            ok, om, _, _ = st["o"].get()
            assert tuples(gk) == tuples(ok), f"stream {si} tick {tick}"
            np.testing.assert_array_equal(gm, om, err_msg=f"mask stream {si} tick {tick}")
            if feats(si) & kpd.FEAT_DESCRIPTOR:
                gd = st["g"].descriptors()
                ob, od = st["o"].descriptors()
                np.testing.assert_array_equal(gd["sector"].astype(np.int64), ob.astype(np.int64),
                                              err_msg=f"sectors stream {si} tick {tick}")
                np.testing.assert_array_equal(gd["bits"], od, err_msg=f"bits stream {si} tick {tick}")
            if feats(si) & kpd.FEAT_REFINE:
                gr = st["g"].refined()
                got = np.stack([gr["x"], gr["y"], gr["log2_scale"], gr["score"]], axis=1).astype(np.float32)
                np.testing.assert_array_equal(got.view(np.uint32), st["o"].refined().view(np.uint32),
                                              err_msg=f"refined stream {si} tick {tick}")
    b.close()
    return streams


def mixed_specs(n=8, seed0=4000):
    specs = []
    for s in range(n):
        res = [(320, 240), (640, 480), (1280, 720)][s % 3]
        det, m, smin, smax, sig = synth.RES_PRESETS[res]
        sc = synth.Scene(res[0], res[1], 8, m, smin, smax, synth.MOTION_LEVELS[s % 3], sig, False, seed0 + s)
        TI, TH = [(8, KB_OFF), (4, 2), (-1, KB_OFF), (255, 1)][s % 4]
        specs.append((sc, (det.fast_t, det.n_octaves, det.grid_cols, det.grid_rows, TI, TH, 0)))
    return specs


@pytest.mark.parametrize("single", [True, False])
def test_mixed_streams_graph(kpd, single):
    run_batch(kpd, mixed_specs(8), 6, use_graph=True, single=single)


@pytest.mark.parametrize("single", [True, False])
def test_mixed_streams_eager_and_host_frames(kpd, single):
    run_batch(kpd, mixed_specs(5, 4100), 4, use_graph=False, mode="host", single=single)


@pytest.mark.parametrize("single", [True, False])
def test_streams_skipping_ticks(kpd, single):
    # streams with no frame in a tick are inactive; their state must not move
    run_batch(kpd, mixed_specs(6, 4200), 7, use_graph=True, skip=lambda s, t: (s + t) % 3 == 0, single=single)


def test_streams_staged_in_one_call(kpd):
    # batch_push_many: every tick's frames in one call, with streams skipping ticks
    run_batch(kpd, mixed_specs(6, 4300), 6, mode="many", single=False, skip=lambda s, t: (s + t) % 3 == 0)


@pytest.mark.parametrize("single", [True, False])
def test_streams_with_features(kpd, single):
    # descriptors, refined values, both or neither, by stream, with streams
    # skipping ticks (their features must stay those of their last frame)
    both = kpd.FEAT_DESCRIPTOR | kpd.FEAT_REFINE
    run_batch(kpd, mixed_specs(8, 4400), 6, single=single, skip=lambda s, t: (s + t) % 4 == 0,
              feats=lambda s: [both, 0, kpd.FEAT_DESCRIPTOR, kpd.FEAT_REFINE][s % 4])


@pytest.mark.parametrize("single", [True, False])
def test_streams_with_per_pixel_masks(kpd, single):
    # the top layer for every octave, one mask per octave, and per-cell
    # streams side by side, with streams skipping ticks
    specs = mixed_specs(9, 4500)

    def masks(s):
        O = specs[s][1][1]
        return [(1, O - 1), (2, 0), None][s % 3]
    run_batch(kpd, specs, 6, single=single, skip=lambda s, t: (s + t) % 4 == 0, masks=masks)


def test_tile_size_does_not_change_results(kpd):
    base = mixed_specs(3, 4300)
    specs = []
    for sc, det in base:
        for tile in (0, 64, 128):
            if tile and tile < (1 << (det[1] - 1)):
                continue
            specs.append((sc, det[:6] + (tile,)))
    run_batch(kpd, specs, 4)


@pytest.mark.parametrize("single", [True, False])
def test_batch_of_64_mixed_streams(kpd, single):
    specs = []
    for sc, det in synth.batch_streams(8):
        specs.append((sc, (det.fast_t, det.n_octaves, det.grid_cols, det.grid_rows, det.id_thresh,
                           det.kb_thresh, 0)))
    run_batch(kpd, specs, 8, single=single)


def test_c4_64_streams_full_length(kpd):
    # the batched workload at full length: 64 mixed streams, 120 generated
    # frames each, one tick per frame (the default four-launch form), every
    # stream's D_n and mask compared with its own oracle stream after every
    # tick
    specs = []
    for sc, det in synth.batch_streams(120):
        specs.append((sc, (det.fast_t, det.n_octaves, det.grid_cols, det.grid_rows, det.id_thresh,
                           det.kb_thresh, 0)))
    assert len(specs) == 64
    run_batch(kpd, specs, 120, lazy=True, single=False)


def test_attach_detach_between_ticks(kpd):
    import torch
    from paper_1503_06959_amd.batch import Batch
    b = Batch(max_streams=4)
    sc = synth.SCENES["c1_320x240"]
    frames = synth.make_video(sc, 6)
    p = kpd.make_params(30, 3, 8, 6, 8)
    g1 = b.open_stream(320, 240, p)
    o1 = oracle.Stream(320, 240, 30, 3, 8, 6, 8)
    g2 = b.open_stream(320, 240, p)
    o2 = oracle.Stream(320, 240, 30, 3, 8, 6, 8)
    for i in range(6):
        if i == 2:
            b.detach(g2)
        if i == 4:
            b.attach(g2)
        b.push(g1, frames[i])
        o1.push(frames[i])
        if i < 2 or i >= 4:
            b.push(g2, frames[i])
            o2.push(frames[i])
        b.tick()
        assert tuples(g1.keypoints()[0]) == tuples(o1.get()[0])
        if i < 2 or i >= 4:
            assert tuples(g2.keypoints()[0]) == tuples(o2.get()[0])
    b.close()


def test_batch_errors(kpd):
    import ctypes
    from paper_1503_06959_amd.batch import Batch
    b = Batch(max_streams=1)
    p = kpd.make_params(30, 3, 8, 6, 8)
    g = b.open_stream(320, 240, p)
    f = synth.make_video(synth.SCENES["c1_320x240"], 1)[0]
    b.push(g, f)
    # one frame per stream per tick
    assert kpd.lib.batch_push(b.handle, g.handle, f.ctypes.data, 320, 0) == kpd.KPD_ESTATE
    # capacity
    other = kpd.Stream(320, 240, p, stream=b.torch_stream)
    assert kpd.lib.batch_attach(b.handle, other.handle) == kpd.KPD_ENOMEM
    # a stream on another HIP stream
    b.tick()
    g.keypoints()
    other.close()
    b.close()


def test_closing_attached_streams_and_closed_handles(kpd):
    from paper_1503_06959_amd.batch import Batch
    b = Batch(max_streams=2)
    p = kpd.make_params(30, 3, 8, 6, 8)
    f = synth.make_video(synth.SCENES["c1_320x240"], 3)
    g = b.open_stream(320, 240, p)
    b.push(g, f[0])
    # a staged frame keeps the stream attached and open
    assert kpd.lib.close_stream(g.handle) == kpd.KPD_ESTATE
    b.tick()
    g.keypoints()
    h = g.handle
    assert kpd.lib.close_stream(h) == kpd.KPD_OK   # leaves the batch, then is released
    b.streams.pop(h, None)
    g.handle = None
    assert kpd.lib.close_stream(h) == kpd.KPD_ESTATE
    assert kpd.lib.push_frame(h, f[1].ctypes.data, 320, 0) == kpd.KPD_ESTATE
    # its place in the batch is free again
    g2 = b.open_stream(320, 240, p)
    g3 = b.open_stream(320, 240, p)
    o2 = oracle.Stream(320, 240, 30, 3, 8, 6, 8, KB_OFF)
    for i in range(2):
        b.push(g2, f[i])
        b.push(g3, f[i])
        o2.push(f[i])
        b.tick()
        assert tuples(g2.keypoints()[0]) == tuples(o2.get()[0])
    hb = b.handle
    b.close()
    assert kpd.lib.batch_tick(hb) == kpd.KPD_ESTATE
    # the batch's streams stay open, detached, and close normally
    g2.close()
    g3.close()
