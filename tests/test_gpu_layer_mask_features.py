"""GPU parity of descriptors and refined values (Sec. 3 feature model,
Sec. 2's interpolation) under the per-pixel masks of Sec. 3.1: with Eq. 1
per feature a marked cell holds both new features (computed) and carried
ones (whose records come from D_{n-1}). Every frame's features against the
oracle's, bit for bit, for single-frame pushes, batch ticks and chunks."""
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


def det_of(name, **kw):
    d = synth.DETECTORS[name]
    v = dict(t=d.fast_t, O=d.n_octaves, Nc=d.grid_cols, Nr=d.grid_rows, TI=d.id_thresh, TH=d.kb_thresh)
    v.update(kw)
    return (v["t"], v["O"], v["Nc"], v["Nr"], v["TI"], v["TH"])


def compare(kpd, g, o, where, desc=True, ref=True):
    gk, gm = g.keypoints()
    ok, om, _, _ = o.get()
    assert tuples(gk) == tuples(ok), where
    np.testing.assert_array_equal(gm, om, err_msg=f"mask {where}")
    if desc:
        gd = g.descriptors()
        ob, od = o.descriptors()
        np.testing.assert_array_equal(gd["sector"].astype(np.int64), ob.astype(np.int64), err_msg=f"sectors {where}")
        np.testing.assert_array_equal(gd["bits"], od, err_msg=f"bits {where}")
    if ref:
        gr = g.refined()
        got = np.stack([gr["x"], gr["y"], gr["log2_scale"], gr["score"]], axis=1).astype(np.float32)
        np.testing.assert_array_equal(got.view(np.uint32), o.refined().view(np.uint32), err_msg=f"refined {where}")
    return len(ok)


def run_single(kpd, frames, det, plan, desc=True, ref=True):
    """plan: {frame: (mode, layer)} set on both sides before that frame."""
    import torch
    F, H, W = frames.shape
    t, O, Nc, Nr, TI, TH = det
    feats = (kpd.FEAT_DESCRIPTOR if desc else 0) | (kpd.FEAT_REFINE if ref else 0)
    g = kpd.Stream(W, H, kpd.make_params(t, O, Nc, Nr, TI, TH, layer_mask=1, features=feats))
    o = oracle.Stream(W, H, t, O, Nc, Nr, TI, TH)
    o.set_descriptors(desc)
    o.set_refine(ref)
    dev = torch.from_numpy(frames).cuda()
    n = 0
    for i in range(F):
        if i in plan:
            g.set_mask_mode(*plan[i])
            o.set_id_mode(*plan[i])
        g.push(dev[i], retain=True)
        o.push(frames[i])
        n += compare(kpd, g, o, f"frame {i}", desc, ref)
    g.close()
    return n


@pytest.mark.parametrize("mode,layer", [(1, 2), (1, 0), (2, 0)])
def test_c1_masks(kpd, mode, layer):
    frames = synth.make_video(synth.SCENES["c1_320x240"], 20)
    assert run_single(kpd, frames, det_of("c1_320x240"), {0: (mode, layer)}) > 0


def test_c2_top_layer_and_octave_masks_60_frames(kpd):
    frames = synth.make_video(synth.SCENES["c2_640x480"], 60)
    run_single(kpd, frames, det_of("c2_640x480"), {0: (1, 3)})
    run_single(kpd, frames, det_of("c2_640x480"), {0: (2, 0)}, ref=False)


def test_keyframe_binning_and_mode_switches(kpd):
    frames = synth.make_video(synth.SCENES["c1_320x240"], 24)
    run_single(kpd, frames, det_of("c1_320x240", TH=3), {0: (1, 1), 8: (0, 0), 12: (2, 0), 18: (1, 2)})


@pytest.mark.parametrize("W,H,det,mode,layer", [
    (333, 251, (25, 4, 7, 5, 4, KB_OFF), 1, 3),
    (127, 255, (15, 7, 2, 4, 8, KB_OFF), 2, 0),
    (101, 77, (15, 4, 6, 4, 4, 3), 1, 2),
])
def test_shapes(kpd, W, H, det, mode, layer):
    sc = synth.Scene(W, H, 6, 6, 3, max(4, min(W, H) // 3), 1.0, 2.0, False, 960 + W)
    run_single(kpd, synth.make_video(sc, 10), det, {0: (mode, layer)})


@pytest.mark.parametrize("single", [True, False])
def test_batch_ticks(kpd, single):
    import torch
    from paper_1503_06959_amd.batch import Batch
    feats = kpd.FEAT_DESCRIPTOR | kpd.FEAT_REFINE
    b = Batch(max_streams=8)
    b.set_single_launch(single)
    streams = []
    for s in range(6):
        name = ["c1_320x240", "c2_640x480"][s % 2]
        sc, d = synth.SCENES[name], synth.DETECTORS[name]
        frames = synth.make_video(sc, 8)
        mode = [(1, d.n_octaves - 1), (2, 0), (0, 0)][s % 3]
        f = feats if s != 4 else 0
        g = b.open_stream(sc.width, sc.height, kpd.make_params(d.fast_t, d.n_octaves, d.grid_cols, d.grid_rows,
                                                               d.id_thresh, d.kb_thresh, layer_mask=1, features=f))
        o = oracle.Stream(sc.width, sc.height, d.fast_t, d.n_octaves, d.grid_cols, d.grid_rows, d.id_thresh,
                          d.kb_thresh)
        o.set_descriptors(f != 0)
        o.set_refine(f != 0)
        g.set_mask_mode(*mode)
        o.set_id_mode(*mode)
        streams.append((g, o, frames, torch.from_numpy(frames).cuda(), f != 0))
    torch.cuda.synchronize()
    for tick in range(8):
        for g, o, frames, dev, _ in streams:
            with torch.cuda.stream(b.torch_stream):
                b.push(g, dev[tick], retain=True)
            o.push(frames[tick])
        b.tick()
        for si, (g, o, _, _, f) in enumerate(streams):
            compare(kpd, g, o, f"stream {si} tick {tick}", desc=f, ref=f)
    b.close()


def test_cells_too_large_for_the_lds(kpd):
    # one 127 x 128 cell's per-pixel scratch and sources exceed a workgroup's LDS
    g = kpd.Stream(127, 255, kpd.make_params(15, 7, 1, 2, 8, KB_OFF, layer_mask=1, features=kpd.FEAT_DESCRIPTOR))
    with pytest.raises(kpd.KpdError):
        g.set_mask_mode(2, 0)
    g.close()


def run_chunks(kpd, frames, det, plan, K, modes, desc=True, ref=True):
    """Chunks (plan: lengths, 0 = one push_frame call) with modes {step:
    (mode, layer)}: every frame's keypoints, mask after each call and
    features against the oracle's."""
    import torch
    F, H, W = frames.shape
    t, O, Nc, Nr, TI, TH = det
    feats = (kpd.FEAT_DESCRIPTOR if desc else 0) | (kpd.FEAT_REFINE if ref else 0)
    g = kpd.Stream(W, H, kpd.make_params(t, O, Nc, Nr, TI, TH, 0, K, layer_mask=1, features=feats))
    o = oracle.Stream(W, H, t, O, Nc, Nr, TI, TH)
    o.set_descriptors(desc)
    o.set_refine(ref)
    dev = torch.from_numpy(frames).cuda()
    i = 0
    n = 0
    for step, m in enumerate(plan):
        if i >= F:
            break
        if step in modes:
            g.set_mask_mode(*modes[step])
            o.set_id_mode(*modes[step])
        if m == 0:
            g.push(dev[i], retain=True)
            o.push(frames[i])
            n += compare(kpd, g, o, f"single frame {i}", desc, ref)
            i += 1
            continue
        m = min(m, F - i)
        g.push_chunk(dev[i:i + m])
        for j in range(m):
            o.push(frames[i + j])
            ok, _, _, _ = o.get()
            where = f"chunk at {i} frame {i + j}"
            assert tuples(g.chunk_keypoints(j)) == tuples(ok), where
            if desc:
                gd = g.chunk_descriptors(j)
                ob, od = o.descriptors()
                np.testing.assert_array_equal(gd["sector"].astype(np.int64), ob.astype(np.int64),
                                              err_msg=f"sectors {where}")
                np.testing.assert_array_equal(gd["bits"], od, err_msg=f"bits {where}")
            if ref:
                gr = g.chunk_refined(j)
                got = np.stack([gr["x"], gr["y"], gr["log2_scale"], gr["score"]], axis=1).astype(np.float32)
                np.testing.assert_array_equal(got.view(np.uint32), o.refined().view(np.uint32),
                                              err_msg=f"refined {where}")
            n += len(ok)
        n += compare(kpd, g, o, f"last frame of chunk at {i}", desc, ref)
        i += m
    g.close()
    return n


@pytest.mark.parametrize("mode,layer", [(1, 2), (1, 0), (2, 0)])
def test_c1_chunks(kpd, mode, layer):
    frames = synth.make_video(synth.SCENES["c1_320x240"], 24)
    assert run_chunks(kpd, frames, det_of("c1_320x240"), [5, 0, 8, 1, 0, 8], K=8, modes={0: (mode, layer)}) > 0


def test_c2_top_layer_whole_video_in_one_chunk(kpd):
    frames = synth.make_video(synth.SCENES["c2_640x480"], 300)
    assert run_chunks(kpd, frames, det_of("c2_640x480"), [300], K=300, modes={0: (1, 3)}) > 0


def test_chunks_mode_switches_and_parts(kpd):
    frames = synth.make_video(synth.SCENES["c1_320x240"], 40)
    run_chunks(kpd, frames, det_of("c1_320x240"), [4, 0, 6, 6, 0, 6, 6, 6], K=6,
               modes={0: (1, 2), 2: (2, 0), 4: (0, 0), 6: (1, 1)}, ref=False)
    run_chunks(kpd, frames[:20], det_of("c1_320x240"), [6, 7, 7], K=7, modes={0: (2, 0)}, desc=False)


@pytest.mark.parametrize("W,H,det,mode,layer", [
    (333, 251, (25, 4, 7, 5, 4, KB_OFF), 1, 3),
    (200, 120, (18, 6, 7, 5, 8, KB_OFF), 2, 0),
])
def test_chunk_shapes(kpd, W, H, det, mode, layer):
    sc = synth.Scene(W, H, 6, 6, 3, max(4, min(W, H) // 3), 1.0, 2.0, False, 980 + W)
    run_chunks(kpd, synth.make_video(sc, 14), det, [7, 0, 6], K=7, modes={0: (mode, layer)})
