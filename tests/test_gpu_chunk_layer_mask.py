"""GPU parity of the per-pixel masks of Sec. 3.1 (Eq. 2 per pixel, Eq. 1 per
feature) in chunks: one mask on a pyramid layer for all octaves (mode 1)
and one mask per octave on its own level (mode 2), pushed as push_frames
chunks mixed with single-frame pushes. Every frame's D_n, and the last
frame's cell mask and counts, against the oracle's frame-by-frame run, bit
for bit, on every layer, odd shapes, mode switches and whole videos in one
chunk."""
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


def run_layer_chunks(kpd, frames, det, plan, K, modes):
    """plan: chunk lengths (0 = one push_frame call); modes: {step: (mode,
    layer)} set on both sides before that step (step 0 must set one).
    Returns the keypoints compared."""
    import torch
    F, H, W = frames.shape
    t, O, Nc, Nr, TI, TH = det
    g = kpd.Stream(W, H, kpd.make_params(t, O, Nc, Nr, TI, TH, 0, K, layer_mask=1))
    o = oracle.Stream(W, H, t, O, Nc, Nr, TI, TH)
    dev = torch.from_numpy(frames).cuda()
    i = 0
    compared = 0
    for step, n in enumerate(plan):
        if i >= F:
            break
        if step in modes:
            g.set_mask_mode(*modes[step])
            o.set_id_mode(*modes[step])
        if n == 0:
            g.push(dev[i], retain=True)
            o.push(frames[i])
            gk, gm = g.keypoints()
            ok, om, _, ocnt = o.get()
            assert tuples(gk) == tuples(ok), f"single frame {i}"
            np.testing.assert_array_equal(gm, om, err_msg=f"mask frame {i}")
            compared += len(ok)
            i += 1
            continue
        n = min(n, F - i)
        g.push_chunk(dev[i:i + n])
        for j in range(n):
            o.push(frames[i + j])
            ok, om, _, ocnt = o.get()
            assert tuples(g.chunk_keypoints(j)) == tuples(ok), f"chunk at {i} frame {i + j}"
            compared += len(ok)
        gk, gm = g.keypoints()
        assert tuples(gk) == tuples(ok), f"last frame of chunk at {i}"
        np.testing.assert_array_equal(gm, om, err_msg=f"mask after chunk at {i}")
        np.testing.assert_array_equal(g.cell_stats()[1], ocnt, err_msg=f"counts after chunk at {i}")
        i += n
    g.close()
    return compared


@pytest.mark.parametrize("layer", [0, 1, 2])
def test_c1_every_layer(kpd, layer):
    frames = synth.make_video(synth.SCENES["c1_320x240"], 24)
    run_layer_chunks(kpd, frames, det_of("c1_320x240"), [5, 0, 8, 1, 0, 8], K=8, modes={0: (1, layer)})


def test_c1_octave_masks(kpd):
    frames = synth.make_video(synth.SCENES["c1_320x240"], 24)
    run_layer_chunks(kpd, frames, det_of("c1_320x240"), [5, 0, 8, 1, 0, 8], K=8, modes={0: (2, 0)})


def test_c2_top_layer_whole_video_in_one_chunk(kpd):
    # the paper's choice (the top layer of four octaves) over all 300 frames
    frames = synth.make_video(synth.SCENES["c2_640x480"], 300)
    assert run_layer_chunks(kpd, frames, det_of("c2_640x480"), [300], K=300, modes={0: (1, 3)}) > 0


def test_c2_octave_masks_whole_video_in_one_chunk(kpd):
    frames = synth.make_video(synth.SCENES["c2_640x480"], 300)
    assert run_layer_chunks(kpd, frames, det_of("c2_640x480"), [300], K=300, modes={0: (2, 0)}) > 0


def test_c3_top_layer_chunks(kpd):
    frames = synth.make_video(synth.SCENES["c3_1920x1080"], 12)
    run_layer_chunks(kpd, frames, det_of("c3_1920x1080"), [6, 0, 5], K=6, modes={0: (1, 4)})


@pytest.mark.parametrize("W,H,det,layer", [
    (333, 251, (25, 4, 7, 5, 4, KB_OFF), 3),   # uncovered strips on the right and at the bottom
    (333, 251, (25, 4, 7, 5, 6, KB_OFF), 0),
    (127, 255, (15, 7, 1, 2, 8, KB_OFF), 6),   # a one-column top layer
    (9, 13, (10, 2, 3, 2, 2, KB_OFF), 1),      # cells narrower than the ring
    (64, 48, (12, 1, 2, 2, 6, KB_OFF), 0),     # one octave
])
@pytest.mark.parametrize("mode", [1, 2])
def test_layer_shapes(kpd, W, H, det, layer, mode):
    sc = synth.Scene(W, H, 6, 6, 3, max(4, min(W, H) // 3), 1.0, 2.0, False, 990 + W)
    run_layer_chunks(kpd, synth.make_video(sc, 20), det, [6, 0, 7, 7], K=7,
                     modes={0: (mode, layer if mode == 1 else 0)})


def test_mode_switches_between_chunks(kpd):
    # per-pixel, per-cell and per-pixel again: each switch re-detects every cell once
    frames = synth.make_video(synth.SCENES["c1_320x240"], 40)
    run_layer_chunks(kpd, frames, det_of("c1_320x240"), [4, 0, 6, 6, 0, 6, 6, 6], K=6,
                     modes={0: (1, 2), 2: (2, 0), 4: (0, 0), 6: (1, 1)})


def test_every_cell_marked(kpd):
    # T_I < 0 or T_H = 0 mark every pixel: every frame is F_n
    frames = synth.make_video(synth.SCENES["c1_320x240"], 10)
    run_layer_chunks(kpd, frames, det_of("c1_320x240", TI=-1), [4, 0, 5], K=5, modes={0: (1, 2)})
    run_layer_chunks(kpd, frames, det_of("c1_320x240", TH=0), [4, 0, 5], K=5, modes={0: (2, 0)})


def test_chunk_longer_than_64_frames(kpd):
    frames = synth.make_video(synth.SCENES["c1_320x240"], 150)
    run_layer_chunks(kpd, frames, det_of("c1_320x240"), [140, 10], K=140, modes={0: (1, 2)})
