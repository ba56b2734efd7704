"""GPU parity of the per-pixel intensity-difference masks of Sec. 3.1 with
Eq. 1 per feature position: one mask on a pyramid layer for all octaves
(mode 1) and one mask per octave on its own level (mode 2). Every frame's
D_n and cell mask against the oracle's, bit for bit, on every layer, with
T_H, odd sizes, mode switches and frame modes."""
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


def run_layer(kpd, frames, det, plan, mode="retain"):
    """plan: {frame index: (mode, layer)} applied before that frame (on both
    sides); frame 0 must set a mode."""
    import torch
    F, H, W = frames.shape
    t, O, Nc, Nr, TI, TH = det
    g = kpd.Stream(W, H, kpd.make_params(t, O, Nc, Nr, TI, TH, layer_mask=1))
    o = oracle.Stream(W, H, t, O, Nc, Nr, TI, TH)
    dev = torch.from_numpy(frames).cuda() if mode != "host" else None
    for i in range(F):
        if i in plan:
            g.set_mask_mode(*plan[i])
            o.set_id_mode(*plan[i])
        if mode == "host":
            g.push(frames[i])
        else:
            g.push(dev[i], retain=(mode == "retain"))
        o.push(frames[i])
        gk, gm = g.keypoints()
        ok, om, _, ocnt = o.get()
        assert tuples(gk) == tuples(ok), f"frame {i}"
        np.testing.assert_array_equal(gm, om, err_msg=f"mask frame {i}")
        np.testing.assert_array_equal(g.cell_stats()[1], ocnt, err_msg=f"counts frame {i}")
    g.close()


def det_of(name, **kw):
    d = synth.DETECTORS[name]
    v = dict(t=d.fast_t, O=d.n_octaves, Nc=d.grid_cols, Nr=d.grid_rows, TI=d.id_thresh, TH=d.kb_thresh)
    v.update(kw)
    return (v["t"], v["O"], v["Nc"], v["Nr"], v["TI"], v["TH"])


@pytest.mark.parametrize("layer", [0, 1, 2])
def test_c1_every_layer(kpd, layer):
    frames = synth.make_video(synth.SCENES["c1_320x240"], 16)
    run_layer(kpd, frames, det_of("c1_320x240"), {0: (1, layer)})


def test_c2_top_layer_60_frames(kpd):
    # the paper's choice: the top layer of four octaves
    frames = synth.make_video(synth.SCENES["c2_640x480"], 60)
    run_layer(kpd, frames, det_of("c2_640x480"), {0: (1, 3)})


def test_c2_layers_with_keyframe_binning(kpd):
    frames = synth.make_video(synth.SCENES["c2_640x480"], 20)
    run_layer(kpd, frames, det_of("c2_640x480", TH=3), {0: (1, 2)})
    run_layer(kpd, frames, det_of("c2_640x480", TI=20, TH=2), {0: (1, 0)})


def test_c3_top_layer(kpd):
    frames = synth.make_video(synth.SCENES["c3_1920x1080"], 10)
    run_layer(kpd, frames, det_of("c3_1920x1080"), {0: (1, 4)}, mode="device")


@pytest.mark.parametrize("W,H,det,layer", [
    (333, 251, (25, 4, 7, 5, 4, KB_OFF), 3),   # uncovered strips on the right and at the bottom
    (333, 251, (25, 4, 7, 5, 6, KB_OFF), 0),
    (127, 255, (15, 7, 1, 2, 8, KB_OFF), 6),   # a one-column top layer
    (101, 77, (15, 4, 6, 4, 4, 3), 3),
    (9, 13, (10, 2, 3, 2, 2, 3), 1),           # cells narrower than the ring
])
def test_layer_shapes(kpd, W, H, det, layer):
    sc = synth.Scene(W, H, 6, 6, 3, max(4, min(W, H) // 3), 1.0, 2.0, False, 950 + W)
    run_layer(kpd, synth.make_video(sc), det, {0: (1, layer)})


def test_c1_octave_masks(kpd):
    frames = synth.make_video(synth.SCENES["c1_320x240"], 16)
    run_layer(kpd, frames, det_of("c1_320x240"), {0: (2, 0)})


def test_c2_octave_masks_60_frames(kpd):
    frames = synth.make_video(synth.SCENES["c2_640x480"], 60)
    run_layer(kpd, frames, det_of("c2_640x480"), {0: (2, 0)})
    run_layer(kpd, frames[:20], det_of("c2_640x480", TH=3), {0: (2, 0)})


def test_c3_octave_masks(kpd):
    frames = synth.make_video(synth.SCENES["c3_1920x1080"], 8)
    run_layer(kpd, frames, det_of("c3_1920x1080"), {0: (2, 0)}, mode="device")


@pytest.mark.parametrize("W,H,det", [
    (333, 251, (25, 4, 7, 5, 4, KB_OFF)),
    (127, 255, (15, 7, 1, 2, 8, KB_OFF)),
    (101, 77, (15, 4, 6, 4, 4, 3)),
    (9, 13, (10, 2, 3, 2, 2, 3)),
    (64, 48, (12, 1, 2, 2, 6, KB_OFF)),        # one octave: the same as one mask on level 0
])
def test_octave_mask_shapes(kpd, W, H, det):
    sc = synth.Scene(W, H, 6, 6, 3, max(4, min(W, H) // 3), 1.0, 2.0, False, 970 + W)
    run_layer(kpd, synth.make_video(sc), det, {0: (2, 0)})


def test_mode_switches_and_frame_modes(kpd):
    frames = synth.make_video(synth.SCENES["c1_320x240"], 18)
    plan = {0: (1, 2), 4: (0, 0), 7: (1, 0), 10: (2, 0), 13: (1, 1), 15: (2, 0)}
    for mode in ("retain", "host", "device"):
        run_layer(kpd, frames, det_of("c1_320x240"), plan, mode=mode)


def test_layer_readback_and_errors(kpd):
    import torch
    sc, d = synth.SCENES["c1_320x240"], synth.DETECTORS["c1_320x240"]
    frames = synth.make_video(sc, 4)
    plain = kpd.Stream(320, 240, kpd.make_params(d.fast_t, d.n_octaves, d.grid_cols, d.grid_rows))
    with pytest.raises(kpd.KpdError):
        plain.set_mask_mode(1, 0)                       # opened without layer_mask
    plain.close()
    g = kpd.Stream(320, 240, kpd.make_params(d.fast_t, d.n_octaves, d.grid_cols, d.grid_rows, 8, KB_OFF, 0, 4,
                                             layer_mask=1))
    with pytest.raises(kpd.KpdError):
        g.set_mask_mode(1, d.n_octaves)                 # no such layer
    with pytest.raises(kpd.KpdError):
        g.set_mask_mode(2, 1)                           # mode 2 takes no layer
    for mode, layer in ((1, 1), (2, 0)):
        g.set_mask_mode(mode, layer)
        for f in frames:
            g.push(f)
            ref = oracle.pyramid(f, d.n_octaves)
            for o in range(1, d.n_octaves):
                np.testing.assert_array_equal(g.level(o), ref[o])   # the masked octaves alternate buffers
    g.push_chunk(torch.from_numpy(frames).cuda())       # chunks take the per-pixel masks too
    ref = oracle.pyramid(frames[-1], d.n_octaves)
    for o in range(1, d.n_octaves):
        np.testing.assert_array_equal(g.level(o), ref[o])
    g.set_thresholds(d.fast_t, 8, 3)
    with pytest.raises(kpd.KpdError):
        g.push_chunk(torch.from_numpy(frames).cuda())   # T_H would chain a chunk's marks through its counts
    g.close()
