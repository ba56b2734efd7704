"""GPU parity of the feature descriptors (Sec. 3 feature model; Eq. 1
carries whole features): every frame's orientation sectors and 512-bit
descriptors of D_n against the oracle's, bit for bit, for features new in
the frame and for carried ones, on the three workloads, odd shapes, deep
pyramids, resets and threshold changes."""
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


def run_desc(kpd, frames, det, mode="retain", thresholds=None, resets=()):
    import torch
    F, H, W = frames.shape
    t, O, Nc, Nr, TI, TH = det
    g = kpd.Stream(W, H, kpd.make_params(t, O, Nc, Nr, TI, TH, features=kpd.FEAT_DESCRIPTOR))
    o = oracle.Stream(W, H, t, O, Nc, Nr, TI, TH)
    o.set_descriptors(True)
    dev = torch.from_numpy(frames).cuda() if mode != "host" else None
    described = 0
    for i in range(F):
        if i in resets:
            g.reset()
            o.reset()
        if thresholds and i in thresholds:
            g.set_thresholds(*thresholds[i])
            o.set_thresholds(*thresholds[i])
        if mode == "host":
            g.push(frames[i])
        else:
            g.push(dev[i], retain=(mode == "retain"))
        o.push(frames[i])
        gk, gm = g.keypoints()
        ok, om, _, _ = o.get()
        assert tuples(gk) == tuples(ok), f"frame {i}"
        gd = g.descriptors()
        ob, od = o.descriptors()
        assert len(gd) == len(ob)
        np.testing.assert_array_equal(gd["sector"].astype(np.int64), ob.astype(np.int64), err_msg=f"sectors frame {i}")
        np.testing.assert_array_equal(gd["bits"], od, err_msg=f"bits frame {i}")
        described += len(gd)
    g.close()
    return described


def det_of(name, **kw):
    d = synth.DETECTORS[name]
    v = dict(t=d.fast_t, O=d.n_octaves, Nc=d.grid_cols, Nr=d.grid_rows, TI=d.id_thresh, TH=d.kb_thresh)
    v.update(kw)
    return (v["t"], v["O"], v["Nc"], v["Nr"], v["TI"], v["TH"])


def test_c1_masked_and_full(kpd):
    frames = synth.make_video(synth.SCENES["c1_320x240"], 20)
    assert run_desc(kpd, frames, det_of("c1_320x240")) > 0
    assert run_desc(kpd, frames[:6], det_of("c1_320x240", TI=-1)) > 0


def test_c2_masked_60_frames(kpd):
    frames = synth.make_video(synth.SCENES["c2_640x480"], 60)
    run_desc(kpd, frames, det_of("c2_640x480"), mode="device")


def test_c3_first_frames(kpd):
    frames = synth.make_video(synth.SCENES["c3_1920x1080"], 4)
    run_desc(kpd, frames, det_of("c3_1920x1080"))


@pytest.mark.parametrize("W,H,det", [
    (333, 251, (25, 4, 7, 5, 4, KB_OFF)),     # features near the right and bottom edges
    (127, 255, (15, 7, 1, 2, 8, KB_OFF)),     # a deep pyramid: patterns wider than the coarse levels
    (101, 77, (12, 4, 6, 4, 4, 3)),
    (64, 48, (10, 1, 2, 2, 6, KB_OFF)),
])
def test_shapes(kpd, W, H, det):
    sc = synth.Scene(W, H, 6, 8, 3, max(4, min(W, H) // 3), 1.0, 2.0, False, 990 + W)
    run_desc(kpd, synth.make_video(sc), det)


def test_resets_thresholds_and_host_frames(kpd):
    frames = synth.make_video(synth.SCENES["c1_320x240"], 12)
    run_desc(kpd, frames, det_of("c1_320x240"), mode="host", thresholds={4: (25, 6, 3), 8: (25, 8, KB_OFF)},
             resets=(6,))


def test_descriptor_errors(kpd):
    import torch
    d = synth.DETECTORS["c1_320x240"]
    frames = synth.make_video(synth.SCENES["c1_320x240"], 3)
    g = kpd.Stream(320, 240, kpd.make_params(d.fast_t, d.n_octaves, d.grid_cols, d.grid_rows, features=kpd.FEAT_DESCRIPTOR,
                                             chunk_frames=4, layer_mask=1))
    with pytest.raises(kpd.KpdError):
        g.descriptors()                                # nothing pushed yet
    with pytest.raises(kpd.KpdError):
        g.set_mask_mode(3, 0)                          # no such mask mode
    with pytest.raises(kpd.KpdError):
        g.chunk_descriptors(0)                         # no chunk pushed yet
    g.push(frames[0])
    assert len(g.descriptors()) == len(g.keypoints()[0])
    kpd.profile(g.handle, True)
    g.push(frames[1])
    ms, n = kpd.profile_read(g.handle)
    assert list(n) == [1, 1, 1, 0, 1]
    g.push_chunk(torch.from_numpy(frames[1:3]).cuda())
    assert len(g.chunk_descriptors(0)) == len(g.chunk_keypoints(0))
    with pytest.raises(kpd.KpdError):
        g.chunk_descriptors(2)                         # the chunk had two frames
    with pytest.raises(kpd.KpdError):
        g.chunk_refined(0)                             # opened without refinement
    g.close()
    plain = kpd.Stream(320, 240, kpd.make_params(d.fast_t, d.n_octaves, d.grid_cols, d.grid_rows))
    plain.push(frames[0])
    with pytest.raises(kpd.KpdError):
        plain.descriptors()                            # opened without descriptors
    plain.close()
