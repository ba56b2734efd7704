"""GPU parity of features in chunks (Sec. 3 feature model, Sec. 2's
interpolation; Eq. 1 carries whole features): for every frame of every
push_frames call, D_n's keypoints, orientation sectors, 512-bit descriptors
and refined values against the oracle's frame-by-frame run, bit for bit, in
masked, full-frame and count-marked (T_H) chunks, mixed with single-frame
pushes, resets and threshold changes."""
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


def check_features(kpd, gk, gd, gr, o, desc, ref, where):
    ok, _, _, _ = o.get()
    assert tuples(gk) == tuples(ok), where
    if desc:
        ob, od = o.descriptors()
        assert len(gd) == len(ob), where
        np.testing.assert_array_equal(gd["sector"].astype(np.int64), ob.astype(np.int64), err_msg=f"sectors {where}")
        np.testing.assert_array_equal(gd["bits"], od, err_msg=f"bits {where}")
    if ref:
        orf = o.refined()
        assert len(gr) == len(orf), where
        got = np.stack([gr["x"], gr["y"], gr["log2_scale"], gr["score"]], axis=1).astype(np.float32)
        bad = np.nonzero((got.view(np.uint32) != orf.view(np.uint32)).any(axis=1))[0]
        assert len(bad) == 0, f"{where}: {len(bad)} refined features differ, first gpu {got[bad[0]]} oracle {orf[bad[0]]}"
    return len(gk)


def run_chunk_features(kpd, frames, det, plan, K, desc=True, ref=True, resets=(), thresholds=None):
    """plan: chunk lengths (0 = one push_frame call); returns the features
    compared."""
    import torch
    F, H, W = frames.shape
    t, O, Nc, Nr, TI, TH = det
    feats = (kpd.FEAT_DESCRIPTOR if desc else 0) | (kpd.FEAT_REFINE if ref else 0)
    g = kpd.Stream(W, H, kpd.make_params(t, O, Nc, Nr, TI, TH, 0, K, features=feats))
    o = oracle.Stream(W, H, t, O, Nc, Nr, TI, TH)
    o.set_descriptors(desc)
    o.set_refine(ref)
    dev = torch.from_numpy(frames).cuda()
    i = 0
    compared = 0
    for step, n in enumerate(plan):
        if i >= F:
            break
        if step in resets:
            g.reset()
            o.reset()
        if thresholds and step in thresholds:
            g.set_thresholds(*thresholds[step])
            o.set_thresholds(*thresholds[step])
        if n == 0:
            g.push(dev[i], retain=True)
            o.push(frames[i])
            gk, _ = g.keypoints()
            compared += check_features(kpd, gk, g.descriptors() if desc else None, g.refined() if ref else None,
                                       o, desc, ref, f"single frame {i}")
            i += 1
            continue
        n = min(n, F - i)
        g.push_chunk(dev[i:i + n])
        for j in range(n):
            o.push(frames[i + j])
            compared += check_features(kpd, g.chunk_keypoints(j), g.chunk_descriptors(j) if desc else None,
                                       g.chunk_refined(j) if ref else None, o, desc, ref,
                                       f"chunk at {i} frame {i + j}")
        # the last frame's features are D_n's, which a following push carries
        gk, _ = g.keypoints()
        compared += check_features(kpd, gk, g.descriptors() if desc else None, g.refined() if ref else None,
                                   o, desc, ref, f"last frame of chunk at {i}")
        i += n
    g.close()
    return compared


def test_c1_masked_chunks_mixed_with_single_pushes(kpd):
    frames = synth.make_video(synth.SCENES["c1_320x240"], 30)
    assert run_chunk_features(kpd, frames, det_of("c1_320x240"), [5, 0, 8, 1, 0, 8, 8], K=8) > 0


def test_c1_full_frame_chunks(kpd):
    frames = synth.make_video(synth.SCENES["c1_320x240"], 12)
    assert run_chunk_features(kpd, frames, det_of("c1_320x240", TI=-1), [4, 0, 7], K=8) > 0


def test_c1_count_marked_chunks_resets_and_thresholds(kpd):
    frames = synth.make_video(synth.SCENES["c1_320x240"], 40)
    run_chunk_features(kpd, frames, det_of("c1_320x240", TH=3), [8, 8, 0, 8, 8, 8], K=8, resets=(3,),
                       thresholds={4: (24, 8, 3)})


def test_descriptors_only_and_refinement_only(kpd):
    frames = synth.make_video(synth.SCENES["c1_320x240"], 16)
    run_chunk_features(kpd, frames, det_of("c1_320x240"), [6, 10], K=10, ref=False)
    run_chunk_features(kpd, frames, det_of("c1_320x240"), [6, 10], K=10, desc=False)


@pytest.mark.parametrize("W,H,O", [(333, 251, 4), (200, 120, 6)])
def test_odd_shapes_and_deep_pyramids(kpd, W, H, O):
    sc = synth.Scene(W, H, 14, 12, 4, max(8, min(W, H) // 4), 0.75, 2.0, False, 500 + W + O)
    frames = synth.make_video(sc, 14)
    run_chunk_features(kpd, frames, (18, O, 7, 5, 8, KB_OFF), [7, 0, 6], K=7)


def test_chunk_longer_than_64_frames(kpd):
    # mark words of several 64-frame spans: carries across a word boundary
    frames = synth.make_video(synth.SCENES["c1_320x240"], 150)
    run_chunk_features(kpd, frames, det_of("c1_320x240"), [140, 10], K=140)


def test_c2_whole_video_in_one_chunk(kpd):
    frames = synth.make_video(synth.SCENES["c2_640x480"], 300)
    assert run_chunk_features(kpd, frames, det_of("c2_640x480"), [300], K=300) > 0
