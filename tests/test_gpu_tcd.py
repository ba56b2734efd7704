"""GPU parity of the temporally coherent detector (the comparison system of
Sec. 4): every frame's tracks (quarter-pixel position, octave, score, SAD)
against the oracle's, exactly, over groups of frames, on the three
workloads, panning and odd-sized scenes, every early-termination and match
threshold setting, resets and every frame source."""
import numpy as np
import pytest

import oracle
from paper_1503_06959_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kpd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1503_06959_amd import kpd as k
    return k


def rows(tr, names=("x4", "y4", "octave", "score", "sad")):
    return [tuple(int(r[n]) for n in names) for r in tr]


def run_tcd(kpd, frames, det, gop=10, t_bm=1800, t_et=1000, mode="retain", resets=()):
    import torch
    F, H, W = frames.shape
    t, O, Nc, Nr = det
    g = kpd.Tcd(W, H, kpd.make_params(t, O, Nc, Nr), gop, t_bm, t_et)
    o = oracle.Tcd(W, H, t, O, Nc, Nr, gop, t_bm, t_et)
    dev = torch.from_numpy(frames).cuda() if mode != "host" else None
    tracked = 0
    for i in range(F):
        if i in resets:
            g.reset()
            o.reset()
        if mode == "host":
            g.push(frames[i])
        else:
            g.push(dev[i], retain=(mode == "retain"))
        o.push(frames[i])
        got, exp = rows(g.tracks()), rows(o.tracks())
        assert got == exp, f"frame {i}: {len(got)} vs {len(exp)} tracks"
        if i % gop:
            tracked += len(got)
    g.close()
    return tracked


def det_of(name):
    d = synth.DETECTORS[name]
    return (d.fast_t, d.n_octaves, d.grid_cols, d.grid_rows)


def test_c1_groups(kpd):
    frames = synth.make_video(synth.SCENES["c1_320x240"], 25)
    assert run_tcd(kpd, frames, det_of("c1_320x240")) > 0


def test_c2_device_frames(kpd):
    frames = synth.make_video(synth.SCENES["c2_640x480"], 22)
    assert run_tcd(kpd, frames, det_of("c2_640x480"), mode="device") > 0


def test_c3_first_group(kpd):
    frames = synth.make_video(synth.SCENES["c3_1920x1080"], 6)
    assert run_tcd(kpd, frames, det_of("c3_1920x1080"), gop=6) > 0


@pytest.mark.parametrize("t_bm,t_et", [(1800, 0), (100000, 100000), (600, 1000), (4000, 2500), (0, 0)])
def test_thresholds(kpd, t_bm, t_et):
    frames = synth.make_video(synth.SCENES["c1_320x240"], 8)
    run_tcd(kpd, frames, det_of("c1_320x240"), gop=8, t_bm=t_bm, t_et=t_et)


@pytest.mark.parametrize("W,H,det,pan", [
    (333, 251, (25, 4, 7, 5), True),     # global motion: long displacements
    (101, 77, (12, 3, 6, 4), False),      # most patches meet the border
    (64, 48, (10, 1, 2, 2), True),
    (40, 40, (10, 2, 1, 1), False),       # no usable patch at all
])
def test_shapes(kpd, W, H, det, pan):
    sc = synth.Scene(W, H, 9, 8, 3, max(4, min(W, H) // 3), 1.5, 2.0, pan, 880 + W)
    run_tcd(kpd, synth.make_video(sc), det, gop=5)


def test_reset_host_frames_and_gop_one(kpd):
    frames = synth.make_video(synth.SCENES["c1_320x240"], 12)
    run_tcd(kpd, frames, det_of("c1_320x240"), gop=4, mode="host", resets=(6,))
    run_tcd(kpd, frames[:3], det_of("c1_320x240"), gop=1)


def test_errors_and_device_result(kpd):
    import torch
    frames = synth.make_video(synth.SCENES["c1_320x240"], 2)
    g = kpd.Tcd(320, 240, kpd.make_params(*det_of("c1_320x240")))
    with pytest.raises(kpd.KpdError):
        g.tracks()                                 # nothing pushed yet
    with pytest.raises(ValueError):
        g.push(frames[0][:, ::2])                  # not unit column stride
    g.push(frames[0])
    g.push(frames[1])
    ptr, cnt = g.device_result()
    assert ptr and cnt
    assert len(g.tracks()) > 0
    g.close()
    with pytest.raises(kpd.KpdError):
        kpd.Tcd(320, 240, kpd.make_params(*det_of("c1_320x240")), gop=0)


@pytest.mark.parametrize("seed", range(6))
def test_random_configs(kpd, seed):
    # seeded random sizes, depths, groups and thresholds on panning scenes
    rng = np.random.default_rng(7300 + seed)
    W, H = int(rng.integers(48, 360)), int(rng.integers(48, 280))
    O = int(rng.integers(1, 5))
    det = (int(rng.integers(8, 35)), O, int(rng.integers(1, 8)), int(rng.integers(1, 6)))
    gop = int(rng.integers(1, 6))
    t_bm = int(rng.choice([0, 600, 1800, 5000, 70000]))
    t_et = int(rng.choice([0, 500, 1000, 3000]))
    sc = synth.Scene(W, H, 8, int(rng.integers(3, 12)), 4, max(5, min(W, H) // 3), 1.0, 2.0, True, 6000 + seed)
    run_tcd(kpd, synth.make_video(sc), det, gop=gop, t_bm=t_bm, t_et=t_et, mode="device" if seed % 2 else "retain")


def test_c2_whole_video_as_benchmarked(kpd):
    # the benchmark's configuration: the 300-frame 640x480 video, groups of
    # 10, T_BM = 1800, T_ET = 1000, frames read in place
    frames = synth.make_video(synth.SCENES["c2_640x480"])
    assert frames.shape[0] == 300
    assert run_tcd(kpd, frames, det_of("c2_640x480"), gop=10, t_bm=1800, t_et=1000, mode="retain") > 0
