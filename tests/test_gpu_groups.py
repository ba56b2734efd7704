"""GPU parity of the group detector: when a chunk's parameters mark every cell
(full-frame detection, T_I < 0 or T_H = 0) one workgroup detects a rectangle
of cells. The group shape only changes how the work maps onto workgroups:
every shape must give each frame's D_n = F(I_n) of the oracle, bit for bit,
in the canonical (cell, octave, y, x) order."""
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


def full_frame_chunk(kpd, frames, det, groups, pad=0, threads=0):
    """Push all frames as one chunk with every cell marked; compare every
    frame, the mask and the counts with the oracle's full-frame stream."""
    import torch
    F, H, W = frames.shape
    t, O, Nc, Nr, TI, TH = det
    gx, gy = groups
    g = kpd.Stream(W, H, kpd.make_params(t, O, Nc, Nr, TI, TH, 0, F, group_cols=gx, group_rows=gy,
                                         group_threads=threads))
    buf = np.zeros((F, H, W + pad), np.uint8)
    buf[:, :, :W] = frames
    dev = torch.from_numpy(buf).cuda()
    g.push_chunk(dev[:, :, :W])
    o = oracle.Stream(W, H, t, O, Nc, Nr, TI, TH)
    for j in range(F):
        o.push(frames[j])
        ok, om, _, ocnt = o.get()
        assert tuples(g.chunk_keypoints(j)) == tuples(ok), f"groups {groups} frame {j}"
    gk, gm = g.keypoints()
    np.testing.assert_array_equal(gm, om)
    np.testing.assert_array_equal(g.cell_stats()[1], ocnt)
    g.close()


@pytest.mark.parametrize("groups", [(1, 1), (2, 1), (3, 1), (8, 1), (2, 3), (8, 2), (4, 4)])
def test_c1_every_group_shape(kpd, groups):
    frames = synth.make_video(synth.SCENES["c1_320x240"], 10)
    d = synth.DETECTORS["c1_320x240"]
    full_frame_chunk(kpd, frames, (d.fast_t, d.n_octaves, 8, 6, -1, KB_OFF), groups)


@pytest.mark.parametrize("groups", [(1, 1), (4, 1), (4, 2)])
def test_c2_group_shapes_and_keyframes(kpd, groups):
    # T_H = 0 marks every cell too
    frames = synth.make_video(synth.SCENES["c2_640x480"], 6)
    full_frame_chunk(kpd, frames, (20, 4, 16, 12, 8, 0), groups)


@pytest.mark.parametrize("W,H,det,groups", [
    (333, 251, (25, 4, 7, 5, -1, KB_OFF), (3, 2)),    # uneven cells, odd sizes
    (333, 251, (25, 4, 7, 5, -1, KB_OFF), (7, 1)),    # whole cell rows in one group
    (9, 13, (10, 2, 3, 2, -1, KB_OFF), (2, 2)),       # cells narrower than the ring
    (7, 7, (10, 1, 1, 1, -1, KB_OFF), (1, 1)),        # smallest detectable frame
    (127, 255, (15, 7, 1, 2, -1, KB_OFF), (1, 2)),    # deep pyramid on odd sizes
    (100, 37, (15, 3, 1, 1, -1, KB_OFF), (1, 1)),     # one cell
])
def test_shapes(kpd, W, H, det, groups):
    sc = synth.Scene(W, H, 5, 6, 3, max(4, min(W, H) // 3), 1.0, 2.0, False, 900 + W)
    frames = synth.make_video(sc)[:5]
    full_frame_chunk(kpd, frames, det, groups, pad=13)


@pytest.mark.parametrize("groups", [(1, 1), (2, 2), (9, 9)])
def test_dense_candidates_and_ties(kpd, groups):
    # few grey levels and a low threshold: many candidates, many equal scores
    # (9, 9 stands for the whole grid)
    rng = np.random.default_rng(5)
    frames = rng.choice(np.array([0, 60, 120, 200, 255], np.uint8), size=(3, 150, 200))
    full_frame_chunk(kpd, frames, (10, 3, 5, 3, -1, KB_OFF), (min(groups[0], 5), min(groups[1], 3)))
    frames = rng.integers(0, 256, size=(3, 130, 170), dtype=np.uint8)
    full_frame_chunk(kpd, frames, (5, 4, 3, 2, -1, KB_OFF), (min(groups[0], 3), min(groups[1], 2)))


def test_largest_cells_and_octaves(kpd):
    # 128 x 128 cells (the maximum) and 8 octaves on a 2048 x 1536 frame
    sc = synth.Scene(2048, 1536, 3, 120, 20, 300, 0.5, 3.0, False, 77)
    frames = synth.make_video(sc)[:2]
    full_frame_chunk(kpd, frames, (20, 8, 16, 12, -1, KB_OFF), (0, 0))


@pytest.mark.parametrize("groups", [(0, 0), (4, 1), (1, 1)])
def test_c3_1080p(kpd, groups):
    frames = synth.make_video(synth.SCENES["c3_1920x1080"], 4)
    full_frame_chunk(kpd, frames, (20, 5, 32, 18, -1, KB_OFF), groups)


@pytest.mark.parametrize("groups", [(1, 1), (2, 1), (4, 2)])
def test_512_threads(kpd, groups):
    frames = synth.make_video(synth.SCENES["c2_640x480"], 4)
    full_frame_chunk(kpd, frames, (20, 4, 16, 12, -1, KB_OFF), groups, threads=512)
    rng = np.random.default_rng(9)
    frames = rng.integers(0, 256, size=(2, 130, 170), dtype=np.uint8)
    full_frame_chunk(kpd, frames, (5, 4, 3, 2, -1, KB_OFF), (min(groups[0], 3), min(groups[1], 2)), threads=512)


def test_every_autotuner_choice_gives_identical_keypoints(kpd, tmp_path, monkeypatch):
    # every (cells per workgroup, threads) the tuner may pick gives the
    # oracle's D_n; the tuner's pick is one of them and is cached
    from paper_1503_06959_amd import autotune
    d = synth.DETECTORS["c2_640x480"]
    frames = synth.make_video(synth.SCENES["c2_640x480"], 3)
    cands = autotune.group_candidates(640, 480, d)
    assert (1, 1, 256) in cands and (4, 1, 512) in cands
    for gx, gy, nt in cands:
        full_frame_chunk(kpd, frames, (20, 4, 16, 12, -1, KB_OFF), (gx, gy), threads=nt)
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tune.json"))
    best, times = autotune.best_groups(640, 480, d)
    assert best in cands and set(times) == set(cands)
    assert autotune.best_groups(640, 480, d) == (best, {})   # from the cache
