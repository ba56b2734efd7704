"""GPU parity: the HIP path through the C ABI against the CPU oracle,
element by element (keypoints: x, y, octave, score; masks; per-cell SAD and
counts; pyramid levels), bit-exact since the whole path is integer work."""
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


def gpu_tuples(arr):
    return [(int(k["x"]), int(k["y"]), int(k["octave"]), int(k["score"])) for k in arr]


def orc_tuples(arr):
    return [(int(k["x"]), int(k["y"]), int(k["octave"]), int(k["score"])) for k in arr]


def run_pair(kpd, frames, det, mode="host", thresholds=None, check_sad=True, tile=0, lazy=False):
    """Push frames through a GPU stream and an oracle stream, compare every
    frame. thresholds: {frame_index: (t, TI, TH)} applied before that frame.
    lazy: the oracle in its CPU-masked mode (the same results, pinned against
    the definitional mode; scores only what the marked cells read)."""
    import torch
    F, H, W = frames.shape
    t, O, Nc, Nr, TI, TH = det
    params = kpd.make_params(t, O, Nc, Nr, TI, TH, tile)
    g = kpd.Stream(W, H, params)
    o = oracle.Stream(W, H, t, O, Nc, Nr, TI, TH)
    if lazy:
        o.set_lazy(True)
    dev = torch.from_numpy(frames).cuda() if mode != "host" else None
    forced = True
    cur = (t, TI, TH)
    totals = []
    for i in range(F):
        if thresholds and i in thresholds:
            nt, nti, nth = thresholds[i]
            forced = forced or nt != cur[0]
            cur = (nt, nti, nth)
            g.set_thresholds(nt, nti, nth)
            o.set_thresholds(nt, nti, nth)
        if mode == "host":
            g.push(frames[i])
        else:
            g.push(dev[i], retain=(mode == "retain"))
        o.push(frames[i])
        gk, gm = g.keypoints()
        ok, om, osad, ocnt = o.get()
        assert gpu_tuples(gk) == orc_tuples(ok), f"frame {i}"
        np.testing.assert_array_equal(gm, om, err_msg=f"mask frame {i}")
        gsad, gcnt = g.cell_stats()
        np.testing.assert_array_equal(gcnt, ocnt, err_msg=f"counts frame {i}")
        mask_from_data = not forced and cur[1] >= 0 and cur[2] != 0
        if check_sad and mask_from_data and cur[1] < 255:
            np.testing.assert_array_equal(gsad.astype(np.int64), osad, err_msg=f"sad frame {i}")
        forced = False
        totals.append(len(gk))
    g.close()
    return totals


def scene_frames(name, n):
    return synth.make_video(synth.SCENES[name], n)


def det_of(name, **kw):
    d = synth.DETECTORS[name]
    v = dict(t=d.fast_t, O=d.n_octaves, Nc=d.grid_cols, Nr=d.grid_rows, TI=d.id_thresh, TH=d.kb_thresh)
    v.update(kw)
    return (v["t"], v["O"], v["Nc"], v["Nr"], v["TI"], v["TH"])


# ------------------------------------------------------------ the workloads

def test_c1_320x240_all_30_frames(kpd):
    frames = scene_frames("c1_320x240", 30)
    totals = run_pair(kpd, frames, det_of("c1_320x240"))
    assert min(totals) > 0


def test_c2_640x480_all_300_frames(kpd):
    frames = scene_frames("c2_640x480", 300)
    run_pair(kpd, frames, det_of("c2_640x480"), mode="retain")


def test_c3_1920x1080_all_300_frames(kpd):
    # the whole streaming video, one push_frame per frame
    frames = scene_frames("c3_1920x1080", 300)
    totals = run_pair(kpd, frames, det_of("c3_1920x1080"), mode="device", lazy=True)
    assert len(totals) == 300 and min(totals) > 0


def test_c3_full_frame_mode(kpd):
    frames = scene_frames("c3_1920x1080", 4)
    run_pair(kpd, frames, det_of("c3_1920x1080", TI=-1))


def test_batch_resolution_720p(kpd):
    det, m, smin, smax, sig = synth.RES_PRESETS[(1280, 720)]
    sc = synth.Scene(1280, 720, 8, m, smin, smax, 0.75, sig, False, 4048)
    frames = synth.make_video(sc)
    run_pair(kpd, frames, (det.fast_t, det.n_octaves, det.grid_cols, det.grid_rows, 8, KB_OFF), mode="retain")


# ---------------------------------------------------------------- mask modes

@pytest.mark.parametrize("TI,TH", [(255, 2), (255, 1), (6, 3), (-1, KB_OFF), (0, KB_OFF), (8, 0)])
def test_mask_modes_c1(kpd, TI, TH):
    frames = scene_frames("c1_320x240", 12)
    run_pair(kpd, frames, det_of("c1_320x240", TI=TI, TH=TH))


def test_threshold_changes_mid_stream(kpd):
    frames = scene_frames("c1_320x240", 10)
    thr = {3: (25, 8, KB_OFF), 5: (25, 255, 2), 7: (40, 4, 3)}
    run_pair(kpd, frames, det_of("c1_320x240"), thresholds=thr)


def test_frame_input_modes_agree(kpd):
    frames = scene_frames("c1_320x240", 6)
    a = run_pair(kpd, frames, det_of("c1_320x240"), mode="host")
    b = run_pair(kpd, frames, det_of("c1_320x240"), mode="device")
    c = run_pair(kpd, frames, det_of("c1_320x240"), mode="retain")
    assert a == b == c


def test_padded_pitch_frames(kpd):
    import torch
    frames = scene_frames("c1_320x240", 4)
    padded = np.zeros((4, 240, 352), np.uint8)
    padded[:, :, :320] = frames
    g = kpd.Stream(320, 240, kpd.make_params(30, 3, 8, 6, 8))
    o = oracle.Stream(320, 240, 30, 3, 8, 6, 8)
    dev = torch.from_numpy(padded).cuda()
    for i in range(4):
        view = dev[i, :, :320]
        assert view.stride(0) == 352
        g.push(view if i % 2 else padded[i][:, :320], retain=bool(i % 2))
        o.push(frames[i])
        assert gpu_tuples(g.keypoints()[0]) == orc_tuples(o.get()[0])
    g.close()


@pytest.mark.parametrize("pitch", [333, 336, 340, 384, 400])
def test_copied_frames_every_pitch(kpd, pitch):
    # copied frames keep the caller's pitch when their rows fit the 384-byte
    # slot rows (one linear copy; odd pitches are read bytewise), else they
    # are re-pitched by a 2D copy
    import torch
    sc = synth.Scene(333, 251, 8, 8, 3, 60, 1.0, 2.0, False, 4242)
    frames = synth.make_video(sc)
    buf = np.zeros((len(frames), 251 * pitch), np.uint8)
    for i, f in enumerate(frames):
        buf[i].reshape(251, pitch)[:, :333] = f
    host = [buf[i].reshape(251, pitch)[:, :333] for i in range(len(frames))]
    dev = torch.from_numpy(buf).cuda()
    det = (25, 4, 7, 5, 4, KB_OFF)
    g = kpd.Stream(333, 251, kpd.make_params(*det))
    o = oracle.Stream(333, 251, *det)
    for i in range(len(frames)):
        if i % 2 == 0:
            assert host[i].strides[0] == pitch
            g.push(host[i])
        else:
            view = torch.as_strided(dev[i], (251, 333), (pitch, 1))
            g.push(view, retain=False)
        o.push(frames[i])
        gk, gm = g.keypoints()
        ok, om, _, _ = o.get()
        assert gpu_tuples(gk) == orc_tuples(ok), f"frame {i}"
        np.testing.assert_array_equal(gm, om, err_msg=f"mask frame {i}")
    g.close()


# ------------------------------------------------------------ special inputs

def test_constant_frames_give_no_keypoints(kpd):
    for v in (0, 128, 255):
        frames = np.full((3, 120, 160), v, np.uint8)
        totals = run_pair(kpd, frames, (1, 3, 4, 3, 8, KB_OFF))
        assert totals == [0, 0, 0]


def test_bright_square_four_corners(kpd):
    a, b, t = 40, 190, 30
    img = np.full((96, 128), a, np.uint8)
    img[16:48, 24:56] = b
    g = kpd.Stream(128, 96, kpd.make_params(t, 3, 2, 2, -1))
    g.push(img)
    got = gpu_tuples(g.keypoints()[0])
    v = 11 * (b - a - t)
    assert sorted(got) == sorted([(24, 16, 0, v), (55, 16, 0, v), (24, 47, 0, v), (55, 47, 0, v)])
    g.close()


def test_unchanged_frame_reproduces_previous_set(kpd):
    frames = scene_frames("c1_320x240", 3)
    seq = np.stack([frames[0], frames[1], frames[1], frames[1]])
    g = kpd.Stream(320, 240, kpd.make_params(30, 3, 8, 6, 0))
    prev = None
    for i, f in enumerate(seq):
        g.push(f)
        k, m = g.keypoints()
        if i >= 2:
            assert not m.any()
            assert gpu_tuples(k) == prev
        prev = gpu_tuples(k)
    g.close()


def test_dense_candidates_and_ties(kpd):
    # few grey levels and a low threshold: many candidates, many equal scores
    rng = np.random.default_rng(5)
    frames = rng.choice(np.array([0, 60, 120, 200, 255], np.uint8), size=(4, 150, 200))
    run_pair(kpd, frames, (10, 3, 5, 3, 20, KB_OFF))
    frames = rng.integers(0, 256, size=(3, 130, 170), dtype=np.uint8)
    run_pair(kpd, frames, (5, 4, 3, 2, -1, KB_OFF))


@pytest.mark.parametrize("W,H,det", [
    (333, 251, (25, 4, 7, 5, 4, KB_OFF)),   # uneven cells, odd sizes
    (7, 7, (10, 1, 1, 1, 8, KB_OFF)),        # smallest detectable frame
    (9, 13, (10, 2, 3, 2, 2, 3)),            # cells narrower than the ring
    (100, 37, (15, 3, 1, 1, 8, KB_OFF)),     # one cell
    (127, 255, (15, 7, 1, 2, 8, KB_OFF)),    # deep pyramid on odd sizes
])
def test_shapes(kpd, W, H, det):
    sc = synth.Scene(W, H, 5, 6, 3, max(4, min(W, H) // 3), 1.0, 2.0, False, 900 + W)
    frames = synth.make_video(sc)
    run_pair(kpd, frames, det)


def test_largest_cells_and_octaves(kpd):
    # 128 x 128 cells (the maximum) and 8 octaves on a 2048 x 1536 frame
    sc = synth.Scene(2048, 1536, 3, 120, 20, 300, 0.5, 3.0, False, 77)
    frames = synth.make_video(sc)
    run_pair(kpd, frames, (20, 8, 16, 12, 8, KB_OFF), mode="device")


# ------------------------------------------------------------ pyramid, stats

def test_pyramid_levels_match_oracle(kpd):
    for name in ("c1_320x240", "c3_1920x1080"):
        sc = synth.SCENES[name]
        d = synth.DETECTORS[name]
        f = synth.make_video(sc, 1)[0]
        g = kpd.Stream(sc.width, sc.height, kpd.make_params(d.fast_t, d.n_octaves, d.grid_cols, d.grid_rows))
        g.push(f)
        ref = oracle.pyramid(f, d.n_octaves)
        for o in range(1, d.n_octaves):
            np.testing.assert_array_equal(g.level(o), ref[o], err_msg=f"{name} level {o}")
        g.close()
    # odd sizes and a deep pyramid
    rng = np.random.default_rng(2)
    f = rng.integers(0, 256, size=(201, 333), dtype=np.uint8)
    g = kpd.Stream(333, 201, kpd.make_params(20, 7, 3, 2))
    g.push(f)
    ref = oracle.pyramid(f, 7)
    for o in range(1, 7):
        np.testing.assert_array_equal(g.level(o), ref[o])
    g.close()


@pytest.mark.parametrize("W,H", [(333, 201), (129, 127), (640, 480)])
def test_pyramid_every_tile_and_depth(kpd, W, H):
    # noise exercises the rounding; odd sizes the dropped last row and column
    rng = np.random.default_rng(W)
    frames = rng.integers(0, 256, size=(2, H, W), dtype=np.uint8)
    for O in range(1, 9):
        if (1 << (O - 1)) > min(W, H):
            continue
        ref = oracle.pyramid(frames[1], O)
        for tile in (32, 64, 128):
            if tile < (1 << (O - 1)):
                continue
            g = kpd.Stream(W, H, kpd.make_params(20, O, max(3, W // 40), max(2, H // 40), 8, 0xFFFFFFFF, tile))
            for f in frames:
                g.push(f)
            for o in range(1, O):
                np.testing.assert_array_equal(g.level(o), ref[o], err_msg=f"O={O} tile={tile} level {o}")
            g.close()


@pytest.mark.parametrize("W,H,det,tile", [
    (333, 251, (25, 4, 7, 5, 4, 0xFFFFFFFF), 128),
    (640, 480, (20, 4, 16, 12, 8, 0xFFFFFFFF), 128),
    (1920, 1080, (20, 5, 32, 18, 8, 0xFFFFFFFF), 128),
    (321, 243, (15, 6, 5, 4, 6, 3), 128),
    (200, 150, (15, 1, 4, 3, 6, 0xFFFFFFFF), 128),
])
def test_wide_tiles_match_oracle(kpd, W, H, det, tile):
    sc = synth.Scene(W, H, 10, 8, 3, max(4, min(W, H) // 4), 1.0, 2.0, False, 880 + W)
    frames = synth.make_video(sc, 6)
    run_pair(kpd, frames, det, mode="retain", tile=tile)


# ----------------------------------------------------------------- ABI errors

def test_abi_errors_on_device(kpd):
    import ctypes
    g = kpd.Stream(320, 240, kpd.make_params(30, 3, 8, 6))
    cnt = ctypes.c_size_t()
    assert kpd.lib.get_keypoints(g.handle, None, 0, ctypes.byref(cnt), None) == kpd.KPD_ESTATE
    f = scene_frames("c1_320x240", 1)[0]
    g.push(f)
    out = np.zeros(2, kpd.KEYPOINT_DTYPE)
    rc = kpd.lib.get_keypoints(g.handle, out.ctypes.data, 2, ctypes.byref(cnt), None)
    assert rc == kpd.KPD_ETRUNC and cnt.value > 2
    assert kpd.lib.push_frame(g.handle, f.ctypes.data, 100, 0) == kpd.KPD_EINVAL   # pitch < W
    assert kpd.lib.push_frame(g.handle, f.ctypes.data, 320, 7) == kpd.KPD_EINVAL   # bad flags
    assert kpd.lib.set_thresholds(g.handle, 0, 8, 0) == kpd.KPD_EINVAL
    # nothing above changed the stream's result
    k, _ = g.keypoints()
    assert len(k) == cnt.value
    g.close()


def test_deterministic_and_independent_streams(kpd):
    frames = scene_frames("c2_640x480", 8)
    det = det_of("c2_640x480")
    p = kpd.make_params(*det)
    a, b = kpd.Stream(640, 480, p), kpd.Stream(640, 480, p)
    o = oracle.Stream(640, 480, *det)
    for i in range(8):
        a.push(frames[i])
        b.push(frames[i])
        o.push(frames[i])
        ka, ma = a.keypoints()
        kb, mb = b.keypoints()
        assert ka.tobytes() == kb.tobytes() and ma.tobytes() == mb.tobytes()
        assert gpu_tuples(ka) == orc_tuples(o.get()[0])
    a.close()
    b.close()


def test_reset_stream_acts_like_a_first_frame(kpd):
    frames = scene_frames("c1_320x240", 5)
    g = kpd.Stream(320, 240, kpd.make_params(30, 3, 8, 6, 8))
    for i in range(3):
        g.push(frames[i])
    g.reset()
    g.push(frames[3])
    k, m = g.keypoints()
    assert m.all()
    o = oracle.Stream(320, 240, 30, 3, 8, 6, 8)
    o.push(frames[3])
    assert gpu_tuples(k) == orc_tuples(o.get()[0])
    g.close()


def test_kernel_timing_counts_launches(kpd):
    frames = scene_frames("c1_320x240", 4)
    g = kpd.Stream(320, 240, kpd.make_params(30, 3, 8, 6, 8))
    kpd.profile(g.handle, True)
    for f in frames:
        g.push(f)
    ms, n = kpd.profile_read(g.handle)
    assert list(n) == [4, 4, 4, 0, 0]   # tile pass, cell pass, compaction; no mark pass
    assert (ms[:2] > 0).all()
    kpd.profile(g.handle, False)
    g.push(frames[0])
    ms, n = kpd.profile_read(g.handle)
    assert list(n) == [0, 0, 0, 0, 0]
    g.close()
