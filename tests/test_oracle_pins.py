"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test ties one part of the oracle to something other than itself:
brute force written independently (tests/bruteforce.py), closed forms,
exhaustive enumeration, invariants and metamorphic relations. A plausible
mistake (wrong ring order, off-by-one arc length, a dropped -t term, a wrong
rounding in the pyramid, a transposed neighbourhood, an inverted mask
polarity) fails at least one of them.
"""
import itertools

import numpy as np
import pytest

import bruteforce as bf
import oracle

KB_OFF = 0xFFFFFFFF


def kps_tuples(arr):
    return [(int(k["x"]), int(k["y"]), int(k["octave"]), int(k["score"])) for k in arr]


# ---------------------------------------------------------------- segment test

def test_ring_is_the_radius3_bresenham_circle_in_circular_order():
    # Sec. 2: the AST samples the Bresenham circle of radius 3.
    assert oracle.ring() == bf.RING
    assert len(set(bf.RING)) == 16


def test_arc9_exhaustive_over_all_16bit_masks():
    # Sec. 2: n contiguous ring pixels; n = 9 of 16. All 65536 bright masks.
    for m in range(1 << 16):
        bits = [(m >> k) & 1 == 1 for k in range(16)]
        assert oracle.arc9(m) == bf.has_arc(bits, 9), hex(m)


def test_arc9_boundaries():
    assert oracle.arc9(0x01FF)          # exactly 9 from position 0
    assert not oracle.arc9(0x00FF)      # 8 is not enough
    assert oracle.arc9(0xF01F)          # 9 wrapping through position 15 -> 0
    assert not oracle.arc9(0xF00F)      # 8 wrapping
    assert not oracle.arc9(0x5555)


def _ring_image(p, ring_vals, size=9):
    img = np.full((size, size), p, np.uint8)
    c = size // 2
    for (dx, dy), v in zip(bf.RING, ring_vals):
        img[c + dy, c + dx] = v
    return img, c


@pytest.mark.parametrize("t", [1, 20, 55])
def test_score_hand_computed_cases(t):
    # 9 contiguous ring pixels exactly p+t+10, the rest equal to p: V = 9*10.
    p = 100
    vals = [p + t + 10] * 9 + [p] * 7
    img, c = _ring_image(p, vals)
    V = oracle.score_level(img, t)
    assert V[c, c] == 90
    # 8 contiguous bright only: not a corner.
    vals = [p + t + 10] * 8 + [p] * 8
    img, c = _ring_image(p, vals)
    assert oracle.score_level(img, t)[c, c] == 0
    # strictness: 9 pixels at exactly p+t are not brighter than p+t.
    vals = [p + t] * 9 + [p] * 7
    img, c = _ring_image(p, vals)
    assert oracle.score_level(img, t)[c, c] == 0
    # dark arc of 10, plus 2 isolated bright pixels: V = max(sum bright, sum dark)
    vals = [p - t - 7] * 10 + [p, p + t + 3, p, p + t + 5, p, p]
    img, c = _ring_image(p, vals)
    assert oracle.score_level(img, t)[c, c] == max(10 * 7, 3 + 5)


def test_score_extremes():
    # darkest possible: p=255, all ring 0, t=1 -> 16 * 254 = 4064 (fits u16).
    img, c = _ring_image(255, [0] * 16)
    assert oracle.score_level(img, 1)[c, c] == 4064
    img, c = _ring_image(0, [255] * 16)
    assert oracle.score_level(img, 1)[c, c] == 4064


def test_score_matches_bruteforce_random():
    rng = np.random.default_rng(7)
    for trial in range(6):
        img = rng.integers(0, 256, size=(20, 23), dtype=np.uint8)
        for t in (5, 30, 80):
            V = oracle.score_level(img, t)
            for y in range(20):
                for x in range(23):
                    assert V[y, x] == bf.score(img, x, y, t), (trial, t, x, y)


def test_candidate_scores_are_in_range():
    rng = np.random.default_rng(8)
    img = rng.integers(0, 256, size=(64, 64), dtype=np.uint8)
    for t in (1, 10, 40):
        V = oracle.score_level(img, t).astype(np.int64)
        nz = V[V > 0]
        assert nz.size > 0
        assert nz.min() >= 9 and nz.max() <= 4064
        # border rows/columns never score (3-pixel ring)
        assert not V[:3].any() and not V[-3:].any() and not V[:, :3].any() and not V[:, -3:].any()


# --------------------------------------------------------------------- pyramid

def test_pyramid_matches_numpy_blocks_and_odd_sizes():
    rng = np.random.default_rng(3)
    for (h, w) in [(37, 53), (64, 64), (135, 121), (8, 9)]:
        img = rng.integers(0, 256, size=(h, w), dtype=np.uint8)
        O = 4 if min(h, w) >= 16 else 3
        got = oracle.pyramid(img, O)
        ref = bf.pyramid(img, O)
        assert [g.shape for g in got] == [r.shape for r in ref]
        for g, r in zip(got, ref):
            np.testing.assert_array_equal(g, r)


def test_pyramid_block_constant_closed_form():
    # an image constant on aligned 2^(O-1) blocks keeps its block values exactly
    rng = np.random.default_rng(4)
    blocks = rng.integers(0, 256, size=(5, 7), dtype=np.uint8)
    O = 4
    img = np.kron(blocks, np.ones((8, 8), np.uint8))
    lv = oracle.pyramid(img, O)
    for o in range(O):
        s = 8 >> o
        np.testing.assert_array_equal(lv[o], np.kron(blocks, np.ones((s, s), np.uint8)))


def test_pyramid_round_half_up():
    img = np.array([[0, 1], [0, 1]], np.uint8)       # mean 0.5 -> 1
    assert oracle.pyramid(img, 2)[1][0, 0] == 1
    img = np.array([[0, 1], [0, 0]], np.uint8)       # mean 0.25 -> 0
    assert oracle.pyramid(img, 2)[1][0, 0] == 0
    img = np.array([[255, 255], [255, 254]], np.uint8)  # 254.75 -> 255
    assert oracle.pyramid(img, 2)[1][0, 0] == 255
    img = np.array([[1, 2], [2, 1]], np.uint8)       # 1.5 -> 2
    assert oracle.pyramid(img, 2)[1][0, 0] == 2


# --------------------------------------------------------- detection and NMS

def test_neighbourhood_relation_geometric_equals_index_form():
    # the geometric relation used by the brute force is the index-range form
    for o in range(1, 3):
        for x in range(0, 8):
            for xf in range(0, 20):
                geo = bf.are_neighbours((o, x, 5), (o - 1, xf, 2 * 5))
                idx = 2 * x - 1 <= xf <= 2 * x + 2
                assert geo == idx
                # symmetry
                assert bf.are_neighbours((o - 1, xf, 10), (o, x, 5)) == geo


@pytest.mark.parametrize("seed", range(8))
def test_detect_matches_bruteforce_random(seed):
    rng = np.random.default_rng(100 + seed)
    h, w = int(rng.integers(14, 34)), int(rng.integers(14, 34))
    # few grey levels -> many equal scores, exercising every tie-break
    img = rng.choice(np.array([0, 60, 120, 200, 255], np.uint8), size=(h, w))
    for O in (1, 2, 3):
        for t in (10, 50):
            assert kps_tuples(oracle.detect(img, t, O)) == bf.detect(img, t, O), (O, t)


def test_detect_matches_bruteforce_smooth_scene():
    from paper_1503_06959_amd import synth
    sc = synth.Scene(48, 40, 2, 4, 6, 14, 0.5, 2.0, False, 77)
    frames = synth.make_video(sc)
    for f in frames:
        for O in (1, 2, 3):
            assert kps_tuples(oracle.detect(f, 12, O)) == bf.detect(f, 12, O)


@pytest.mark.parametrize("t", [1, 20, 254])
@pytest.mark.parametrize("O", [1, 3, 5])
def test_constant_frame_has_no_keypoints(t, O):
    for v in (0, 77, 255):
        img = np.full((96, 128), v, np.uint8)
        assert len(oracle.detect(img, t, O)) == 0


@pytest.mark.parametrize("O,side,x0,y0", [
    (1, 8, 6, 9), (1, 9, 11, 5), (1, 12, 7, 7), (1, 20, 10, 10),
    (2, 12, 8, 8), (2, 16, 10, 12), (2, 24, 14, 6),
    (3, 24, 16, 8), (3, 32, 8, 16), (3, 40, 12, 20), (3, 48, 8, 8),
])
def test_bright_square_gives_exactly_its_four_corners(O, side, x0, y0):
    # Closed form: at a corner pixel of a noiseless square the ring holds 11
    # contiguous pixels of the other intensity, so V = 11 * (delta - t); edge
    # pixels next to it score 10 or 9 times, and coarser octaves tie and lose.
    a, b, t = 40, 190, 30
    img = np.full((y0 + side + 30, x0 + side + 30), a, np.uint8)
    img[y0:y0 + side, x0:x0 + side] = b
    got = kps_tuples(oracle.detect(img, t, O))
    x1, y1 = x0 + side - 1, y0 + side - 1
    v = 11 * (b - a - t)
    assert got == [(x0, y0, 0, v), (x1, y0, 0, v), (x0, y1, 0, v), (x1, y1, 0, v)]


def test_square_corner_neighbour_scores_closed_form():
    a, b, t = 40, 190, 30
    img = np.full((40, 40), a, np.uint8)
    img[10:30, 10:30] = b
    V = oracle.score_level(img, t)
    d = b - a - t
    assert V[10, 10] == 11 * d
    assert V[10, 11] == 10 * d and V[11, 10] == 10 * d   # one step along an edge
    assert V[10, 12] == 9 * d                             # two steps: 9-arc, still a corner
    assert V[10, 13] == 0                                 # straight edge: 7 darker pixels only
    assert V[9, 9] == 0                                   # outside the corner: 5 brighter pixels


@pytest.mark.parametrize("seed", range(3))
def test_nms_invariants_on_scene(seed):
    from paper_1503_06959_amd import synth
    sc = synth.Scene(160, 120, 1, 10, 10, 40, 0.5, 2.0, False, 300 + seed)
    img = synth.make_video(sc)[0]
    O, t = 3, 20
    F = kps_tuples(oracle.detect(img, t, O))
    assert len(F) > 0
    levels = oracle.pyramid(img, O)
    V = [oracle.score_level(lv, t) for lv in levels]
    kp = {(k[2], k[0], k[1]) for k in F}
    for k in F:
        assert V[k[2]][k[1], k[0]] == k[3] > 0
    # every candidate is either output or beaten by a neighbour (and outputs are not)
    for o in range(O):
        ys, xs = np.nonzero(V[o])
        for y, x in zip(ys, xs):
            p = (o, int(x), int(y))
            v = int(V[o][y, x])
            beaten = False
            for oq in (o - 1, o, o + 1):
                if oq < 0 or oq >= O:
                    continue
                s = 2.0 ** (oq - o)
                cx, cy = (x + 0.5) / s, (y + 0.5) / s
                for yq in range(int(cy) - 3, int(cy) + 4):
                    for xq in range(int(cx) - 3, int(cx) + 4):
                        if not (0 <= yq < V[oq].shape[0] and 0 <= xq < V[oq].shape[1]):
                            continue
                        q = (oq, xq, yq)
                        if bf.are_neighbours(p, q) and bf.precedes(
                                (int(V[oq][yq, xq]), oq, yq, xq), (v, o, int(y), int(x))):
                            beaten = True
            assert beaten == (p not in kp), p
    # no two keypoints are neighbours
    kl = sorted(kp)
    for i, p in enumerate(kl):
        for q in kl[i + 1:]:
            assert not bf.are_neighbours(p, q)


def test_translation_by_coarsest_pixel_translates_keypoints():
    # shifting the content by a multiple of 2^(O-1) keeps every pyramid level
    # aligned, so F translates exactly (content kept away from the borders)
    from paper_1503_06959_amd import synth
    O = 3
    sc = synth.Scene(64, 64, 1, 5, 8, 20, 0.0, 2.0, False, 55)
    content = synth.make_video(sc)[0]
    canvas = np.full((160, 160), 128, np.uint8)
    canvas[24:88, 32:96] = content
    F0 = kps_tuples(oracle.detect(canvas, 20, O))
    for sx, sy in [(4, 0), (0, 8), (12, 16), (-8, 4)]:
        shifted = np.full_like(canvas, 128)
        shifted[24 + sy:88 + sy, 32 + sx:96 + sx] = content
        F1 = kps_tuples(oracle.detect(shifted, 20, O))
        exp = sorted([(x + (sx >> o), y + (sy >> o), o, v) for (x, y, o, v) in F0],
                     key=lambda k: (k[2], k[1], k[0]))
        assert F1 == exp


# ------------------------------------------------------------ mask and Eq. (1)

def test_cells_of_keypoints():
    W, H, Nc, Nr = 320, 240, 8, 6
    for (x, y, o) in [(0, 0, 0), (39, 39, 0), (40, 0, 0), (19, 19, 1), (20, 20, 1), (9, 9, 2), (10, 10, 2),
                      (319, 239, 0), (79, 59, 2)]:
        assert oracle.cell_of(x, y, o, W, H, Nc, Nr) == bf.kp_cell((x, y, o), W, H, Nc, Nr)
    # uneven division: cell = floor(X * Nc / W)
    assert oracle.cell_of(99, 0, 0, 100, 10, 3, 1) == 2
    assert oracle.cell_of(33, 0, 0, 100, 10, 3, 1) == 0
    assert oracle.cell_of(34, 0, 0, 100, 10, 3, 1) == 1


def _scene(seed=21, frames=6, w=96, h=72, pan=False, move=0.5):
    from paper_1503_06959_amd import synth
    return synth.make_video(synth.Scene(w, h, frames, 6, 8, 24, move, 2.0, pan, seed))


@pytest.mark.parametrize("TI,TH", [(8, KB_OFF), (3, KB_OFF), (255, 2), (6, 3), (0, KB_OFF)])
def test_stream_matches_bruteforce(TI, TH):
    frames = _scene()
    W, H, t, O, Nc, Nr = 96, 72, 15, 3, 6, 4
    s = oracle.Stream(W, H, t, O, Nc, Nr, TI, TH)
    b = bf.Stream(W, H, t, O, Nc, Nr, TI, TH)
    for f in frames:
        s.push(f)
        exp = b.push(f)
        kps, mask, sad, cnt = s.get()
        assert kps_tuples(kps) == exp
        np.testing.assert_array_equal(mask, b.mask)
        assert cnt.sum() == len(exp)


def test_stream_sad_is_block_sum():
    frames = _scene(seed=5, frames=3)
    W, H, Nc, Nr = 96, 72, 5, 3   # uneven cells
    s = oracle.Stream(W, H, 20, 2, Nc, Nr, 4)
    s.push(frames[0])
    s.push(frames[1])
    _, _, sad, _ = s.get()
    cells = bf.cell_grid(W, H, Nc, Nr)
    d = np.abs(frames[1].astype(np.int64) - frames[0].astype(np.int64))
    exp = np.array([d[cells == c].sum() for c in range(Nc * Nr)])
    np.testing.assert_array_equal(sad, exp)


def test_first_frame_and_all_ones_mask_give_full_detection():
    frames = _scene(seed=9)
    W, H, t, O, Nc, Nr = 96, 72, 15, 3, 6, 4
    s = oracle.Stream(W, H, t, O, Nc, Nr, -1)
    for f in frames:
        s.push(f)
        kps, mask, _, _ = s.get()
        assert mask.all()
        F = kps_tuples(oracle.detect(f, t, O))
        key = lambda k: (bf.kp_cell(k, W, H, Nc, Nr), k[2], k[1], k[0])
        assert kps_tuples(kps) == sorted(F, key=key)


def test_unchanged_frame_reproduces_previous_set():
    frames = _scene(seed=10)
    W, H, t, O, Nc, Nr = 96, 72, 15, 3, 6, 4
    for TI, TH in [(0, KB_OFF), (8, KB_OFF), (255, 1), (2, 4)]:
        s = oracle.Stream(W, H, t, O, Nc, Nr, TI, TH)
        s.push(frames[0])
        s.push(frames[1])
        k1, _, _, _ = s.get()
        s.push(frames[1])
        k2, mask, sad, _ = s.get()
        assert not sad.any()
        assert kps_tuples(k2) == kps_tuples(k1)


def test_marked_cells_redetect_unmarked_cells_carry():
    frames = _scene(seed=11, frames=8, move=1.0)
    W, H, t, O, Nc, Nr = 96, 72, 15, 3, 6, 4
    s = oracle.Stream(W, H, t, O, Nc, Nr, 3)
    prev = None
    for f in frames:
        s.push(f)
        kps, mask, _, _ = s.get()
        cur = kps_tuples(kps)
        F = kps_tuples(oracle.detect(f, t, O))
        cell = lambda k: bf.kp_cell(k, W, H, Nc, Nr)
        for c in range(Nc * Nr):
            mine = [k for k in cur if cell(k) == c]
            if mask[c]:
                assert mine == [k for k in F if cell(k) == c]
            else:
                assert mine == [k for k in prev if cell(k) == c]
        prev = cur


def test_mask_polarity_marks_changed_cells():
    # Eq. (2) as printed marks unchanged pixels; the text asks for the
    # changed ones. A cell whose pixels all change by 20 must be marked at
    # T_I = 8 and a cell with no change must not.
    W, H = 64, 32
    f0 = np.full((H, W), 100, np.uint8)
    f1 = f0.copy()
    f1[:, :32] = 120
    s = oracle.Stream(W, H, 20, 1, 2, 1, 8)
    s.push(f0)
    s.push(f1)
    _, mask, sad, _ = s.get()
    assert list(mask) == [1, 0]
    assert sad[0] == 20 * 32 * 32 and sad[1] == 0
    # the threshold is strict: a mean difference equal to T_I does not mark
    s = oracle.Stream(W, H, 20, 1, 2, 1, 20)
    s.push(f0)
    s.push(f1)
    assert list(s.get()[1]) == [0, 0]


def test_keypoint_binning_threshold_is_inclusive():
    # Eq. (4): a bin is marked when its count is >= T_H.
    a, b, t = 40, 190, 30
    img = np.full((64, 64), a, np.uint8)
    img[8:24, 8:24] = b          # 4 corners, all in cell 0 of a 2x2 grid
    s = oracle.Stream(64, 64, t, 1, 2, 2, 255, 4)
    s.push(img)
    s.push(img)
    assert list(s.get()[1]) == [1, 0, 0, 0]
    s = oracle.Stream(64, 64, t, 1, 2, 2, 255, 5)
    s.push(img)
    s.push(img)
    assert list(s.get()[1]) == [0, 0, 0, 0]


def test_threshold_change_forces_full_redetection():
    frames = _scene(seed=12)
    W, H, O, Nc, Nr = 96, 72, 3, 6, 4
    s = oracle.Stream(W, H, 15, O, Nc, Nr, 255)
    s.push(frames[0])
    s.push(frames[1])
    assert not s.get()[1].any()
    s.set_thresholds(25, 255)
    s.push(frames[2])
    kps, mask, _, _ = s.get()
    assert mask.all()
    F = kps_tuples(oracle.detect(frames[2], 25, O))
    assert sorted(kps_tuples(kps)) == sorted(F)
    s.set_thresholds(25, 200)        # T_I change only: not forced
    s.push(frames[3])
    assert not s.get()[1].any()


def test_reset_forces_full_redetection_once():
    frames = _scene(seed=13)
    W, H, O, Nc, Nr = 96, 72, 3, 6, 4
    s = oracle.Stream(W, H, 15, O, Nc, Nr, 255)
    s.push(frames[0])
    s.push(frames[1])
    assert not s.get()[1].any()
    s.reset()
    s.push(frames[2])
    kps, mask, _, _ = s.get()
    assert mask.all()
    assert sorted(kps_tuples(kps)) == sorted(kps_tuples(oracle.detect(frames[2], 15, O)))
    s.push(frames[3])                # only the frame after the reset
    assert not s.get()[1].any()


# ------------------------------------- paper-literal mask on a pyramid layer

@pytest.mark.parametrize("layer,TI,TH,w,h,O", [
    (0, 8, KB_OFF, 96, 72, 3), (1, 6, KB_OFF, 96, 72, 3), (2, 4, KB_OFF, 96, 72, 3),
    (2, 5, 3, 98, 75, 3),
    # level-0 features in the strip that halving leaves uncovered (x >= 96)
    # take the layer's last column
    (3, 4, KB_OFF, 101, 77, 4),
    (1, 0, KB_OFF, 90, 70, 3), (2, 255, 2, 96, 72, 3),
])
def test_layer_mask_stream_matches_bruteforce(layer, TI, TH, w, h, O):
    frames = _scene(seed=30 + layer, frames=5, w=w, h=h, move=0.7)
    t, Nc, Nr = 15, 6, 4
    o = oracle.Stream(w, h, t, O, Nc, Nr, TI, TH)
    o.set_id_mode(1, layer)
    b = bf.Stream(w, h, t, O, Nc, Nr, TI, TH, id_mode=1, layer=layer)
    for i, f in enumerate(frames):
        o.push(f)
        exp = b.push(f)
        kps, mask, _, _ = o.get()
        assert kps_tuples(kps) == [(k[0], k[1], k[2], k[3]) for k in exp], f"frame {i}"
        np.testing.assert_array_equal(mask, b.mask, err_msg=f"mask frame {i}")


def test_layer_mask_unchanged_frame_and_all_marked():
    frames = _scene(seed=41)
    W, H, t, O, Nc, Nr = 96, 72, 15, 3, 6, 4
    s = oracle.Stream(W, H, t, O, Nc, Nr, 8)
    s.set_id_mode(1, 2)
    s.push(frames[0])
    first = kps_tuples(s.get()[0])
    s.push(frames[0])                 # nothing changed: D_n = D_{n-1}, nothing marked
    k, m, _, _ = s.get()
    assert kps_tuples(k) == first and not m.any()
    a = oracle.Stream(W, H, t, O, Nc, Nr, -1)
    a.set_id_mode(1, 1)
    for f in frames[:3]:
        a.push(f)
        k, m, _, _ = a.get()
        assert m.all()
        F = kps_tuples(oracle.detect(f, t, O))
        key = lambda q: (bf.kp_cell(q, W, H, Nc, Nr), q[2], q[1], q[0])
        assert kps_tuples(k) == sorted(F, key=key)


def test_layer_mask_is_per_feature_position():
    # one changed level-0 pixel: only features sitting on it are re-detected,
    # every other feature of the cell is carried
    rng = np.random.default_rng(7)
    W, H, t, O, Nc, Nr = 64, 48, 12, 1, 1, 1
    f0 = rng.choice(np.array([20, 200], np.uint8), size=(H, W))
    s = oracle.Stream(W, H, t, O, Nc, Nr, 10)
    s.set_id_mode(1, 0)
    s.push(f0)
    D0 = kps_tuples(s.get()[0])
    assert len(D0) > 10
    x, y = D0[len(D0) // 2][:2]
    f1 = f0.copy()
    f1[y, x] = 255 - f1[y, x]          # a dark/bright flip at one feature
    s.push(f1)
    D1 = kps_tuples(s.get()[0])
    F1 = {(k[0], k[1]): k for k in kps_tuples(oracle.detect(f1, t, O))}
    exp = [k for k in D0 if (k[0], k[1]) != (x, y)] + ([F1[(x, y)]] if (x, y) in F1 else [])
    assert D1 == sorted(exp, key=lambda k: (k[2], k[1], k[0]))


# ------------------------------------------ one mask per octave (option i)

@pytest.mark.parametrize("TI,TH,w,h,O", [
    (6, KB_OFF, 96, 72, 3), (4, KB_OFF, 101, 77, 4), (5, 3, 98, 75, 3), (0, KB_OFF, 90, 70, 2),
])
def test_octave_masks_stream_matches_bruteforce(TI, TH, w, h, O):
    frames = _scene(seed=60 + O, frames=5, w=w, h=h, move=0.7)
    t, Nc, Nr = 15, 6, 4
    o = oracle.Stream(w, h, t, O, Nc, Nr, TI, TH)
    o.set_id_mode(2, 0)
    b = bf.Stream(w, h, t, O, Nc, Nr, TI, TH, id_mode=2)
    for i, f in enumerate(frames):
        o.push(f)
        exp = b.push(f)
        kps, mask, _, _ = o.get()
        assert kps_tuples(kps) == [(k[0], k[1], k[2], k[3]) for k in exp], f"frame {i}"
        np.testing.assert_array_equal(mask, b.mask, err_msg=f"mask frame {i}")


def test_octave_masks_test_each_octave_on_its_own_level():
    # a level-0 change of 30 at one octave-0 feature moves its level-1 box
    # mean by at most 8 <= T_I: under one mask per octave only that octave-0
    # feature is re-detected and every octave-1 feature is carried; under one
    # mask built on layer 1 nothing is re-detected at all
    rng = np.random.default_rng(11)
    W, H, t, O, Nc, Nr, TI = 64, 48, 12, 2, 1, 1, 10
    f0 = rng.choice(np.array([20, 200], np.uint8), size=(H, W))
    s2 = oracle.Stream(W, H, t, O, Nc, Nr, TI)
    s2.set_id_mode(2, 0)
    s1 = oracle.Stream(W, H, t, O, Nc, Nr, TI)
    s1.set_id_mode(1, 1)
    s2.push(f0)
    s1.push(f0)
    D0 = kps_tuples(s2.get()[0])
    assert kps_tuples(s1.get()[0]) == D0
    assert any(k[2] == 1 for k in D0) and sum(k[2] == 0 for k in D0) > 10
    x, y = next(k for k in D0[len(D0) // 3:] if k[2] == 0)[:2]
    f1 = f0.copy()
    f1[y, x] = f0[y, x] + 30 if f0[y, x] == 20 else f0[y, x] - 30
    lv0, lv1 = oracle.pyramid(f0, 2)[1].astype(int), oracle.pyramid(f1, 2)[1].astype(int)
    assert np.abs(lv0 - lv1).max() <= TI          # level 1 sees no change
    s2.push(f1)
    s1.push(f1)
    F1 = {(k[0], k[1]): k for k in kps_tuples(oracle.detect(f1, t, O)) if k[2] == 0}
    exp = [k for k in D0 if not (k[2] == 0 and (k[0], k[1]) == (x, y))] + ([F1[(x, y)]] if (x, y) in F1 else [])
    assert kps_tuples(s2.get()[0]) == sorted(exp, key=lambda k: (k[2], k[1], k[0]))
    assert kps_tuples(s1.get()[0]) == D0
    assert s2.get()[1].all() and not s1.get()[1].any()


def test_octave_masks_unchanged_frame_and_mode_errors():
    frames = _scene(seed=43)
    W, H, t, O, Nc, Nr = 96, 72, 15, 3, 6, 4
    s = oracle.Stream(W, H, t, O, Nc, Nr, 8)
    s.set_id_mode(2, 0)
    s.push(frames[0])
    first = kps_tuples(s.get()[0])
    s.push(frames[0])
    k, m, _, _ = s.get()
    assert kps_tuples(k) == first and not m.any()
    with pytest.raises(AssertionError):
        s.set_id_mode(2, 1)                        # option i has no layer to choose
    with pytest.raises(AssertionError):
        s.set_id_mode(3, 0)


# ------------------------------------------------ descriptors (R13-R16)

def test_descriptor_matches_bruteforce():
    rng = np.random.default_rng(17)
    for h, w in ((40, 56), (25, 31), (9, 13)):
        img = rng.integers(0, 256, size=(h + 4, w + 4)).astype(np.float64)
        img = (img[:-4, :-4] + img[2:-2, 2:-2] + img[4:, 4:] + img[4:, :-4]) / 4   # some spatial structure
        level = np.clip(np.rint(img), 0, 255).astype(np.uint8)
        for x, y in ((w // 2, h // 2), (0, 0), (w - 1, h - 1), (3, h - 2), (w - 4, 5)):
            b, bits = oracle.describe(level, x, y)
            eb, ebits = bf.describe(level, x, y)
            assert b == eb, (h, w, x, y)
            np.testing.assert_array_equal(bits, ebits, err_msg=f"{h}x{w} at {x},{y}")


def test_descriptor_pattern_is_the_stated_rings():
    # 60 points: the centre, then rings of 10, 14, 15 and 20 points at radii
    # 3, 5, 7.5 and 11; the rounded offsets stay within half a pixel of the ring
    for b in (0, 5, 17):
        pat = oracle.desc_pattern(b)
        assert pat.shape == (60, 3)
        assert tuple(pat[0]) == (0, 0, 1)
        starts = [1, 11, 25, 40, 60]
        for R, h, s0, s1 in zip((3, 5, 7.5, 11), (1, 1, 2, 2), starts[:-1], starts[1:]):
            r = np.hypot(pat[s0:s1, 0], pat[s0:s1, 1])
            assert np.all(np.abs(r - R) <= np.sqrt(0.5) + 1e-9)
            assert np.all(pat[s0:s1, 2] == h)
        assert len({(int(a), int(c)) for a, c, _ in pat}) == 60


def test_descriptor_of_constant_patch():
    level = np.full((30, 30), 77, np.uint8)
    b, bits = oracle.describe(level, 15, 15)
    assert b == 0 and not bits.any()


@pytest.mark.parametrize("direction,sector", [((1, 0), 0), ((0, 1), 8), ((-1, 0), 16), ((0, -1), 24)])
def test_descriptor_orientation_follows_the_gradient(direction, sector):
    # a linear ramp: the pattern's intensity gradient points along it
    yy, xx = np.mgrid[0:64, 0:64]
    level = np.clip(128 + 3 * (direction[0] * (xx - 32) + direction[1] * (yy - 32)), 0, 255).astype(np.uint8)
    b, bits = oracle.describe(level, 32, 32)
    if direction[1] == 0:
        # the pattern is symmetric under y -> -y, so a ramp along x gives a
        # gradient exactly on the x axis: a sector boundary, which belongs
        # to the sector it starts
        assert b == sector
    else:
        assert (b - sector) % 32 in (0, 1, 31)
    # brighter points lie further along the ramp: bit k is set iff point a is further along than point b
    pat = oracle.desc_pattern(b)
    _, short_pairs = bf.desc_pairs()
    along = lambda i: direction[0] * pat[i, 0] + direction[1] * pat[i, 1]
    for k, (a, c) in enumerate(short_pairs):
        if along(a) != along(c):
            assert bool((int(bits[k >> 6]) >> (k & 63)) & 1) == (along(a) > along(c)), k


def test_stream_descriptors_follow_eq1():
    frames = _scene(seed=52, frames=4, w=96, h=72, move=0.8)
    W, H, t, O, Nc, Nr = 96, 72, 15, 3, 6, 4
    s = oracle.Stream(W, H, t, O, Nc, Nr, 6)
    s.set_descriptors(True)
    s.push(frames[0])
    k0 = kps_tuples(s.get()[0])
    b0, d0 = s.descriptors()
    pyr = oracle.pyramid(frames[0], O)
    for (x, y, o, _), b, d in zip(k0, b0, d0):   # frame 0 marks every cell: every feature is new
        eb, ed = oracle.describe(pyr[o], x, y)
        assert b == eb and np.array_equal(d, ed)
    s.push(frames[0])                               # unchanged: every feature and descriptor carried
    assert kps_tuples(s.get()[0]) == k0
    b1, d1 = s.descriptors()
    assert np.array_equal(b1, b0) and np.array_equal(d1, d0)
    s.push(frames[1])                               # marked cells: new descriptors; the rest carried
    k2, m2, _, _ = s.get()
    b2, d2 = s.descriptors()
    old = {k: (b, tuple(d)) for k, b, d in zip(k0, b0, d0)}
    pyr = oracle.pyramid(frames[1], O)
    for (x, y, o, v), b, d in zip(kps_tuples(k2), b2, d2):
        if m2[bf.kp_cell((x, y, o), W, H, Nc, Nr)]:
            eb, ed = oracle.describe(pyr[o], x, y)
            assert b == eb and np.array_equal(d, ed)
        else:
            assert old[(x, y, o, v)] == (b, tuple(d))
    assert m2.any() and not m2.all()


# ------------------------------------- sub-pixel and sub-scale refinement

def _smooth_random(seed, h, w):
    rng = np.random.default_rng(seed)
    img = rng.integers(0, 256, size=(h + 4, w + 4)).astype(np.float64)
    img = (img[:-4, :-4] + img[4:, 4:] + img[2:-2, 2:-2]) / 3
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


@pytest.mark.parametrize("seed,h,w,O,t,noise", [(3, 72, 96, 3, 15, False), (4, 77, 101, 4, 12, False),
                                                 (5, 40, 40, 1, 10, True), (6, 60, 80, 2, 12, False)])
def test_refine_matches_bruteforce(seed, h, w, O, t, noise):
    # the closed-form integer fit against a numpy least-squares fit, the
    # parabola along scale and the interpolation written out again
    img = _smooth_random(seed, h, w) if noise else _scene(seed=seed, frames=1, w=w, h=h)[0]
    lv = oracle.pyramid(img, O)
    kps = oracle.detect(img, t, O)
    assert len(kps) > 10
    octaves = set()
    sample = [k for k in kps if int(k["octave"]) > 0] + list(kps[::max(1, len(kps) // 40)])
    for k in sample:
        x, y, o = int(k["x"]), int(k["y"]), int(k["octave"])
        octaves.add(o)
        got = oracle.refine(lv, t, x, y, o)
        exp = bf.refine([np.asarray(l) for l in lv], t, x, y, o)
        np.testing.assert_allclose(got, exp, rtol=1e-6, atol=2e-4, err_msg=f"{x},{y},{o}")
        assert o - 1 <= got[2] <= o + 1
        # the refined position stays within the patches it was fit on
        assert abs(got[0] - (x + 0.5) * 2 ** o) <= 1.5 * 2 ** (o + 1)
        assert abs(got[1] - (y + 0.5) * 2 ** o) <= 1.5 * 2 ** (o + 1)
    assert len(octaves) >= min(O, 2)


def test_refine_of_a_square_corner_closed_form():
    # a single-octave bright square (contrast D, threshold t, k = D - t): a
    # corner scores 11k, its two edge neighbours 10k and the diagonal one 9k,
    # the outside 0 (the closed forms of the FAST score). The fit through
    # k [[0,0,0],[0,11,10],[0,10,9]] puts the maximum at (38/65, 38/65)
    # towards the square's inside with value k (86/9 + 2*19/6*38/65 +
    # (-23/3 + 9/4)(38/65)^2); with one layer the scale stays (t = 0)
    img = np.full((48, 48), 40, np.uint8)
    img[12:36, 12:36] = 200
    lv = oracle.pyramid(img, 1)
    k = 200 - 40 - 30
    u = 38 / 65
    m = k * (86 / 9 + 2 * 19 / 6 * u + (-23 / 3 + 9 / 4) * u * u)
    corners = {(int(q["x"]), int(q["y"])) for q in oracle.detect(img, 30, 1)}
    assert corners == {(12, 12), (35, 12), (12, 35), (35, 35)}
    for x, y in corners:
        r = oracle.refine(lv, 30, x, y, 0)
        sx = 1 if x == 12 else -1
        sy = 1 if y == 12 else -1
        np.testing.assert_allclose(r, [x + 0.5 + sx * u, y + 0.5 + sy * u, 0.0, m], rtol=1e-6)


def test_stream_refinement_follows_eq1():
    frames = _scene(seed=53, frames=3, w=96, h=72, move=0.8)
    W, H, t, O, Nc, Nr = 96, 72, 15, 3, 6, 4
    s = oracle.Stream(W, H, t, O, Nc, Nr, 6)
    s.set_refine(True)
    s.push(frames[0])
    k0 = kps_tuples(s.get()[0])
    r0 = s.refined()
    lv = oracle.pyramid(frames[0], O)
    for (x, y, o, _), r in zip(k0, r0):
        np.testing.assert_array_equal(r, oracle.refine(lv, t, x, y, o))
    s.push(frames[0])
    np.testing.assert_array_equal(s.refined(), r0)        # carried whole
    s.push(frames[1])
    k2, m2, _, _ = s.get()
    r2 = s.refined()
    old = {k: tuple(r) for k, r in zip(k0, r0)}
    lv = oracle.pyramid(frames[1], O)
    for (x, y, o, v), r in zip(kps_tuples(k2), r2):
        if m2[bf.kp_cell((x, y, o), W, H, Nc, Nr)]:
            np.testing.assert_array_equal(r, oracle.refine(lv, t, x, y, o))
        else:
            assert old[(x, y, o, v)] == tuple(r)


# ------------------------------------------------------ stored regression values

@pytest.mark.parametrize("name,det", [
    ("c1_320x240_first4.txt", (30, 3, 8, 6, 8, KB_OFF)),
    ("c1_320x240_kb2_first4.txt", (30, 3, 8, 6, 255, 2)),
])
def test_oracle_reproduces_stored_fixture(name, det):
    from golden_io import read_stream_fixture
    from paper_1503_06959_amd import synth
    exp = read_stream_fixture(name)
    sc = synth.SCENES["c1_320x240"]
    frames = synth.make_video(sc, len(exp))
    t, O, Nc, Nr, TI, TH = det
    s = oracle.Stream(sc.width, sc.height, t, O, Nc, Nr, TI, TH)
    for f, (mask_bits, kps) in zip(frames, exp):
        s.push(f)
        got, mask, _, _ = s.get()
        assert "".join(str(int(m)) for m in mask) == mask_bits
        assert kps_tuples(got) == kps


def test_oracle_reproduces_stored_layer_stream_fixture():
    from golden_io import read_stream_fixture
    from paper_1503_06959_amd import synth
    exp = read_stream_fixture("c1_320x240_layers_first4.txt")
    sc = synth.SCENES["c1_320x240"]
    frames = synth.make_video(sc, len(exp))
    s = oracle.Stream(sc.width, sc.height, 30, 3, 8, 6, 8, KB_OFF)
    s.set_layers(True)
    for f, (mask_bits, kps) in zip(frames, exp):
        s.push(f)
        got, mask, _, _ = s.get()
        assert "".join(str(int(m)) for m in mask) == mask_bits
        assert kps_tuples(got) == kps


def test_oracle_reproduces_stored_tcd_fixture():
    from golden_io import read_tcd_fixture
    from paper_1503_06959_amd import synth
    exp = read_tcd_fixture("c1_320x240_tcd_first7.txt")
    sc = synth.SCENES["c1_320x240"]
    frames = synth.make_video(sc, len(exp))
    s = oracle.Tcd(sc.width, sc.height, 30, 3, 8, 6, 3, 1800, 1000)
    for f, tr in zip(frames, exp):
        s.push(f)
        assert [tuple(int(v) for v in r) for r in s.tracks()] == tr


# ------------------------------------------- temporally coherent detector

def _texture(seed, h, w, passes=3, width=5):
    """Smooth random texture: box-blurred noise stretched to 10..245."""
    rng = np.random.default_rng(seed)
    img = rng.random((h, w))
    k = np.ones(width) / width
    for _ in range(passes):
        img = np.apply_along_axis(lambda r: np.convolve(r, k, mode="same"), 1, img)
        img = np.apply_along_axis(lambda c: np.convolve(c, k, mode="same"), 0, img)
    img = (img - img.min()) / (img.max() - img.min())
    return np.rint(10 + 235 * img).astype(np.uint8)


def test_tcd_spiral_order():
    # the walk of the oracle against a sort on (ring, clockwise perimeter
    # position); every ring of radius r holds 8r offsets
    order = bf.spiral_offsets(7)
    assert [oracle.tcd_spiral(k) for k in range(len(order))] == order
    assert len(set(order)) == 225
    for r in range(1, 8):
        start = (2 * r - 1) ** 2
        assert order[start] == (-r, -r)
        ring = order[start:(2 * r + 1) ** 2]
        assert len(ring) == 8 * r and all(max(abs(u), abs(v)) == r for u, v in ring)
        # consecutive offsets on a ring are 4-neighbours (a walk)
        assert all(abs(a[0] - b[0]) + abs(a[1] - b[1]) == 1 for a, b in zip(ring, ring[1:]))
        assert ring[1] == (-r + 1, -r)   # first step to the right along the top row (y down)


def test_tcd_sample_closed_forms():
    # bilinear sampling is exact on a linear ramp: the sample at quarter
    # position (X, Y) of I = 2x + 3y is round-half-up((2X + 3Y) / 4)
    H, W = 30, 40
    ys, xs = np.mgrid[0:H, 0:W]
    ramp = (2 * xs + 3 * ys).astype(np.uint8)
    for X in range(0, 4 * (W - 1) + 1, 3):
        for Y in range(0, 4 * (H - 1) + 1, 5):
            assert oracle.tcd_sample(ramp, X, Y) == (2 * X + 3 * Y + 2) >> 2, (X, Y)
    img = _texture(3, H, W)
    assert oracle.tcd_sample(img, 4 * 7, 4 * 9) == img[9, 7]            # whole pixels read the pixel
    assert oracle.tcd_sample(img, 4 * 7 + 2, 4 * 9) == (int(img[9, 7]) + int(img[9, 8]) + 1) >> 1
    assert oracle.tcd_sample(img, 4 * (W - 1), 0) == img[0, W - 1]      # last column, no right neighbour
    assert oracle.tcd_sample(img, 4 * (W - 1) + 1, 0) == -1
    assert oracle.tcd_sample(img, -1, 0) == -1


@pytest.mark.parametrize("dx,dy", [(0, 0), (2, -4), (3, 1), (-5, 7), (12, -12), (13, -1), (-1, 0)])
def test_tcd_integer_translation_is_found_exactly(dx, dy):
    # the content moves by (dx, dy) whole pixels (up to 13.75 is reachable:
    # 12 by the coarse step, 1.75 more by the fine one): every track whose
    # patches stay in the frame moves by exactly (4dx, 4dy) with SAD 0
    H, W = 120, 140
    big = _texture(11 + dx, H + 40, W + 40)
    prev = big[20:20 + H, 20:20 + W]
    cur = big[20 - dy:20 - dy + H, 20 - dx:20 - dx + W]
    pts = [(x, y) for x in range(36, W - 36, 9) for y in range(36, H - 36, 11)]
    tr = np.array([(4 * x, 4 * y, 0, 50, 0) for x, y in pts], oracle.TRACK_DTYPE)
    out = oracle.tcd_track(prev, cur, tr, t_bm=1, t_et=0)
    assert len(out) == len(tr)
    np.testing.assert_array_equal(out["x4"], tr["x4"] + 4 * dx)
    np.testing.assert_array_equal(out["y4"], tr["y4"] + 4 * dy)
    assert (out["sad"] == 0).all()
    np.testing.assert_array_equal(out["score"], tr["score"])


@pytest.mark.parametrize("t_bm,t_et,seed", [(1800, 1000, 1), (1800, 0, 2), (4000, 2500, 3), (600, 1000, 4),
                                            (100000, 100000, 5)])
def test_tcd_track_matches_bruteforce(t_bm, t_et, seed):
    # moving scenes on a small frame, so that many candidates and tracks
    # meet the border: every survivor, position, SAD and the order
    frames = _scene(seed=40 + seed, frames=3, w=72, h=56, move=1.5)
    kps = oracle.detect(frames[0], 12, 2)
    tr = np.array([(4 * (k["x"] << k["octave"]) + 2 * ((1 << k["octave"]) - 1),
                    4 * (k["y"] << k["octave"]) + 2 * ((1 << k["octave"]) - 1), k["octave"], k["score"], 0)
                   for k in kps], oracle.TRACK_DTYPE)
    assert len(tr) > 10
    for i in (1, 2):
        got = oracle.tcd_track(frames[i - 1], frames[i], tr, t_bm, t_et)
        exp = bf.track_step(frames[i - 1], frames[i], [tuple(int(v) for v in r) for r in tr], t_bm, t_et)
        assert [tuple(int(v) for v in r) for r in got] == exp
        tr = got


def test_tcd_stream_groups_and_drops():
    # T1: the first frame of every group is F(I_n) in the detector's order,
    # the others propagate the previous frame's tracks; a reset starts a new
    # group; an unrelated frame drops every track
    frames = _scene(seed=61, frames=7, w=96, h=72, move=0.8)
    W, H, t, O, Nc, Nr = 96, 72, 15, 3, 6, 4
    tc = oracle.Tcd(W, H, t, O, Nc, Nr, gop=3, t_bm=1800, t_et=1000)
    prev, prev_tr = None, None
    for i, f in enumerate(frames):
        if i == 5:
            tc.reset()
        n = tc.push(f)
        got = tc.tracks()
        assert n == len(got)
        if i in (0, 3, 5):   # groups of 3 from the first frame and from the reset
            det = oracle.Stream(W, H, t, O, Nc, Nr, -1)
            det.push(f)
            kps = det.get()[0]
            seeded = [(4 * (int(k["x"]) << int(k["octave"])) + 2 * ((1 << int(k["octave"])) - 1),
                       4 * (int(k["y"]) << int(k["octave"])) + 2 * ((1 << int(k["octave"])) - 1),
                       int(k["octave"]), int(k["score"]), 0) for k in kps]
            assert [tuple(int(v) for v in r) for r in got] == seeded, i
        else:
            exp = oracle.tcd_track(prev, f, prev_tr, 1800, 1000)
            np.testing.assert_array_equal(got, exp)
            assert len(got) > 0
        prev, prev_tr = f, got
    noise = np.random.default_rng(9).integers(0, 256, (H, W)).astype(np.uint8)
    tc.push(noise)   # the third frame of the group that the reset started
    assert len(tc.tracks()) == 0
    tc.close()


def test_tcd_thresholds_are_strict():
    # T_ET and T_BM compare with "below": a SAD equal to T_ET does not stop
    # the search, and a match whose SAD equals T_BM is dropped
    H, W = 100, 120
    big = _texture(77, H + 20, W + 20)
    prev = big[10:10 + H, 10:10 + W]
    cur = big[10 - 3:10 - 3 + H, 10 - 4:10 - 4 + W].astype(np.int64)
    cur = np.clip(cur + np.random.default_rng(5).integers(-3, 4, cur.shape), 0, 255).astype(np.uint8)
    for x, y in ((40, 40), (60, 52), (75, 45)):
        tr = np.array([(4 * x, 4 * y, 0, 30, 0)], oracle.TRACK_DTYPE)
        ref = bf._patch(prev, 4 * x, 4 * y)
        sad0 = int(np.abs(bf._patch(cur, 4 * x, 4 * y) - ref).sum())   # the first coarse candidate
        row = [tuple(int(v) for v in r) for r in tr]
        for t_et in (sad0, sad0 + 1):
            got = oracle.tcd_track(prev, cur, tr, 10 ** 6, t_et)
            assert [tuple(int(v) for v in r) for r in got] == bf.track_step(prev, cur, row, 10 ** 6, t_et)
        stopped = oracle.tcd_track(prev, cur, tr, 10 ** 6, sad0 + 1)[0]
        full = oracle.tcd_track(prev, cur, tr, 10 ** 6, sad0)[0]
        assert (stopped["x4"], stopped["y4"]) != (full["x4"], full["y4"])   # the threshold decided
        s = int(full["sad"])
        assert len(oracle.tcd_track(prev, cur, tr, s, sad0)) == 0
        assert len(oracle.tcd_track(prev, cur, tr, s + 1, sad0)) == 1


# ------------------------------------------------ intra-octave layers

def test_twothirds_closed_forms():
    rng = np.random.default_rng(31)
    img = rng.integers(0, 256, (61, 47)).astype(np.uint8)   # partial blocks dropped
    np.testing.assert_array_equal(oracle.twothirds(img), bf.twothirds(img))
    assert oracle.twothirds(img).shape == (40, 30)
    for v in (0, 1, 128, 255):   # a constant stays constant
        assert (oracle.twothirds(np.full((9, 12), v, np.uint8)) == v).all()
    # one bright pixel per block position: its weight over 9 at each output
    for j in range(3):
        for i in range(3):
            img = np.zeros((3, 3), np.uint8)
            img[j, i] = 90
            w = [[2, 1, 0], [0, 1, 2]]
            exp = [[(90 * w[q][j] * w[p][i] + 4) // 9 for p in range(2)] for q in range(2)]
            np.testing.assert_array_equal(oracle.twothirds(img), np.array(exp, np.uint8))
    # columns c, c + 3, c + 6 (constant down each column): the outputs are
    # the area means c + 1 and c + 5 exactly
    img = np.tile(np.array([30, 33, 36, 60, 63, 66], np.uint8), (3, 1))
    np.testing.assert_array_equal(oracle.twothirds(img), np.array([[31, 35, 61, 65]] * 2, np.uint8))


def test_layers_and_their_sizes():
    img = _smooth_random(5, 100, 131)
    L = oracle.layers(img, 4)
    ref = bf.layer_stack(img, 4)
    assert len(L) == 8
    for got, (exp, s) in zip(L, ref):
        np.testing.assert_array_equal(got, exp)
    dims = oracle.layer_dims(131, 100, 4)
    # pixel sizes (half level-0 pixels): 2^(i+1) for octaves, 3 * 2^i between
    assert [d[2] for d in dims] == [2, 3, 4, 6, 8, 12, 16, 24]
    assert [(d[0], d[1]) for d in dims] == [(a.shape[1], a.shape[0]) for a in L]


def test_layer_neighbourhood_between_octaves_is_r4():
    # the footprint rule reproduces R4 between octaves: 4x4 finer, 2x2 coarser
    for x in range(0, 40):
        assert oracle.layer_range(4, 2, x) == (2 * x - 1, 2 * x + 2)
        lo = min(X for X in range(-2, 40) if 2 * X - 1 <= x <= 2 * X + 2)
        hi = max(X for X in range(-2, 40) if 2 * X - 1 <= x <= 2 * X + 2)
        assert oracle.layer_range(2, 4, x) == (lo, hi)
        assert oracle.layer_range(2, 2, x) == (x - 1, x + 1)
        # octave <-> intra-octave: closed intervals [x s, (x+1) s] meet
        for S1, S2 in ((2, 3), (3, 2), (3, 4), (4, 3), (6, 8), (12, 8)):
            exp = [q for q in range(-3, 80) if max(x * S1, q * S2) <= min((x + 1) * S1, (q + 1) * S2)]
            assert oracle.layer_range(S1, S2, x) == (exp[0], exp[-1])


@pytest.mark.parametrize("seed", range(4))
def test_detect_layers_matches_bruteforce(seed):
    rng = np.random.default_rng(300 + seed)
    h, w = int(rng.integers(18, 40)), int(rng.integers(18, 40))
    img = rng.choice(np.array([0, 60, 120, 200, 255], np.uint8), size=(h, w))
    for O in (1, 2, 3):
        for t in (10, 50):
            assert kps_tuples(oracle.detect_layers(img, t, O)) == bf.detect_layers(img, t, O), (O, t)


def test_detect_layers_matches_bruteforce_scene():
    frames = _scene(seed=88, frames=1, w=64, h=52)
    for O in (2, 3):
        assert kps_tuples(oracle.detect_layers(frames[0], 12, O)) == bf.detect_layers(frames[0], 12, O)


def test_detect_layers_invariants():
    # on a scene at three octaves: keypoints on octave and intra-octave
    # layers alike; a candidate is kept exactly when no neighbour (by the
    # footprint rule) ranks above it, and no two keypoints are neighbours
    img = _scene(seed=91, frames=1, w=160, h=120)[0]
    t, O = 15, 3
    kps = kps_tuples(oracle.detect_layers(img, t, O))
    assert any(k[2] % 2 == 1 for k in kps) and any(k[2] % 2 == 0 for k in kps)
    L = oracle.layers(img, O)
    dims = oracle.layer_dims(160, 120, O)
    V = [oracle.score_level(l, t).astype(np.int64) for l in L]
    kept = {(k[2], k[0], k[1]) for k in kps}

    def nbrs(l, x, y):
        for m in (l - 1, l, l + 1):
            if m < 0 or m >= len(L):
                continue
            x0, x1 = oracle.layer_range(dims[l][2], dims[m][2], x)
            y0, y1 = oracle.layer_range(dims[l][2], dims[m][2], y)
            for qy in range(max(y0, 0), min(y1, dims[m][1] - 1) + 1):
                for qx in range(max(x0, 0), min(x1, dims[m][0] - 1) + 1):
                    if (m, qx, qy) != (l, x, y):
                        yield m, qx, qy

    def ranks_above(q, p):
        return (-V[q[0]][q[2], q[1]], q[0], q[2], q[1]) < (-V[p[0]][p[2], p[1]], p[0], p[2], p[1])

    for l in range(len(L)):
        ys, xs = np.nonzero(V[l])
        for y, x in zip(ys.tolist(), xs.tolist()):
            p = (l, x, y)
            above = [q for q in nbrs(l, x, y) if ranks_above(q, p)]
            assert (p in kept) == (len(above) == 0), p
            if p in kept:
                assert not any(q in kept for q in nbrs(l, x, y))


@pytest.mark.parametrize("seed,h,w,O,t,noise", [(1, 60, 80, 2, 10, True), (2, 90, 70, 3, 15, False),
                                                (3, 120, 160, 3, 12, False), (4, 64, 64, 4, 8, True)])
def test_refine_layers_matches_bruteforce(seed, h, w, O, t, noise):
    # the integer fits against numpy least squares and the Newton-form
    # parabola against numpy.polyfit, on octave and intra-octave keypoints
    img = _smooth_random(seed, h, w) if noise else _scene(seed=seed, frames=1, w=w, h=h)[0]
    kps = oracle.detect_layers(img, t, O)
    assert len(kps) > 5
    got = oracle.refine_layers(img, t, O, kps)
    stack = bf.layer_stack(img, O)
    for k, g in zip(kps, got):
        x, y, l = int(k["x"]), int(k["y"]), int(k["octave"])
        exp = bf.refine_layers(stack, t, x, y, l)
        np.testing.assert_allclose(g, exp, rtol=1e-6, atol=2e-4, err_msg=f"{x},{y},{l}")
        # the scale stays between the neighbouring layers' scales
        s_lo = (l - 1) // 2 + (np.log2(1.5) if (l - 1) % 2 else 0.0)
        s_hi = (l + 1) // 2 + (np.log2(1.5) if (l + 1) % 2 else 0.0)
        assert s_lo - 1e-6 <= g[2] <= s_hi + 1e-6
    assert any(int(k["octave"]) % 2 for k in kps) and any(int(k["octave"]) % 2 == 0 for k in kps)


@pytest.mark.parametrize("TI,TH", [(8, KB_OFF), (3, KB_OFF), (255, 2), (6, 3), (-1, KB_OFF)])
def test_layer_stream_matches_bruteforce(TI, TH):
    # L5: the mask and Eq. 1 over octaves and intra-octaves, cells from the
    # layers' footprints, against the brute-force stream
    frames = _scene(seed=23, frames=4, w=72, h=54, move=0.8)
    W, H, t, O, Nc, Nr = 72, 54, 15, 3, 5, 4
    s = oracle.Stream(W, H, t, O, Nc, Nr, TI, TH)
    s.set_layers(True)
    b = bf.LayerStream(W, H, t, O, Nc, Nr, TI, TH)
    for f in frames:
        s.push(f)
        exp = b.push(f)
        kps, mask, _, cnt = s.get()
        assert kps_tuples(kps) == exp
        np.testing.assert_array_equal(mask, b.mask)
        assert cnt.sum() == len(exp)
    assert any(k[2] % 2 for k in exp)


def test_layer_stream_carries_and_switches():
    frames = _scene(seed=29, frames=3, w=96, h=72, move=0.8)
    W, H, t, O, Nc, Nr = 96, 72, 15, 3, 6, 4
    s = oracle.Stream(W, H, t, O, Nc, Nr, 6)
    s.set_layers(True)
    s.push(frames[0])
    full = kps_tuples(s.get()[0])
    assert sorted(full, key=lambda k: (k[2], k[1], k[0])) == kps_tuples(oracle.detect_layers(frames[0], t, O))
    s.push(frames[0])                      # unchanged: nothing marked, D carried whole
    k1, m1, _, _ = s.get()
    assert kps_tuples(k1) == full and m1.sum() == 0
    s.set_layers(False)                    # switching marks every cell once
    s.push(frames[0])
    k2, m2, _, _ = s.get()
    assert m2.all()
    assert sorted(kps_tuples(k2), key=lambda k: (k[2], k[1], k[0])) == kps_tuples(oracle.detect(frames[0], t, O))
    s.set_descriptors(True)
    with pytest.raises(AssertionError):
        s.set_layers(True)                 # descriptors run over the octaves only


@pytest.mark.parametrize("TI,TH", [(8, KB_OFF), (3, KB_OFF), (255, 2), (6, 3), (-1, KB_OFF)])
def test_cpu_masked_mode_equals_definitional(TI, TH):
    # the CPU-masked mode scores only what marked cells' suppression reads;
    # D_n, the mask and the counts equal the definitional mode's on every frame
    from paper_1503_06959_amd import synth
    sc = synth.Scene(160, 120, 8, 10, 6, 30, 0.5, 2.0, True, 55)
    frames = synth.make_video(sc)
    W, H, t, O, Nc, Nr = 160, 120, 15, 3, 8, 6
    a = oracle.Stream(W, H, t, O, Nc, Nr, TI, TH)
    b = oracle.Stream(W, H, t, O, Nc, Nr, TI, TH)
    b.set_lazy(True)
    for f in frames:
        a.push(f)
        b.push(f)
        ka, ma, _, ca = a.get()
        kb, mb, _, cb = b.get()
        assert kps_tuples(ka) == kps_tuples(kb)
        np.testing.assert_array_equal(ma, mb)
        np.testing.assert_array_equal(ca, cb)
