"""GPU parity of batches of the masked stream over octaves and
intra-octaves (Sec. 2's layered scale space under Sec. 3's per-cell mask
and Eq. 1): kpd_lbatch_* advances many same-shape streams per tick, and
every slot's D and mask after every tick must equal its own oracle
layered stream, bit for bit, with slots skipping ticks, resets and T_H."""
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


def run_lbatch(kpd, W, H, det, n_slots, n_ticks, seed0, skip=lambda s, t: False, resets=()):
    """resets: (slot, tick) pairs reset before that tick. Returns the
    keypoints compared."""
    import torch
    t, O, Nc, Nr, TI, TH = det
    b = kpd.LayerBatch(W, H, kpd.make_params(t, O, Nc, Nr, TI, TH), n_slots)
    slots = []
    for s in range(n_slots):
        sc = synth.Scene(W, H, n_ticks, 6 + s % 5, 3, max(4, min(W, H) // 4), [0.2, 0.6, 1.0][s % 3], 2.0,
                         bool(s % 2), seed0 + s)
        frames = synth.make_video(sc, n_ticks)
        o = oracle.Stream(W, H, t, O, Nc, Nr, TI, TH)
        o.set_layers(True)
        slots.append(dict(o=o, frames=frames, dev=torch.from_numpy(frames).cuda(), next=0))
    torch.cuda.synchronize()
    compared = 0
    for tick in range(n_ticks):
        pushed = []
        for s, st in enumerate(slots):
            if skip(s, tick):
                continue
            if (s, tick) in resets:
                b.reset(s)
                st["o"].reset()
            i = st["next"]
            b.push(s, st["dev"][i])
            st["o"].push(st["frames"][i])
            st["next"] += 1
            pushed.append(s)
        b.tick()
        for s in pushed:
            gk, gm = b.keypoints(s)
            ok, om, _, _ = slots[s]["o"].get()
            assert tuples(gk) == tuples(ok), f"slot {s} tick {tick}"
            np.testing.assert_array_equal(gm, om, err_msg=f"mask slot {s} tick {tick}")
            compared += len(ok)
    b.close()
    return compared


def c1_det(**kw):
    d = synth.DETECTORS["c1_320x240"]
    v = dict(t=d.fast_t, O=d.n_octaves, Nc=d.grid_cols, Nr=d.grid_rows, TI=d.id_thresh, TH=d.kb_thresh)
    v.update(kw)
    return (v["t"], v["O"], v["Nc"], v["Nr"], v["TI"], v["TH"])


def test_c1_slots_skipping_ticks(kpd):
    assert run_lbatch(kpd, 320, 240, c1_det(), 6, 8, 6100, skip=lambda s, t: (s + t) % 3 == 0) > 0


@pytest.mark.parametrize("TI,TH", [(6, 3), (-1, KB_OFF), (255, 2), (0, 0)])
def test_c1_thresholds_and_resets(kpd, TI, TH):
    run_lbatch(kpd, 320, 240, c1_det(TI=TI, TH=TH), 4, 6, 6200, resets={(1, 3), (2, 2)})


@pytest.mark.parametrize("W,H,det", [(333, 251, (25, 4, 7, 5, 4, KB_OFF)), (97, 65, (10, 6, 5, 3, 6, KB_OFF)),
                                     (64, 48, (10, 1, 2, 2, 6, 2))])
def test_shapes(kpd, W, H, det):
    run_lbatch(kpd, W, H, det, 3, 6, 6300 + W, skip=lambda s, t: s == 2 and t == 1)


def test_c2_64_slots(kpd):
    d = synth.DETECTORS["c2_640x480"]
    det = (d.fast_t, d.n_octaves, d.grid_cols, d.grid_rows, d.id_thresh, d.kb_thresh)
    assert run_lbatch(kpd, 640, 480, det, 64, 6, 6400) > 0


def test_errors(kpd):
    import torch
    d = synth.DETECTORS["c1_320x240"]
    frames = torch.from_numpy(synth.make_video(synth.SCENES["c1_320x240"], 2)).cuda()
    b = kpd.LayerBatch(320, 240, kpd.make_params(d.fast_t, d.n_octaves, d.grid_cols, d.grid_rows), 2)
    with pytest.raises(kpd.KpdError):
        b.keypoints(0)                      # no tick yet
    b.push(0, frames[0])
    with pytest.raises(kpd.KpdError):
        b.push(0, frames[1])                # one frame per slot per tick
    with pytest.raises(kpd.KpdError):
        b.push(2, frames[1])                # no such slot
    b.tick()
    assert len(b.keypoints(0)[0]) > 0
    with pytest.raises(kpd.KpdError):
        b.keypoints(1)                      # slot 1 had no frame
    b.close()
