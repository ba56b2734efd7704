"""GPU check of the entry point that allocates nothing:
kpd_detect_layers_static must give exactly what kpd_detect_layers gives with
a caller workspace, on two calls in a row (the second on a smaller frame, so
the static workspace holds the first call's data), and refuse frames too
large for its static workspace."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1503_06959_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kpd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1503_06959_amd import kpd as k
    return k


def run(kpd, frame, t, O, static):
    H, W = frame.shape
    det = kpd.LayerDetector(W, H, t, O)
    dev = torch.from_numpy(np.ascontiguousarray(frame)).cuda()
    det.out.fill_(0xAB)
    if static:
        det.detect_static_async(dev)
    else:
        det.detect_async(dev)
    torch.cuda.synchronize()
    n = int(det.count.item())
    raw = det.out[:min(n, det.capacity) * kpd.KEYPOINT_DTYPE.itemsize].cpu().numpy().view(kpd.KEYPOINT_DTYPE)
    return n, raw.copy()


def test_static_workspace_matches_caller_workspace(kpd):
    big = synth.make_video(synth.SCENES["c3_1920x1080"], 1)[0]
    small = synth.make_video(synth.SCENES["c1_320x240"], 1)[0]
    for frame, t, O in [(big, 20, 5), (small, 30, 3), (big[:480, :640].copy(), 20, 4)]:
        ref_n, ref = run(kpd, frame, t, O, static=False)
        got_n, got = run(kpd, frame, t, O, static=True)
        assert ref_n > 0 and got_n == ref_n
        np.testing.assert_array_equal(got, ref)


def test_static_workspace_limit(kpd):
    f = torch.zeros((2160, 3840), dtype=torch.uint8, device="cuda")
    out = torch.empty(1024, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    assert kpd.layers_bytes(3840, 2160, 5) > kpd.STATIC_WORKSPACE
    rc = kpd.lib.kpd_detect_layers_static(f.data_ptr(), 3840, 3840, 2160, 20, 5, out.data_ptr(), 128,
                                          cnt.data_ptr(), None)
    assert rc == kpd.KPD_EINVAL
    assert b"static workspace" in kpd.lib.kpd_last_error()
