"""CPU-side checks of the C ABI library: it loads, exports every symbol that
include/kpd.h declares, validates parameters before touching the device, and
its cell geometry covers every neighbourhood the detector reads."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kpd.h")


def _lib_built():
    from paper_1503_06959_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    return build.LIB


@pytest.fixture(scope="module")
def kpd():
    _lib_built()
    from paper_1503_06959_amd import kpd as k
    return k


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b([A-Za-z_]\w*)\s*\([^;{]*\)\s*;", text, flags=re.M)
    return [n for n in names if n not in ("if", "while")]


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("stream_bytes", "open_stream", "set_thresholds", "push_frame", "get_keypoints",
              "close_stream", "kpd_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(kpd):
    lib = _lib_built()
    out = subprocess.run(["nm", "-D", "--defined-only", lib], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for n in declared_functions():
        assert n in exported, n
        assert hasattr(kpd.lib, n)
    assert set(kpd.EXPORTED) <= set(declared_functions())


def test_struct_layouts_match_header(kpd):
    assert ctypes.sizeof(kpd.KpdParams) == 52
    assert kpd.KEYPOINT_DTYPE.itemsize == 8
    assert kpd.KEYPOINT_DTYPE.fields["octave"][1] == 4
    assert kpd.KEYPOINT_DTYPE.fields["score"][1] == 6


@pytest.mark.parametrize("W,H,det", [
    (320, 240, (30, 3, 8, 6)), (640, 480, (20, 4, 16, 12)), (1920, 1080, (20, 5, 32, 18)),
    (1280, 720, (20, 5, 32, 18)), (333, 251, (25, 4, 7, 5)),
])
def test_stream_bytes_covers_frames_pyramid_and_keypoint_slots(kpd, W, H, det):
    p = kpd.make_params(*det)
    n = kpd.stream_bytes(W, H, p)
    O = det[1]
    pyr = sum((W >> o) * (H >> o) for o in range(1, O))
    # two frame slots, the pyramid, and two keypoint lists of >= 1 entry per 4 px of level 0
    assert n >= 2 * W * H + pyr + 2 * 8 * ((W - 6) // 2) * ((H - 6) // 2)
    assert n < 64 * W * H + (1 << 20)


def test_chunk_frames_sizes_the_arena(kpd):
    base = kpd.stream_bytes(640, 480, kpd.make_params(20, 4, 16, 12))
    assert kpd.stream_bytes(640, 480, kpd.make_params(20, 4, 16, 12, chunk_frames=1)) == base
    prev = base
    for K in (2, 8, 64, 256, 512):
        n = kpd.stream_bytes(640, 480, kpd.make_params(20, 4, 16, 12, chunk_frames=K))
        # per chunk frame at least its octaves 1.. and one keypoint list
        pyr = sum((640 >> o) * (480 >> o) for o in range(1, 4))
        assert n >= base + (K - 1) * pyr + K * 8 * (317 // 2) * (237 // 2)
        assert n > prev
        prev = n
    for K in (-1, 513):
        p = kpd.make_params(20, 4, 16, 12, chunk_frames=K)
        assert kpd.lib.stream_bytes(640, 480, ctypes.byref(p)) == 0


@pytest.mark.parametrize("W,H,det,why", [
    (320, 240, (0, 3, 8, 6), "t"), (320, 240, (255, 3, 8, 6), "t"),
    (320, 240, (20, 0, 8, 6), "O"), (320, 240, (20, 9, 8, 6), "O"),
    (8, 8, (20, 5, 1, 1), "O vs size"), (320, 240, (20, 3, 0, 6), "grid"),
    (320, 240, (20, 3, 321, 6), "grid"), (320, 240, (20, 3, 2, 6), "cell > 128"),
    (0, 240, (20, 3, 8, 6), "size"), (20000, 240, (20, 3, 8, 6), "size"),
])
def test_invalid_parameters_are_rejected(kpd, W, H, det, why):
    p = kpd.make_params(*det)
    assert kpd.lib.stream_bytes(W, H, ctypes.byref(p)) == 0, why
    h = ctypes.c_void_p()
    rc = kpd.lib.open_stream(W, H, ctypes.byref(p), ctypes.c_void_p(1 << 20), 1 << 30, None, ctypes.byref(h))
    assert rc == kpd.KPD_EINVAL
    assert kpd.lib.kpd_last_error().decode()


def test_small_or_misaligned_arena_is_rejected_before_any_device_call(kpd):
    p = kpd.make_params(30, 3, 8, 6)
    need = kpd.stream_bytes(320, 240, p)
    h = ctypes.c_void_p()
    rc = kpd.lib.open_stream(320, 240, ctypes.byref(p), ctypes.c_void_p(1 << 20), need - 1, None, ctypes.byref(h))
    assert rc == kpd.KPD_ENOMEM
    rc = kpd.lib.open_stream(320, 240, ctypes.byref(p), ctypes.c_void_p((1 << 20) + 8), need, None,
                             ctypes.byref(h))
    assert rc == kpd.KPD_EINVAL
    rc = kpd.lib.open_stream(320, 240, ctypes.byref(p), None, need, None, ctypes.byref(h))
    assert rc == kpd.KPD_EINVAL


def test_null_handles_report_state_errors(kpd):
    assert kpd.lib.push_frame(None, None, 0, 0) == kpd.KPD_ESTATE
    cnt = ctypes.c_size_t()
    assert kpd.lib.get_keypoints(None, None, 0, ctypes.byref(cnt), None) == kpd.KPD_ESTATE
    assert kpd.lib.set_thresholds(None, 20, 8, 0) == kpd.KPD_ESTATE
    assert kpd.lib.close_stream(None) == kpd.KPD_ESTATE


@pytest.fixture(scope="module")
def geom_check(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("geom") / "geom_check")
    subprocess.run(["g++", "-std=c++17", "-O2", "-o", exe, os.path.join(ROOT, "tests", "geom_check.cpp")],
                   check=True)
    return exe


@pytest.mark.parametrize("shape", [
    "320 240 3 8 6", "640 480 4 16 12", "1920 1080 5 32 18", "1280 720 5 32 18",
    "2048 1536 8 16 12", "7 7 1 1 1", "13 9 2 3 2", "100 37 3 1 1", "127 255 7 1 2", "1000 999 6 8 8",
    "333 251 4 7 5", "64 64 7 1 1",
])
def test_cell_geometry_partitions_and_covers_neighbourhoods(geom_check, shape):
    out = subprocess.run([geom_check, *shape.split()], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout
    lds = int(out.stdout.split()[1])
    assert lds <= 160 * 1024


@pytest.fixture(scope="module")
def group_check(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("group") / "group_check")
    subprocess.run(["g++", "-std=c++17", "-O2", "-o", exe, os.path.join(ROOT, "tests", "group_check.cpp")],
                   check=True)
    return exe


@pytest.mark.parametrize("shape", [
    "320 240 3 8 6 1 1", "320 240 3 8 6 3 1", "320 240 3 8 6 2 3", "320 240 3 8 6 8 2", "320 240 3 8 6 4 4",
    "640 480 4 16 12 4 1", "640 480 4 16 12 4 2", "1920 1080 5 32 18 2 1", "1920 1080 5 32 18 4 1",
    "1920 1080 5 32 18 1 1", "1280 720 5 32 18 4 1", "2048 1536 8 16 12 1 1", "7 7 1 1 1 1 1",
    "13 9 2 3 2 2 2", "9 13 2 3 2 2 2", "100 37 3 1 1 1 1", "127 255 7 1 2 1 2", "1000 999 6 8 8 3 3",
    "333 251 4 7 5 3 2", "333 251 4 7 5 7 1", "64 64 7 1 1 1 1", "200 150 3 5 3 5 3", "170 130 4 3 2 3 2",
])
def test_group_geometry_covers_scores_reads_and_cells(group_check, shape):
    out = subprocess.run([group_check, *shape.split()], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout


def test_group_params_are_validated(kpd):
    ok = kpd.make_params(20, 4, 16, 12, chunk_frames=4, group_cols=4, group_rows=2)
    assert kpd.lib.stream_bytes(640, 480, ctypes.byref(ok)) > 0
    for gc, gr, gt in [(4, 0, 0), (0, 2, 0), (17, 1, 0), (1, 13, 0), (-1, 1, 0), (4, 1, 128), (4, 1, 1024)]:
        p = kpd.make_params(20, 4, 16, 12, chunk_frames=4, group_cols=gc, group_rows=gr, group_threads=gt)
        assert kpd.lib.stream_bytes(640, 480, ctypes.byref(p)) == 0, (gc, gr, gt)
    p = kpd.make_params(20, 4, 16, 12, chunk_frames=4, group_cols=4, group_rows=1, group_threads=512)
    assert kpd.lib.stream_bytes(640, 480, ctypes.byref(p)) > 0
    # more LDS than a workgroup holds
    p = kpd.make_params(20, 3, 8, 6, chunk_frames=4, group_cols=8, group_rows=6)
    assert kpd.lib.stream_bytes(320, 240, ctypes.byref(p)) == 0


def test_descriptor_pattern_matches_the_oracle(kpd):
    # the library builds its pattern tables from the same stated rings as the
    # oracle, in code of its own: every point of every sector agrees
    import oracle
    for sector in range(32):
        pat = oracle.desc_pattern(sector)
        lib_pat = [kpd.desc_point(sector, i) for i in range(60)]
        assert [tuple(int(v) for v in row) for row in pat] == lib_pat, sector
    with pytest.raises(kpd.KpdError):
        kpd.desc_point(32, 0)


def test_descriptor_flag_is_validated(kpd):
    p = kpd.make_params(20, 4, 16, 12, features=4)
    assert kpd.lib.stream_bytes(640, 480, ctypes.byref(p)) == 0
    base = kpd.stream_bytes(640, 480, kpd.make_params(20, 4, 16, 12))
    with_desc = kpd.stream_bytes(640, 480, kpd.make_params(20, 4, 16, 12, features=kpd.FEAT_DESCRIPTOR))
    assert with_desc > base + 2 * 72 * 1000   # two descriptor lists and the tables
    with_ref = kpd.stream_bytes(640, 480, kpd.make_params(20, 4, 16, 12, features=kpd.FEAT_REFINE))
    assert with_ref > base + 2 * 16 * 1000    # two lists of refined values
    both = kpd.stream_bytes(640, 480, kpd.make_params(20, 4, 16, 12, features=3))
    assert both > max(with_desc, with_ref)


def test_tcd_structs_and_sizes(kpd):
    # the tracker's records and parameter block match the header, and its
    # arena holds the inner stream plus two frame slots and three track lists
    assert kpd.TRACK_DTYPE.itemsize == 16 and ctypes.sizeof(kpd.KpdTcdParams) == 16
    p = kpd.make_params(20, 4, 16, 12)
    tp = kpd.KpdTcdParams(10, 1800, 1000, 0)
    n = kpd.tcd_bytes(640, 480, p, tp)
    inner = kpd.stream_bytes(640, 480, kpd.make_params(20, 4, 16, 12, id_thresh=-1))
    cap = sum(((640 >> o) + 1) // 2 * (((480 >> o) + 1) // 2) for o in range(4)) + 16
    assert n >= inner + 2 * 640 * 480 + 3 * 16 * cap
    for bad in (kpd.KpdTcdParams(0, 1800, 1000, 0), kpd.KpdTcdParams(10, -1, 1000, 0),
                kpd.KpdTcdParams(10, 1800, -5, 0), kpd.KpdTcdParams(10, 1800, 1000, 1)):
        assert kpd.lib.tcd_bytes(640, 480, ctypes.byref(p), ctypes.byref(bad)) == 0
    assert kpd.lib.tcd_bytes(640, 480, ctypes.byref(kpd.make_params(20, 0, 16, 12)), ctypes.byref(tp)) == 0


def test_layer_workspace_sizes(kpd):
    # the workspace holds every layer past the frame, 2-byte scores and a
    # flag per layer pixel, and two words per block of 256 layer pixels
    import oracle
    for W, H, O in ((640, 480, 4), (101, 77, 6), (1, 1, 1)):
        dims = oracle.layer_dims(W, H, O)
        N = sum(w * h for w, h, _ in dims)
        n = kpd.layers_bytes(W, H, O)
        assert n >= sum(w * h for w, h, _ in dims[1:]) + 3 * N + 8 * ((N + 255) // 256)
        end = 0
        for l in range(1, 2 * O):
            off, w, h = kpd.layer_plane(W, H, O, l)
            assert (w, h) == dims[l][:2] and off >= end and off % 256 == 0
            end = off + w * h
    assert kpd.lib.kpd_layers_bytes(640, 480, 0) == 0
    assert kpd.lib.kpd_layers_bytes(640, 480, 9) == 0
    assert kpd.lib.kpd_layers_bytes(0, 480, 4) == 0
    with pytest.raises(kpd.KpdError):
        kpd.layer_plane(640, 480, 4, 0)
    with pytest.raises(kpd.KpdError):
        kpd.layer_plane(640, 480, 4, 8)


def test_layer_stream_radius_bound():
    # the masked layered stream scores the cells within R / (narrowest
    # cell) + 1 of a marked one, R = S_max / 2 + 1 level-0 pixels: every
    # suppression neighbour's footprint start lies within max(S_p, S_q) / 2
    # + 1 pixels of the pixel's own (S in half pixels)
    import oracle
    sizes = [2, 3, 4, 6, 8, 12, 16, 24, 32, 48]
    for i, S1 in enumerate(sizes):
        for S2 in sizes[max(i - 1, 0):i + 2]:
            for x in range(0, 200):
                lo, hi = oracle.layer_range(S1, S2, x)
                for q in range(max(lo, 0), hi + 1):
                    d = abs((q * S2) // 2 - (x * S1) // 2)
                    assert d <= max(S1, S2) // 2 + 1, (S1, S2, x, q)


def test_lstream_sizes(kpd):
    # the masked layered stream holds the layer workspace, two frame slots,
    # the cell tables and two D lists of the layers' keypoint bound
    import oracle
    p = kpd.make_params(20, 4, 16, 12)
    n = kpd.lib.kpd_lstream_bytes(640, 480, ctypes.byref(p))
    dims = oracle.layer_dims(640, 480, 4)
    cap = sum(((w + 1) // 2) * ((h + 1) // 2) for w, h, _ in dims) + 16
    assert n >= kpd.layers_bytes(640, 480, 4) + 2 * 640 * 480 + 2 * 8 * cap
    for bad in (kpd.make_params(0, 4, 16, 12), kpd.make_params(20, 9, 16, 12), kpd.make_params(20, 4, 0, 12),
                kpd.make_params(20, 4, 641, 12), kpd.make_params(20, 4, 16, 481)):
        assert kpd.lib.kpd_lstream_bytes(640, 480, ctypes.byref(bad)) == 0


HANDLE_TYPES = ("kpd_stream", "kpd_batch", "kpd_lstream", "kpd_lbatch", "kpd_tcd")


def handle_calls():
    """(name, number of parameters) of every int-returning call of the header
    whose first parameter is a handle (opens, which take a handle's address,
    excluded)."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = []
    for ret, name, params in re.findall(r"^(int)\s+([A-Za-z_]\w*)\s*\(([^;{]*)\)\s*;", text, flags=re.M):
        ps = [p.strip() for p in params.split(",")]
        first = ps[0].replace("const", "").replace("*", " * ").split()
        if first and first[0] in HANDLE_TYPES and first.count("*") == 1:
            out.append((name, len(ps)))
    return out


def test_unknown_handles_are_refused_before_use(kpd):
    # a pointer the library never handed out (here zeroed host memory) is
    # refused with KPD_ESTATE by every call that takes a handle, closes
    # included, without reading through it
    calls = handle_calls()
    names = {n for n, _ in calls}
    for n in ("push_frame", "get_keypoints", "close_stream", "batch_tick", "close_batch", "kpd_lbatch_tick",
              "kpd_lstream_push", "tcd_push"):
        assert n in names, n
    fake = ctypes.create_string_buffer(4096)
    lib = ctypes.CDLL(kpd.lib._name)
    for name, nparams in calls:
        fn = getattr(lib, name)
        fn.restype = ctypes.c_int
        fn.argtypes = [ctypes.c_void_p] * nparams
        rc = fn(ctypes.addressof(fake), *([None] * (nparams - 1)))
        assert rc == kpd.KPD_ESTATE, f"{name} returned {rc}"
