"""CPU tier under the address and undefined-behaviour sanitizers.

The oracle is rebuilt with -fsanitize=address,undefined and its pins
(tests/test_oracle_pins.py) run against that build in a child process with
the sanitizer runtime preloaded; any report fails the test. The host-side
geometry of the library (cell layouts, group layouts, their checks) runs the
same way through the two geometry checkers, and the library's parameter
validation (stream_bytes over valid and invalid parameters) through a host
build of libkpd.so with the host code sanitized."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV_SAN = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:exitcode=86",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:exitcode=87"}


def gcc_runtime(name):
    return subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True,
                          check=True).stdout.strip()


def test_oracle_pins_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "libkpd_oracle_san.so")
    subprocess.run(["gcc", *SAN, "-std=c99", "-ffp-contract=off", "-shared", "-fPIC", "-o", lib,
                    os.path.join(ROOT, "oracle", "kpd_oracle.c"), "-lm"], check=True)
    env = dict(os.environ, **ENV_SAN, KPD_ORACLE_LIB=lib, LD_PRELOAD=gcc_runtime("libasan.so"))
    # the slowest brute-force cases are left to the unsanitized run
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1500)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail


@pytest.mark.parametrize("prog,shapes", [
    ("geom_check.cpp", ["320 240 3 8 6", "1920 1080 5 32 18", "13 9 2 3 2", "127 255 7 1 2", "333 251 4 7 5"]),
    ("group_check.cpp", ["320 240 3 8 6 3 1", "1920 1080 5 32 18 2 1", "9 13 2 3 2 2 2", "127 255 7 1 2 1 2",
                         "333 251 4 7 5 3 2"]),
])
def test_geometry_checkers_under_asan_ubsan(tmp_path, prog, shapes):
    exe = str(tmp_path / prog.replace(".cpp", ""))
    subprocess.run(["g++", *SAN, "-std=c++17", "-o", exe, os.path.join(ROOT, "tests", prog)], check=True)
    env = dict(os.environ, **ENV_SAN)
    for shape in shapes:
        r = subprocess.run([exe, *shape.split()], capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0 and r.stdout.startswith("ok"), (shape, r.stdout, r.stderr[-2000:])


CHILD = r'''
import ctypes, sys
L = ctypes.CDLL(sys.argv[1])
class P(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("fast_t", "n_octaves", "grid_cols", "grid_rows", "id_thresh")] + \
               [("kb_thresh", ctypes.c_uint32)] + \
               [(n, ctypes.c_int32) for n in ("tile", "chunk_frames", "layer_mask", "features", "group_cols",
                                               "group_rows", "group_threads")]
L.stream_bytes.restype = ctypes.c_size_t
L.stream_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
L.kpd_last_error.restype = ctypes.c_char_p
L.kpd_layers_bytes.restype = ctypes.c_size_t
L.kpd_lstream_bytes.restype = ctypes.c_size_t
L.kpd_lstream_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
L.batch_bytes.restype = ctypes.c_size_t
good = [(320, 240, (30, 3, 8, 6, 8, 0xFFFFFFFF, 0, 0, 0, 0, 0, 0)),
        (640, 480, (20, 4, 16, 12, 8, 0xFFFFFFFF, 64, 300, 1, 3, 0, 0)),
        (1920, 1080, (20, 5, 32, 18, -1, 0, 0, 300, 0, 0, 2, 1)),
        (333, 251, (25, 4, 7, 5, 4, 3, 0, 5, 0, 0, 3, 2)),
        (7, 7, (10, 1, 1, 1, 8, 0xFFFFFFFF, 0, 2, 0, 0, 1, 1)),
        (2048, 1536, (20, 8, 16, 12, 8, 0xFFFFFFFF, 128, 4, 0, 0, 0, 0)),
        (1920, 1080, (20, 5, 32, 18, -1, 0, 0, 300, 0, 0, 4, 1, 512))]
bad = [(320, 240, (0, 3, 8, 6, 8, 0, 0, 0, 0, 0, 0, 0)), (320, 240, (30, 9, 8, 6, 8, 0, 0, 0, 0, 0, 0, 0)),
       (320, 240, (30, 3, 0, 6, 8, 0, 0, 0, 0, 0, 0, 0)), (320, 240, (30, 3, 1, 1, 8, 0, 0, 0, 0, 0, 0, 0)),
       (320, 240, (30, 3, 8, 6, 8, 0, 48, 0, 0, 0, 0, 0)), (320, 240, (30, 3, 8, 6, 8, 0, 0, 513, 0, 0, 0, 0)),
       (320, 240, (30, 3, 8, 6, 8, 0, 0, 0, 2, 0, 0, 0)), (320, 240, (30, 3, 8, 6, 8, 0, 0, 0, 0, 8, 0, 0)),
       (320, 240, (30, 3, 8, 6, 8, 0, 0, 4, 0, 0, 9, 1)), (320, 240, (30, 3, 8, 6, 8, 0, 0, 4, 0, 0, 8, 6)),
       (0, 240, (30, 3, 8, 6, 8, 0, 0, 0, 0, 0, 0, 0)), (20000, 240, (30, 3, 8, 6, 8, 0, 0, 0, 0, 0, 0, 0)),
       (3, 3, (30, 3, 1, 1, 8, 0, 0, 0, 0, 0, 0, 0)), (320, 240, (30, 3, 8, 6, 8, 0, 0, 4, 0, 0, 1, 1, 300))]
for W, H, v in good:
    p = P(*v)
    assert L.stream_bytes(W, H, ctypes.byref(p)) > 0, (W, H, v, L.kpd_last_error())
    assert L.kpd_lstream_bytes(W, H, ctypes.byref(p)) > 0 or v[1] > 6, (W, H, v, L.kpd_last_error())
for W, H, v in bad:
    p = P(*v)
    assert L.stream_bytes(W, H, ctypes.byref(p)) == 0, (W, H, v)
    assert L.kpd_last_error(), (W, H, v)
assert L.stream_bytes(320, 240, None) == 0
assert L.kpd_layers_bytes(640, 480, 4) > 0 and L.kpd_layers_bytes(0, 480, 4) == 0
assert L.batch_bytes(64, 1 << 16) > 0
print("ok")
'''


def test_library_parameter_validation_under_asan_ubsan(tmp_path):
    from paper_1503_06959_amd import build as kbuild
    # host code sanitized (the device code is built plainly; the calls here never launch)
    src = os.path.join(ROOT, "paper_1503_06959_amd", "csrc")
    lib = str(tmp_path / "libkpd_san.so")
    sources = [os.path.join(src, f) for f in ("kpd_api.cpp", "kpd_kernels.hip", "kpd_group.hip", "kpd_tcd.cpp",
                                              "kpd_tcd.hip", "kpd_layers.cpp", "kpd_layers.hip")]
    subprocess.run(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
                    "-fPIC", "-shared", "-ffp-contract=off", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                    "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=undefined", "-shared-libsan",
                    "-o", lib, *sources, *kbuild.LIBS], check=True, capture_output=True)
    rt = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rt:
        pytest.skip("clang's address-sanitizer runtime is not installed")
    env = dict(os.environ, **ENV_SAN, LD_PRELOAD=rt[0])
    r = subprocess.run([sys.executable, "-c", CHILD, lib], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), (r.stdout + r.stderr)[-3000:]
