"""Host-side check of the projector pair's index arithmetic (CPU only).

Builds tests/index_check/index_check.cpp together with the library's host
geometry (geometry.cpp) under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only) and runs it over the workload geometries, the ragged and
random geometries of the GPU parity tests and the batched slice shapes.  The
checker replays, with the kernels' own index helpers, every wave of R and
every pixel and angle of R^T -- the pixels of partial tiles past the image
edge included -- and fails if a ray's bands fall outside its wave's step
range, a gathered pair or candidate window of an image pixel leaves its
padded row, or a crossed pixel or bin falls outside what is gathered."""
import math
import os
import shutil
import subprocess

import pytest

from tests._problems import random_geometries

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "_build", "index_check")


def geometries():
    """(rows, cols, A, B, pixel, theta0, dtheta, spacing, offset, ray_stride, pixel_stride)."""
    g = []
    add = lambda r, c, a, b, px=1.0, t0=0.0, dt=-1.0, sp=1.0, off=0.0, rs=1, ps=1: g.append(
        (r, c, a, b, px, t0, dt, sp, off, rs, ps))
    add(64, 64, 90, 91)                       # the 64 x 64 workload
    add(512, 512, 720, 725, rs=5, ps=11)      # the 512^2 workload (sampled rays and pixels)
    add(243, 243, 360, 345, rs=3, ps=5)       # the paper's shape
    add(2048, 2048, 2048, 2899, rs=211, ps=1999)
    for side in (256, 384, 512, 768, 1024):   # batched slice shapes
        A = 8 * int(round(1.4 * side / 8))
        B = int(math.ceil(side * math.sqrt(2.0))) + 1
        add(side, side, A, B, rs=7 + side // 128, ps=13 + side // 64)
    # the ragged geometries of the operator tests
    for r, c, a, b, px, t0, dt, sp, off in [
            (37, 53, 45, 61, 1, 0, -1, 1, 0), (50, 30, 24, 60, 1, 0, -1, 1, 0),
            (16, 16, 8, 24, 0.7, 0, -1, 0.5, 0.13), (20, 24, 7, 33, 1, 0.1, 0.45, 1, 0),
            (1, 1, 4, 3, 1, 0, -1, 1, 0), (3, 70, 1, 5, 1, 0, -1, 1, 0),
            (33, 33, 360, 47, 1, 0, -1, 1, 0), (200, 150, 30, 251, 1, 0, -1, 1, 0),
            (9, 300, 12, 301, 1, 0.3, -1, 1, 0), (260, 240, 16, 360, 1, 0, 0.19, 1, 0),
            (522, 520, 90, 741, 1, 0, -1, 1, 0), (512, 640, 180, 900, 1, 0, -1, 1, 0),
            (48, 80, 60, 97, 1, 0, -1, 1, 0), (100, 70, 45, 123, 1, 0.1, -1, 1, 0),
            (40, 56, 70, 100, 1, 0, -1, 0.7, 0.3), (130, 96, 128, 165, 1, 0, math.pi / 160, 1, 0),
            (41, 57, 4, 75, 1, 1e-7, math.pi / 2, 1, 0),
            (64, 48, 6, 85, 1, math.pi / 4 - 1e-9, math.pi / 4, 1, 0),
            (30, 30, 5, 47, 1, math.pi / 2 - 3e-8, 1e-8, 1, 0)]:
        add(r, c, a, b, px, t0, dt, sp, off)
    for og in random_geometries(24):
        add(og.rows, og.cols, og.n_angles, og.n_bins, og.pixel, og.theta0,
            og.dtheta if og.dtheta is not None else -1.0, og.bin_spacing, og.bin_offset)
    return g


@pytest.fixture(scope="module")
def checker():
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if not hipcc:
        pytest.skip("hipcc not available")
    os.makedirs(os.path.dirname(EXE), exist_ok=True)
    cmd = [hipcc, "-std=c++17", "-O1", "-g", "-ffp-contract=off",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"),
           "-o", EXE, os.path.join(ROOT, "tests", "index_check", "index_check.cpp"),
           os.path.join(ROOT, "paper_1807_10151_amd", "csrc", "geometry.cpp")]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return EXE


def test_projector_indices_stay_in_rows_and_cover_every_crossing(checker):
    lines = "\n".join(" ".join(repr(v) if isinstance(v, float) else str(v) for v in row)
                      for row in geometries()) + "\n"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([checker], input=lines, capture_output=True, text=True, env=env, timeout=900)
    print(res.stdout[-4000:])
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert f"checked {len(geometries())} geometries" in res.stdout
    assert "tile order: ok" in res.stdout
