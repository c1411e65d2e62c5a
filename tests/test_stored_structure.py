"""Host-side check of the stored-matrix build (CPU only).

Builds tests/index_check/stored_check.cpp with the library's host geometry
(geometry.cpp) under AddressSanitizer and UndefinedBehaviorSanitizer (host code
only).  The checker replays the row enumeration the build kernels run
(sp_stored.h): counted and filled rows agree, every index is in range and R^T
is exactly R transposed.  Its dump of R is then compared with the oracle's R
(Section 2, eq. 2.1): the same nonzero (ray, pixel) pairs with the same
lengths, to 1e-12 of a pixel plus the rounding that a near-axis angle's
narrow ramp amplifies (a pair missing on one side counts as length 0)."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import projector as oproj
from oracle.geometry import Geometry as OG
from oracle.geometry import angle_cos_sin
from tests._problems import random_geometries

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "_build", "stored_check")

# (rows, cols, A, B, pixel, theta0, dtheta (<= 0: pi / A), spacing, offset)
GEOMS = [
    (64, 64, 90, 91, 1.0, 0.0, -1.0, 1.0, 0.0),          # the 64 x 64 workload
    (37, 53, 45, 61, 1.0, 0.0, -1.0, 1.0, 0.0),
    (16, 16, 8, 24, 0.7, 0.0, -1.0, 0.5, 0.13),
    (20, 24, 7, 33, 1.0, 0.1, 0.45, 1.0, 0.0),
    (1, 1, 4, 3, 1.0, 0.0, -1.0, 1.0, 0.0),
    (3, 70, 1, 5, 1.0, 0.0, -1.0, 1.0, 0.0),
    (41, 57, 4, 75, 1.0, 1e-7, np.pi / 2, 1.0, 0.0),     # near-axis angles
    (64, 48, 6, 85, 1.0, np.pi / 4 - 1e-9, np.pi / 4, 1.0, 0.0),
    (30, 30, 5, 47, 1.0, np.pi / 2 - 3e-8, 1e-8, 1.0, 0.0),
    (40, 56, 70, 100, 1.0, 0.0, -1.0, 0.7, 0.3),
]


def line(r):
    return " ".join(repr(float(v)) if isinstance(v, float) else str(v) for v in r)


@pytest.fixture(scope="module")
def checker():
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if not hipcc:
        pytest.skip("hipcc not available")
    os.makedirs(os.path.dirname(EXE), exist_ok=True)
    cmd = [hipcc, "-std=c++17", "-O1", "-g", "-ffp-contract=off",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"),
           "-o", EXE, os.path.join(ROOT, "tests", "index_check", "stored_check.cpp"),
           os.path.join(ROOT, "paper_1807_10151_amd", "csrc", "geometry.cpp")]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return EXE


ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def test_rows_in_range_and_transposes_exact(checker):
    rows = list(GEOMS)
    for og in random_geometries(24):
        rows.append((og.rows, og.cols, og.n_angles, og.n_bins, og.pixel, og.theta0,
                     og.dtheta if og.dtheta is not None else -1.0, og.bin_spacing, og.bin_offset))
    res = subprocess.run([checker], input="\n".join(line(r) for r in rows) + "\n",
                         capture_output=True, text=True, env=ENV, timeout=900)
    print(res.stdout[-3000:])
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert f"checked {len(rows)} geometries" in res.stdout


@pytest.mark.parametrize("geom", GEOMS, ids=[f"{g[0]}x{g[1]}x{g[2]}x{g[3]}" for g in GEOMS])
def test_stored_r_matches_oracle(checker, geom):
    r, c, a, b, px, t0, dt, sp, off = geom
    og = OG(r, c, a, b, pixel=px, theta0=t0, dtheta=None if dt <= 0 else dt, bin_spacing=sp, bin_offset=off)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "r.bin")
        res = subprocess.run([checker, "--dump", path], input=line(geom) + "\n", capture_output=True,
                             text=True, env=ENV, timeout=300)
        assert res.returncode == 0, res.stdout + res.stderr
        rec = np.fromfile(path, dtype=np.dtype([("ray", "<i4"), ("pix", "<i4"), ("w", "<f8")]))
    R, _ = oproj.matrix(og)
    R = R.tocoo()
    keep = R.data > 0
    want = dict(zip(zip(R.row[keep].tolist(), R.col[keep].tolist()), R.data[keep].tolist()))
    got = dict(zip(zip(rec["ray"].tolist(), rec["pix"].tolist()), rec["w"].tolist()))
    assert len(got) == len(rec)                       # no pair twice
    # Both sides evaluate the exact chord length of a line through a square:
    # a trapezoid in the offset d of the pixel centre whose ramps are min(|c|,
    # |s|) wide.  Rounding of d (a few ulp of the image extent) moves a weight
    # on a ramp by up to that error over the ramp width, which is large only
    # for angles within ~1e-6 rad of an axis that do not snap to it.
    ext = (og.rows + og.cols) * px + og.n_bins * og.bin_spacing + abs(og.bin_offset)
    tol_a = []
    for ai in range(og.n_angles):
        _, co, si = angle_cos_sin(og, ai)
        ramp = min(abs(co), abs(si))
        tol_a.append(1e-12 * px + (8e-16 * ext / ramp * px if ramp > 0 else 0.0))
    worst = 0.0
    for k in set(got) | set(want):
        diff = abs(got.get(k, 0.0) - want.get(k, 0.0))
        worst = max(worst, diff / tol_a[k[0] // og.n_bins])
    assert worst <= 1.0, worst
    # rows in the order the kernels store them: rays ascending
    assert np.all(np.diff(rec["ray"]) >= 0)
