"""The BlobART kernels' blob projection table against the oracle (CPU only).

tests/index_check/blob_check.cpp builds the table of sp_blob.h (p(d) and its
derivative at 2,049 knots over the blob's radius, cubic Hermite in between)
with the kernels' constants and evaluates it at given distances.  Pinned to
oracle.blob.blob_projection (scipy's Bessel functions, an independent route
to the line integral of Section 3.4's blob), and the series the table is
built from pinned the same way."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import blob

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "_build", "blob_check")


@pytest.fixture(scope="module")
def checker():
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if not hipcc:
        pytest.skip("hipcc not available")
    os.makedirs(os.path.dirname(EXE), exist_ok=True)
    cmd = [hipcc, "-std=c++17", "-O1", "-ffp-contract=off", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all",
           "-o", EXE, os.path.join(ROOT, "tests", "index_check", "blob_check.cpp")]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return EXE


def evaluate(exe, d):
    res = subprocess.run([exe], input="\n".join(repr(float(v)) for v in d) + "\n", capture_output=True,
                         text=True, timeout=120,
                         env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1"))
    assert res.returncode == 0, res.stderr[-2000:]
    out = np.array([[float(t) for t in ln.split()] for ln in res.stdout.splitlines()])
    return out[:, 0], out[:, 1]


def test_table_matches_the_oracle(checker):
    rng = np.random.default_rng(7)
    d = np.concatenate([np.linspace(-2.2, 2.2, 4401), rng.uniform(-2.0, 2.0, 4000),
                        [0.0, 1e-12, 1.0, 1.999, 1.9999999, 2.0, -2.0, 2.0000001, 5.0]])
    tab, series = evaluate(checker, d)
    want = blob.blob_projection(d)
    peak = float(blob.blob_projection(0.0))
    # the series the table is built from: the line integral to rounding
    assert np.max(np.abs(series - want)) <= 1e-13 * peak
    # the interpolated table: within 1e-11 of the peak everywhere; relative to
    # the weight, 1e-11 above a hundredth of the peak and 1e-8 above a
    # millionth (near the radius p vanishes like (1 - d/a)^(5/2), which a cubic
    # follows less closely; those weights are tiny)
    assert np.max(np.abs(tab - want)) <= 1e-11 * peak
    for floor, rel in ((1e-2, 1e-11), (1e-6, 1e-8)):
        big = want > floor * peak
        assert np.max(np.abs(tab[big] - want[big]) / want[big]) <= rel
    assert np.all(tab[np.abs(d) >= 2.0] == 0.0)
    assert np.array_equal(tab[d > 0][:100], evaluate(checker, -d[d > 0][:100])[0])   # even in d
