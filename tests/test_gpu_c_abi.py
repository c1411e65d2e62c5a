"""The C ABI used from C alone: tests/c_abi/solve_example (built by
__graft_entry__.build() with gcc against libsuppcg.so and the HIP runtime, no
Python or PyTorch in it) projects, backprojects and solves a 64 x 64 disk
problem; its outputs must equal the Python binding's bit for bit (same library,
same inputs) and R x the oracle's to 1e-5."""
import os
import subprocess

import numpy as np
import pytest

from oracle import projector as oproj
from oracle.geometry import Geometry as OG
from tests._problems import rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "c_abi", "solve_example")


def test_c_client_matches_binding(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.exists(EXE), "tests/c_abi/solve_example is missing: run __graft_entry__.build()"
    out = os.path.join(tmp_path, "out.bin")
    print("C client 64x64x90x91", flush=True)
    res = subprocess.run([EXE, out], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.split()[:2] == ["k", "11"]
    data = np.fromfile(out, dtype=np.float32)
    m, n = 90 * 91, 64 * 64
    y_c, g_c, xh_c = data[:m], data[m:m + n], data[m + n:]

    import paper_1807_10151_amd as sp
    g = sp.Geometry(64, 64, 90, 91)
    ys, xs = np.mgrid[0:64, 0:64]
    img = (((xs - 31.5) ** 2 + (31.5 - ys) ** 2) <= 20.0 ** 2).astype(np.float32)
    x = torch.from_numpy(img).cuda()
    y = sp.sp_project(g, x)
    gg = sp.sp_backproject(g, y)
    r = sp.sp_suppcg_solve(g, y, None, K=1, a=0.5, gamma=0.5, mu=1e-5, rho=0.8, max_iter=10, graph=True,
                           trace=False)
    assert np.array_equal(y.cpu().numpy().ravel(), y_c)
    assert np.array_equal(gg.cpu().numpy().ravel(), g_c)
    assert np.array_equal(r.x_half.cpu().numpy().ravel(), xh_c)
    assert rel_l2(y_c, oproj.project(OG(64, 64, 90, 91), img)) <= 1e-5
