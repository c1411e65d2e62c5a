"""R and R^T on seeded random parallel-beam geometries against the CPU oracle:
image sizes, angle sets (start, step, count), bin counts, spacings and offsets
drawn at random, so the projector's workgroup order, its per-step product
table and the backprojector's scaled rows meet shapes the fixed cases do not.
Same bar as the fixed cases (1e-5 relative L2), plus the adjoint identity, and
a short batched solve over several of the geometries against single solves
(bitwise)."""
import math

import numpy as np
import pytest

from oracle import projector as oproj
from oracle.geometry import Geometry as OG
from tests._problems import random_geometries, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1807_10151_amd as sp_mod
    return sp_mod


GEOMS = random_geometries(24) + [
    # angles a hair away from the axes and from 45 degrees: the split walk's
    # band shares 1/|slope| become huge or reach 1
    OG(41, 57, 4, 75, theta0=1e-7, dtheta=math.pi / 2),
    OG(64, 48, 6, 85, theta0=math.pi / 4 - 1e-9, dtheta=math.pi / 4),
    OG(30, 30, 5, 47, theta0=math.pi / 2 - 3e-8, dtheta=1e-8),
]


def G(sp, og):
    return sp.Geometry(og.rows, og.cols, og.n_angles, og.n_bins, og.pixel, og.theta0, og.dtheta,
                       og.bin_spacing, og.bin_offset)


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("idx", range(len(GEOMS)))
def test_random_geometry_operators(sp, idx):
    og = GEOMS[idx]
    print(f"geometry {idx}: {og}", flush=True)
    rng = np.random.default_rng(100 + idx)
    x = rng.standard_normal((og.rows, og.cols)).astype(np.float32)
    y = rng.standard_normal((og.n_angles, og.n_bins)).astype(np.float32)
    g = G(sp, og)
    Rx = sp.sp_project(g, cuda(x))
    RTy = sp.sp_backproject(g, cuda(y))
    want_R = oproj.project(og, x.astype(np.float64))
    want_RT = oproj.backproject(og, y.astype(np.float64))
    assert rel_l2(Rx.cpu().numpy().ravel(), want_R) <= 1e-5
    assert rel_l2(RTy.cpu().numpy().ravel(), want_RT) <= 1e-5
    lhs = float((Rx.double() * cuda(y).double()).sum())
    rhs = float((cuda(x).double() * RTy.double()).sum())
    assert abs(lhs - rhs) <= 1e-6 * max(abs(lhs), float(Rx.double().norm()) * float(np.linalg.norm(y)))


def test_random_geometries_batched_equals_single(sp):
    picks = [GEOMS[i] for i in (0, 3, 7, 11, 16, 21)]
    geoms = [G(sp, og) for og in picks]
    bs = []
    for i, og in enumerate(picks):
        rng = np.random.default_rng(300 + i)
        x = np.abs(rng.standard_normal((og.rows, og.cols))).astype(np.float32)
        bs.append(sp.sp_project(geoms[i], cuda(x)).contiguous())
    kw = dict(K=1, a=0.5, gamma=0.5, mu=1e-5, rho=0.8, max_iter=3)
    got = sp.sp_suppcg_solve_batched(geoms, bs, graph=True, **kw)
    for i, g in enumerate(geoms):
        r = sp.sp_suppcg_solve(g, bs[i], None, graph=True, **kw)
        assert got[i].k == r.k
        np.testing.assert_array_equal(got[i].x_half.cpu().numpy(), r.x_half.cpu().numpy())
        np.testing.assert_array_equal(got[i].trace["f_half"], r.trace["f_half"])
