"""Launch-shape tuning of the projector pair on the GPU.

Bars: every part count gives R within 1e-12 relative of the one-part result
(the parts' float64 sums are added in order; only rounding differs) and within
1e-5 of the oracle; R^T is bitwise the same for 2 and 4 pixels per lane; a
batch whose slices carry tuned shapes equals the same slices solved one by
one, bit for bit; the tuner stores a valid choice for every geometry it
times, and the batched solver's autotune tunes the geometries the table lacks.
"""
import numpy as np
import pytest

from oracle import projector as oproj
from tests._problems import A, GAMMA, K, MU, RHO, rel_l2, workload_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1807_10151_amd as sp_mod
    sp_mod.tuning_clear()
    yield sp_mod
    sp_mod.tuning_clear()


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def test_shapes_change_rounding_only(sp):
    og, img, b = workload_problem("small64")
    g = sp.Geometry(og.rows, og.cols, og.n_angles, og.n_bins)
    R, _ = oproj.matrix(og)
    rng = np.random.default_rng(5)
    y = rng.standard_normal((og.n_angles, og.n_bins)).astype(np.float32)
    want_R = R @ img.astype(np.float64).ravel()
    want_RT = R.T @ y.astype(np.float64).ravel()
    ref_R = ref_RT = None
    for parts in (1, 2, 4, 8):
        for px in (2, 4):
            print(f"shape parts={parts} px={px}", flush=True)
            sp.tuning_set(g, parts, px)
            r = sp.sp_project(g, cuda(img)).cpu().numpy().ravel()
            t = sp.sp_backproject(g, cuda(y)).cpu().numpy().ravel()
            assert rel_l2(r, want_R) <= 1e-5 and rel_l2(t, want_RT) <= 1e-5
            if ref_R is None:
                ref_R, ref_RT = r, t
            assert rel_l2(r, ref_R) <= 1e-12
            assert np.array_equal(t, ref_RT)
    sp.tuning_set(g, 0, 0)


def test_tuner_stores_a_valid_choice(sp):
    g = sp.Geometry(256, 256, 360, 362)
    print("tune 256x256x360x362", flush=True)
    res = sp.tune_shapes(g)
    assert res["parts"] in (1, 2, 4, 8) and res["px"] in (2, 4)
    assert all(v > 0 for v in res["R_ms"].values()) and all(v > 0 for v in res["RT_ms"].values())
    assert (g, res["parts"], res["px"]) in sp.tuning_list()
    # the chosen shape is no slower than the others by more than the 2% tie margin
    assert res["R_ms"][res["parts"]] <= 1.02 * min(res["R_ms"].values()) + 1e-3
    sp.tuning_set(g, 0, 0)


def test_batch_equals_single_with_tuned_shapes(sp):
    geoms = [sp.Geometry(64, 64, 90, 91), sp.Geometry(37, 53, 45, 61), sp.Geometry(130, 96, 128, 165)]
    shapes = [(2, 4), (4, 2), (8, 4)]
    for g, (p, x) in zip(geoms, shapes):
        sp.tuning_set(g, p, x)
    rng = np.random.default_rng(11)
    bs = [cuda(rng.uniform(0, 10, (g.n_angles, g.n_bins))) for g in geoms]
    kw = dict(K=K, a=A, gamma=GAMMA, mu=MU, rho=RHO, max_iter=6)
    print("batched with tuned shapes", flush=True)
    res_b = sp.sp_suppcg_solve_batched(geoms, bs, graph=True, **kw)
    for g, b, rb in zip(geoms, bs, res_b):
        rs = sp.sp_suppcg_solve(g, b, None, graph=True, trace=False, **kw)
        assert rs.k == rb.k
        assert torch.equal(rs.x_half, rb.x_half) and torch.equal(rs.x_last, rb.x_last)
    for g in geoms:
        sp.tuning_set(g, 0, 0)


def test_batched_autotune_tunes_missing_geometries(sp):
    sp.tuning_clear()
    geoms = [sp.Geometry(64, 64, 90, 91), sp.Geometry(96, 80, 60, 131), sp.Geometry(64, 64, 90, 91)]
    rng = np.random.default_rng(12)
    bs = [cuda(rng.uniform(0, 10, (g.n_angles, g.n_bins))) for g in geoms]
    print("batched autotune", flush=True)
    res = sp.sp_suppcg_solve_batched(geoms, bs, graph=True, autotune=True, K=K, a=A, gamma=GAMMA, mu=MU,
                                     rho=RHO, max_iter=3)
    assert all(r.k == 4 for r in res)
    tuned = {k for k, _, _ in sp.tuning_list()}
    assert tuned == {geoms[0], geoms[1]}
    # a single solve now uses the same shapes: bitwise the batch's slice
    rs = sp.sp_suppcg_solve(geoms[1], bs[1], None, graph=True, trace=False, K=K, a=A, gamma=GAMMA, mu=MU,
                            rho=RHO, max_iter=3)
    assert torch.equal(rs.x_half, res[1].x_half)
    sp.tuning_clear()
