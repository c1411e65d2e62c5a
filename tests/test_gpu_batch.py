"""Batched SupPCG (many slices, one launch per stage) on the GPU.

Per slice the batched solve runs the single-slice arithmetic with the same
partial sums in the same order, so each slice must equal its own
sp_suppcg_solve bit for bit; the single-slice solver is itself pinned to the
float64 oracle (test_gpu_solver.py), and one slice here is checked against the
oracle directly."""
import numpy as np
import pytest

from oracle import projector as oproj
from oracle import suppcg as osup
from tests._problems import A, GAMMA, K, MU, RHO, oracle_precond, rel_l2, workload_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1807_10151_amd as sp_mod
    return sp_mod


def mixed_batch(sp):
    """Mixed shapes, angle sets and bin spacings; data = R x + noise (GPU R)."""
    from synth import random_ellipses
    geoms = [sp.Geometry(64, 64, 90, 91),
             sp.Geometry(48, 80, 60, 97),
             sp.Geometry(33, 33, 360, 47),
             sp.Geometry(100, 70, 45, 123, theta0=0.1),
             sp.Geometry(16, 16, 8, 24),
             sp.Geometry(40, 56, 70, 100, bin_spacing=0.7, bin_offset=0.3),
             sp.Geometry(130, 96, 128, 165, dtheta=np.pi / 160),
             sp.Geometry(200, 150, 64, 251, theta0=0.05)]
    bs = []
    for i, g in enumerate(geoms):
        img, rng = random_ellipses(g.rows, g.cols, 5, 300 + i)
        x = torch.from_numpy(img.astype(np.float32)).cuda()
        b = sp.sp_project(g, x)
        noise = torch.from_numpy(rng.standard_normal(g.m).astype(np.float32)).cuda()
        bs.append((b + 0.01 * float(b.max()) * noise.reshape(b.shape)).contiguous())
    return geoms, bs


def singles(sp, geoms, bs, x0s=None, **kw):
    out = []
    for i, (g, b) in enumerate(zip(geoms, bs)):
        x0 = x0s[i] if x0s is not None else None
        out.append(sp.sp_suppcg_solve(g, b, x0, **kw))
    return out


def assert_same(res_b, res_s):
    assert res_b.k == res_s.k
    assert res_b.status == res_s.status
    np.testing.assert_array_equal(res_b.x_half.cpu().numpy(), res_s.x_half.cpu().numpy())
    np.testing.assert_array_equal(res_b.x_last.cpu().numpy(), res_s.x_last.cpu().numpy())
    np.testing.assert_array_equal(res_b.trace["ell"], res_s.trace["ell"])
    np.testing.assert_array_equal(res_b.trace["f_half"], res_s.trace["f_half"])
    np.testing.assert_array_equal(res_b.trace["tv_half"], res_s.trace["tv_half"])


@pytest.mark.parametrize("graph,autotune", [(True, True), (False, False)])
def test_batch_equals_single_solves(sp, graph, autotune):
    geoms, bs = mixed_batch(sp)
    kw = dict(K=K, a=A, gamma=GAMMA, mu=MU, rho=RHO, max_iter=12)
    got = sp.sp_suppcg_solve_batched(geoms, bs, graph=graph, autotune=autotune, **kw)
    want = singles(sp, geoms, bs, **kw)
    for i, (rb, rs) in enumerate(zip(got, want)):
        print(f"slice {i}: k {rb.k} status {rb.status_name}", flush=True)
        assert_same(rb, rs)
    if autotune:
        print("tuning:", sp.batch_tuning(), flush=True)


def test_batch_pixels_per_lane_keep_results(sp):
    """The 512 x 640 slice gives the batch 1,280 four-pixel R^T tiles (5,120
    waves, over 16 per CU on 256 CUs), so the whole batch takes four pixels per
    lane; the 64 x 64 slice alone has 16 such tiles and takes two. R^T's
    dot-product partials are per 8 x 16 sub-tile in one order whatever the
    pixels per lane, so the small slice must still match its own solve bit for
    bit (and the large one, four pixels per lane on both sides, too)."""
    from synth import random_ellipses
    # plus two ragged slices: 522 x 520 (partial four-pixel tiles on the right
    # and at the bottom, four pixels per lane alone too) and 37 x 53 (two
    # alone, four in the batch)
    geoms = [sp.Geometry(512, 640, 180, 900), sp.Geometry(64, 64, 90, 91),
             sp.Geometry(522, 520, 90, 741), sp.Geometry(37, 53, 45, 61)]
    bs = []
    for i, g in enumerate(geoms):
        img, rng = random_ellipses(g.rows, g.cols, 5, 700 + i)
        b = sp.sp_project(g, torch.from_numpy(img.astype(np.float32)).cuda())
        noise = torch.from_numpy(rng.standard_normal(g.m).astype(np.float32)).cuda()
        bs.append((b + 0.01 * float(b.max()) * noise.reshape(b.shape)).contiguous())
    kw = dict(K=K, a=A, gamma=GAMMA, mu=MU, rho=RHO, max_iter=6)
    got = sp.sp_suppcg_solve_batched(geoms, bs, graph=False, autotune=False, **kw)
    want = singles(sp, geoms, bs, **kw)
    for i, (rb, rs) in enumerate(zip(got, want)):
        print(f"slice {i}: k {rb.k} status {rb.status_name}", flush=True)
        assert_same(rb, rs)


def test_batch_cg_start_and_halting(sp):
    # M = I, K = 2, a nonzero start on some slices and an all-zero data slice
    # that breaks down at once while the others run on
    geoms, bs = mixed_batch(sp)
    bs[2] = torch.zeros_like(bs[2])
    x0s = [None] * len(geoms)
    x0s[1] = torch.full((geoms[1].rows, geoms[1].cols), 0.25, device="cuda")
    x0s[4] = torch.rand((geoms[4].rows, geoms[4].cols), device="cuda")
    kw = dict(K=2, a=A, gamma=GAMMA, precond="none", max_iter=9)
    got = sp.sp_suppcg_solve_batched(geoms, bs, x0s, graph=True, **kw)
    want = singles(sp, geoms, bs, x0s, **kw)
    assert got[2].status_name.startswith("breakdown") and got[2].k == 1
    for rb, rs in zip(got, want):
        assert_same(rb, rs)


@pytest.mark.parametrize("K", [3, 4, 5])
def test_batch_inner_steps_match_single(sp, K):
    # several S_TV inner steps per body: the single-slice solver applies each
    # step and forms the next t_bar in one launch, alternating two iterate
    # buffers (odd and even K end on either), while the batched solver keeps
    # separate launches; both must give the same bits (a = 0.7 and gamma = 3
    # reject trials in the early bodies)
    geoms, bs = mixed_batch(sp)
    kw = dict(K=K, a=0.7, gamma=3.0, mu=MU, rho=RHO, max_iter=6)
    print(f"K {K}", flush=True)
    got = sp.sp_suppcg_solve_batched(geoms, bs, graph=True, **kw)
    want = singles(sp, geoms, bs, graph=True, **kw)
    for rb, rs in zip(got, want):
        assert_same(rb, rs)


def test_batch_inner_steps_match_single_large_slice(sp):
    # from 2^18 pixels up the t_bar launches after an S_TV call's first inner
    # step and the trials take four pixels per thread, in the single solver's
    # fused update-and-t_bar kernel as in the batched t_bar kernel: a 512^2
    # slice next to a small one, K = 3 with rejected trials, bit for bit
    from synth import random_ellipses
    geoms = [sp.Geometry(512, 512, 720, 725), sp.Geometry(64, 64, 90, 91)]
    bs = []
    for i, g in enumerate(geoms):
        img, rng = random_ellipses(g.rows, g.cols, 8, 400 + i)
        b = sp.sp_project(g, torch.from_numpy(img.astype(np.float32)).cuda())
        noise = torch.from_numpy(rng.standard_normal(g.m).astype(np.float32)).cuda()
        bs.append((b + 0.01 * float(b.max()) * noise.reshape(b.shape)).contiguous())
    kw = dict(K=3, a=0.5, gamma=300.0, mu=MU, rho=RHO, max_iter=4)
    got = sp.sp_suppcg_solve_batched(geoms, bs, graph=True, **kw)
    want = singles(sp, geoms, bs, graph=True, **kw)
    for rb, rs in zip(got, want):
        print(f"k {rb.k}, ell {list(rb.trace['ell'])}", flush=True)
        assert_same(rb, rs)
        assert int(rb.trace["ell"][-1]) > 3 * 4   # trials were rejected


def test_batch_slice_matches_oracle(sp):
    # the 64 x 64 workload inside a mixed batch, 20 iterations, against the
    # float64 oracle (same bar as the single-slice solver)
    og, img, b = workload_problem("small64")
    R, _ = oproj.matrix(og)
    prob = osup.Problem(R, b.astype(np.float64), (og.rows, og.cols), oracle_precond)
    ref = osup.suppcg(prob, np.zeros(og.n), osup.TVParams(K, A, GAMMA), n_iter=20)
    geoms, bs = mixed_batch(sp)
    bs[0] = torch.from_numpy(np.ascontiguousarray(b, dtype=np.float32)).cuda()
    got = sp.sp_suppcg_solve_batched(geoms, bs, K=K, a=A, gamma=GAMMA, mu=MU, rho=RHO, max_iter=20)
    assert got[0].k == ref.k == 21
    assert list(got[0].trace["ell"]) == ref.trace["ell"]
    assert rel_l2(got[0].x_half.cpu().numpy(), ref.x_half) <= 1e-3


def test_batch_eps_termination(sp):
    geoms, bs = mixed_batch(sp)
    kw = dict(K=K, a=A, gamma=GAMMA, mu=MU, rho=RHO, max_iter=60)
    free = sp.sp_suppcg_solve_batched(geoms, bs, **kw)
    # each slice stops at its own level: 1.05 x its f after 10 bodies
    eps = min(float(r.trace["f_half"][9]) for r in free) * 1.05
    got = sp.sp_suppcg_solve_batched(geoms, bs, eps=eps, **kw)
    want = singles(sp, geoms, bs, eps=eps, graph=True, **kw)
    for rb, rs in zip(got, want):
        assert_same(rb, rs)
    assert any(r.status_name == "converged" for r in got)


def test_batch_eps_matches_oracle(sp):
    # slice 0 = the 64 x 64 workload; its eps stop (at body 7, and at x_0)
    # against the oracle, x_last included
    og, img, b = workload_problem("small64")
    R, _ = oproj.matrix(og)
    prob = osup.Problem(R, b.astype(np.float64), (og.rows, og.cols), oracle_precond)
    tvp = osup.TVParams(K, A, GAMMA)
    free = osup.suppcg(prob, np.zeros(og.n), tvp, n_iter=10)
    geoms, bs = mixed_batch(sp)
    bs[0] = torch.from_numpy(np.ascontiguousarray(b, dtype=np.float32)).cuda()
    for eps in (0.5 * (free.trace["f_half"][5] + free.trace["f_half"][6]), 2.0 * free.trace["f0"]):
        ref = osup.suppcg(prob, np.zeros(og.n), tvp, n_iter=40, eps=eps)
        got = sp.sp_suppcg_solve_batched(geoms, bs, K=K, a=A, gamma=GAMMA, mu=MU, rho=RHO,
                                         max_iter=40, eps=eps)
        assert ref.status == "converged" and got[0].status_name == "converged"
        assert got[0].k == ref.k
        assert rel_l2(got[0].x_last.cpu().numpy(), ref.x_last) <= 1e-3
        if ref.k > 1:
            assert rel_l2(got[0].x_half.cpu().numpy(), ref.x_half) <= 1e-3


def test_batch_rejects_unsupported(sp):
    geoms, bs = mixed_batch(sp)
    with pytest.raises(sp.SupPCGError) as e:
        sp.sp_suppcg_solve_batched(geoms, bs, precond="learned", max_iter=2)
    assert e.value.code == 1
    bad = list(geoms)
    bad[3] = sp.Geometry(100, 70, 45, 123, bin_spacing=0.1)
    with pytest.raises(sp.SupPCGError) as e:
        sp.sp_suppcg_solve_batched(bad, bs, max_iter=2)
    assert e.value.code == 1 and "slice 3" in str(e.value)


def test_batch_64_mixed_slices_sampled(sp):
    # The 64-slice batch: sides from {256, 384, 512, 768, 1024}, 1.4 x side
    # angles (multiple of 8), ceil(side sqrt 2) + 1 bins, 20-ellipse phantoms,
    # noise 0.2%-2%; 50 iterations in one batched solve.  One slice of each
    # side is re-solved alone and must agree bit for bit.  R splits the rays
    # of the 256^2 slices in 4 parts and of the 384^2 slices in 2 (their grids
    # alone would not fill the GPU); larger slices run whole rays.
    from synth import batched_slices, random_ellipses
    work = batched_slices(64, seed=2)
    geoms = [sp.Geometry(w.rows, w.cols, w.n_angles, w.n_bins) for w in work]
    bs = []
    for w, g in zip(work, geoms):
        img, rng = random_ellipses(w.rows, w.cols, w.n_ellipses, w.seed)
        x = torch.from_numpy(img.astype(np.float32)).cuda()
        b = sp.sp_project(g, x)
        noise = torch.from_numpy(rng.standard_normal(g.m).astype(np.float32)).cuda()
        bs.append((b + w.noise_frac * float(b.max()) * noise.reshape(b.shape)).contiguous())
    kw = dict(K=1, a=0.5, gamma=0.5, mu=MU, rho=RHO, max_iter=50)
    got = sp.sp_suppcg_solve_batched(geoms, bs, graph=True, autotune=True, **kw)
    print("tuning:", sp.batch_tuning(), flush=True)
    picked = {}
    for i, w in enumerate(work):
        picked.setdefault(w.rows, i)
    for side, i in sorted(picked.items()):
        rs = sp.sp_suppcg_solve(geoms[i], bs[i], None, graph=True, **kw)
        print(f"slice {i} ({side}^2, {geoms[i].n_angles} angles): k {got[i].k}", flush=True)
        assert_same(got[i], rs)
    for r in got:
        assert r.k == 51 and np.all(np.isfinite(r.trace["f_half"]))
