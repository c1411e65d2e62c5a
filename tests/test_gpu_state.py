"""Checkpoint / resume of Algorithm 3's carried state, and asynchronous solves.

A run of N loop bodies must equal, bit for bit, a run of N1 bodies whose state
is saved, loaded (into the same or a fresh context) and resumed for N - N1
more, in eager and in graph mode; the resumed run's trace continues the
straight run's trace."""
import numpy as np
import pytest

from tests._problems import A, GAMMA, K, MU, RHO, workload_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1807_10151_amd as sp_mod
    return sp_mod


@pytest.fixture(scope="module")
def prob(sp):
    og, img, b = workload_problem("small64")
    g = sp.Geometry(og.rows, og.cols, og.n_angles, og.n_bins)
    return g, torch.from_numpy(np.ascontiguousarray(b)).cuda()


KW = dict(K=2, a=0.7, gamma=3.0, mu=MU, rho=RHO)   # rejections in early bodies


@pytest.mark.parametrize("graph", [False, True])
def test_save_load_resume_equals_straight_run(sp, prob, graph):
    g, b = prob
    straight = sp.sp_suppcg_solve(g, b, None, max_iter=20, graph=graph, **KW)
    first = sp.sp_suppcg_solve(g, b, None, max_iter=10, graph=graph, **KW)
    blob = sp.sp_state_save()
    # something else runs on the context in between (operators do not touch the state)
    sp.sp_tv_perturb(g, first.x_half, 0, 1, 0.5, 0.5)
    sp.sp_project(g, first.x_half)
    other = sp.sp_suppcg_solve(g, b, None, max_iter=3, graph=graph, K=1, a=0.5, gamma=0.5, mu=MU,
                               rho=RHO)
    assert other.k == 4
    sp.sp_state_load(blob)
    rest = sp.sp_suppcg_solve(g, b, None, max_iter=10, graph=graph, resume=True, **KW)
    assert rest.k == straight.k == 21
    assert torch.equal(rest.x_half, straight.x_half) and torch.equal(rest.x_last, straight.x_last)
    for key in ("f_half", "tv_half", "alpha", "beta", "s_norm", "ell"):
        both = np.concatenate([first.trace[key], rest.trace[key]])
        assert np.array_equal(both, straight.trace[key]), key
    assert np.array_equal(np.concatenate([first.trace["trials"], rest.trace["trials"]]),
                          straight.trace["trials"])
    # resuming directly (no save/load) continues the same way
    sp.sp_suppcg_solve(g, b, None, max_iter=10, graph=graph, **KW)
    rest2 = sp.sp_suppcg_solve(g, b, None, max_iter=10, graph=graph, resume=True, **KW)
    assert torch.equal(rest2.x_half, straight.x_half)


def test_state_moves_to_a_fresh_context(sp, prob):
    g, b = prob
    straight = sp.sp_suppcg_solve(g, b, None, max_iter=12, **KW)
    sp.sp_suppcg_solve(g, b, None, max_iter=5, **KW)
    blob = sp.sp_state_save()
    ctx2 = sp.Context(0)
    try:
        sp.sp_state_load(blob, ctx=ctx2)
        rest = sp.sp_suppcg_solve(g, b, None, max_iter=7, resume=True, ctx=ctx2, **KW)
        assert rest.k == 13 and torch.equal(rest.x_half, straight.x_half)
    finally:
        ctx2.close()


def test_resume_rejects_mismatch(sp, prob):
    g, b = prob
    sp.sp_suppcg_solve(g, b, None, max_iter=3, **KW)
    bad = dict(KW, gamma=2.0)
    with pytest.raises(sp.SupPCGError) as e:
        sp.sp_suppcg_solve(g, b, None, max_iter=3, resume=True, **bad)
    assert e.value.code == 1
    g2 = sp.Geometry(64, 64, 90, 93)
    with pytest.raises(sp.SupPCGError):
        sp.sp_suppcg_solve(g2, torch.zeros((90, 93), device="cuda"), None, max_iter=3, resume=True,
                           **KW)
    ctx2 = sp.Context(0)
    try:
        with pytest.raises(sp.SupPCGError):
            sp.sp_state_save(ctx=ctx2)                     # nothing solved there yet
        with pytest.raises(sp.SupPCGError):
            sp.sp_state_load(b"not a state blob" * 40, ctx=ctx2)
    finally:
        ctx2.close()


def test_resume_after_eps_stop(sp, prob):
    # a run stopped by the eps test continues when resumed with a smaller eps
    g, b = prob
    free = sp.sp_suppcg_solve(g, b, None, max_iter=30, **KW)
    f = free.trace["f_half"]
    first = sp.sp_suppcg_solve(g, b, None, max_iter=30, eps=0.5 * (f[7] + f[8]), **KW)
    assert first.status_name == "converged" and first.k == 10
    rest = sp.sp_suppcg_solve(g, b, None, max_iter=21, resume=True, **KW)
    assert rest.k == 31 and torch.equal(rest.x_half, free.x_half)


@pytest.mark.parametrize("graph", [False, True])
def test_async_solve(sp, prob, graph):
    g, b = prob
    ref = sp.sp_suppcg_solve(g, b, None, max_iter=15, graph=graph, **KW)
    k, xh, xl = sp.sp_suppcg_solve_async(g, b, None, max_iter=15, graph=graph, **KW)
    torch.cuda.synchronize()
    assert int(k.item()) == ref.k == 16
    assert torch.equal(xh, ref.x_half) and torch.equal(xl, ref.x_last)
    ks, st = sp.sp_solve_status(1)
    assert ks == [16] and st == [16]           # SP_MAXITER
    # with eps: the bodies after the stop are enqueued and do nothing
    f = ref.trace["f_half"]
    eps = 0.5 * (f[4] + f[5])
    ref_e = sp.sp_suppcg_solve(g, b, None, max_iter=15, eps=eps, graph=graph, **KW)
    k, xh, xl = sp.sp_suppcg_solve_async(g, b, None, max_iter=15, eps=eps, graph=graph, **KW)
    ks, st = sp.sp_solve_status(1)
    assert ks == [ref_e.k] and st == [17]      # SP_CONVERGED
    assert int(k.item()) == ref_e.k
    assert torch.equal(xh, ref_e.x_half) and torch.equal(xl, ref_e.x_last)


def test_async_batched(sp, prob):
    g, b = prob
    g2 = sp.Geometry(48, 80, 60, 97)
    from synth import random_ellipses
    img, _ = random_ellipses(48, 80, 5, 11)
    b2 = sp.sp_project(g2, torch.from_numpy(img.astype(np.float32)).cuda()).contiguous()
    ref = sp.sp_suppcg_solve_batched([g, g2], [b, b2], max_iter=9, **KW)
    import ctypes
    from paper_1807_10151_amd import _lib as L
    from paper_1807_10151_amd.api import _precond, context
    ctx = context(0)
    k = torch.zeros(2, dtype=torch.int32, device="cuda")
    xh = [torch.empty((gg.rows, gg.cols), device="cuda") for gg in (g, g2)]
    garr = (L.sp_geometry * 2)(g.c(), g2.c())
    vp = lambda ts: (ctypes.c_void_p * 2)(*[t.data_ptr() for t in ts])
    tvp = L.sp_tv_params(KW["K"], KW["a"], KW["gamma"], 100)
    pc = _precond("ramp", MU, RHO)
    spp = L.sp_solve_params(0.0, 9, L.SP_FLAG_ASYNC | L.SP_FLAG_GRAPH, None)
    ctx._stream()
    rc = ctx.lib.sp_suppcg_solve_batched(ctx.h, 2, garr, vp([b, b2]), None, ctypes.byref(tvp),
                                         ctypes.byref(pc), ctypes.byref(spp), vp(xh), None,
                                         ctypes.cast(ctypes.c_void_p(k.data_ptr()),
                                                     ctypes.POINTER(ctypes.c_int32)), None)
    assert rc == L.SP_OK
    ks, st = sp.sp_solve_status(2)
    assert ks == [10, 10] and st == [16, 16]
    assert k.cpu().tolist() == [10, 10]
    for i in range(2):
        assert torch.equal(xh[i], ref[i].x_half)


def test_rejected_call_keeps_the_state(sp, prob):
    # a solve rejected for its trace options (ellipse semi-axes) must leave the
    # carried state resumable
    g, b = prob
    straight = sp.sp_suppcg_solve(g, b, None, max_iter=8, **KW)
    sp.sp_suppcg_solve(g, b, None, max_iter=4, **KW)
    ref = torch.ones((g.rows, g.cols), device="cuda")
    with pytest.raises(sp.SupPCGError):
        sp.sp_suppcg_solve(g, b, None, max_iter=4, resume=True, se_ref=ref, se_axes=(0.0, 3.0), **KW)
    rest = sp.sp_suppcg_solve(g, b, None, max_iter=4, resume=True, **KW)
    assert torch.equal(rest.x_half, straight.x_half)


def _blob_vectors(blob, n, m):
    # layout after the header: x_k, x_{k-1/2}, p_{k-1} (n float64 each), then
    # q = R p_{k-1} (m float64)
    head = len(blob) - 3 * n * 8 - m * 8
    v = np.frombuffer(blob, dtype=np.float64, offset=head)
    return v[2 * n:3 * n], v[3 * n:3 * n + m]


@pytest.mark.parametrize("kw,bodies", [(dict(K=1, a=A, gamma=GAMMA, mu=MU, rho=RHO), 60),
                                       (dict(KW), 40),
                                       (dict(K=0, precond="none"), 30)])
def test_carried_ray_vector_is_projection_of_direction(sp, prob, kw, bodies):
    # the solver keeps Algorithm 2's h = R^T R p through q = R p, updated by
    # the direction's recurrence; after many bodies q must still be the
    # projection of the saved direction p (float64 R of the oracle), with no
    # drift beyond rounding
    from oracle import projector as oproj
    og, _, _ = workload_problem("small64")
    g, b = prob
    res = sp.sp_suppcg_solve(g, b, None, max_iter=bodies, graph=True, **kw)
    assert res.k == bodies + 1
    p, q = _blob_vectors(sp.sp_state_save(), og.n, og.m)
    R, _ = oproj.matrix(og)
    rp = R @ p
    err = np.linalg.norm(q - rp) / np.linalg.norm(rp)
    print(f"{kw}: ||q - R p|| / ||R p|| = {err:.2e} after {bodies} bodies", flush=True)
    assert err <= 1e-9


def test_state_blob_size(sp, prob):
    og, _, _ = workload_problem("small64")
    g, b = prob
    sp.sp_suppcg_solve(g, b, None, max_iter=2, **KW)
    blob = sp.sp_state_save()
    head = len(blob) - 3 * og.n * 8 - og.m * 8
    assert 0 < head < 4096 and head % 8 == 0
