"""GPU parity of the learned preconditioner against the float64 oracle."""
import numpy as np
import pytest

from oracle import learned as ol
from oracle import projector as oproj
from oracle import suppcg as osup
from tests._problems import A, GAMMA, K, MU, RHO, rel_l2, workload_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1807_10151_amd as sp_mod
    return sp_mod


def cuda(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def params(seed, layers=4, scale_d=0.5):
    Ws, d = ol.init_params(layers, 16, seed)
    rng = np.random.default_rng(seed + 100)
    d = d + scale_d * rng.standard_normal(16)
    return Ws, d


@pytest.mark.parametrize("shape,layers", [((3, 37, 53), 4), ((2, 16, 16), 2), ((1, 64, 64), 4),
                                          ((2, 5, 70), 1)])
def test_apply_matches_oracle(sp, shape, layers):
    Ws, d = params(1, layers)
    net = sp.LearnedPrecond(layers)
    theta = ol.flatten(Ws, d)
    net.set_params(theta)
    np.testing.assert_array_equal(net.get_params(), theta.astype(np.float32))
    u = np.random.default_rng(2).standard_normal(shape).astype(np.float32)
    Ws32, d32 = ol.unflatten(theta.astype(np.float32).astype(np.float64), layers, 16)
    want = ol.apply(Ws32, d32, u.astype(np.float64))
    got = net.apply(cuda(u)).cpu().numpy()
    assert rel_l2(got, want) <= 1e-5, rel_l2(got, want)


@pytest.mark.parametrize("margin", [0, 8])
def test_loss_grad_matches_oracle(sp, margin):
    Ws, d = params(3)
    theta = ol.flatten(Ws, d).astype(np.float32).astype(np.float64)
    Ws, d = ol.unflatten(theta, 4, 16)
    rng = np.random.default_rng(4)
    Av = rng.standard_normal((6, 24, 40)).astype(np.float32)
    v = rng.standard_normal((6, 24, 40)).astype(np.float32)
    idx = np.array([5, 0, 3, 3], dtype=np.int32)
    loss, gW, gd = ol.loss_and_grad(Ws, d, Av[idx].astype(np.float64), v[idx].astype(np.float64),
                                    margin=margin)
    net = sp.LearnedPrecond(4)
    net.set_params(theta)
    gl, gg = net.loss_grad(cuda(Av), cuda(v), cuda(idx, np.int32), margin=margin)
    assert float(gl.item()) == pytest.approx(loss, rel=1e-5)
    want = ol.flatten(gW, gd)
    got = gg.cpu().numpy().astype(np.float64)
    assert rel_l2(got, want) <= 1e-4, rel_l2(got, want)
    off = 0
    for W in gW:                                   # every layer, not just the largest
        sz = W.size
        assert rel_l2(got[off:off + sz], W.ravel()) <= 1e-4
        off += sz
    assert rel_l2(got[off:], gd) <= 1e-4


def test_adam_step_matches_oracle(sp):
    Ws, d = params(5)
    theta = ol.flatten(Ws, d).astype(np.float32)
    g = np.random.default_rng(6).standard_normal(theta.size).astype(np.float32)
    net = sp.LearnedPrecond(4)
    net.set_params(theta)
    opt = ol.Adam([theta.astype(np.float64)], lr=1e-3)
    want = theta.astype(np.float64)
    gt = cuda(g)
    for step in (1, 2, 3):
        net.adam_step(gt, 1e-3, step)
        want = opt.step([want], [g.astype(np.float64)])[0]
    assert rel_l2(net.get_params(), want) <= 1e-6


@pytest.fixture(scope="module")
def small():
    og, img, b = workload_problem("small64")
    R, _ = oproj.matrix(og)
    return og, img, b, R


def test_solver_with_learned_matches_oracle(sp, small):
    og, img, b, R = small
    Ws, d = params(7)
    theta = ol.flatten(Ws, d).astype(np.float32).astype(np.float64)
    Ws, d = ol.unflatten(theta, 4, 16)
    prob = osup.Problem(R, b.astype(np.float64), (og.rows, og.cols), lambda v: ol.apply(Ws, d, v))
    ref = osup.suppcg(prob, np.zeros(og.n), osup.TVParams(K, A, GAMMA), n_iter=10)
    net = sp.LearnedPrecond(4)
    net.set_params(theta)
    g = sp.Geometry(og.rows, og.cols, og.n_angles, og.n_bins)
    res = sp.sp_suppcg_solve(g, cuda(b), None, K=K, a=A, gamma=GAMMA, precond="learned", net=net,
                             mu=MU, rho=RHO, max_iter=10)
    assert res.trace["fallbacks"] == 0
    assert list(res.trace["ell"]) == ref.trace["ell"]
    assert rel_l2(res.x_half.cpu().numpy(), ref.x_half) <= 1e-3


@pytest.mark.parametrize("bad", ["nan", "zero"])
def test_solver_falls_back_to_fourier_preconditioner(sp, small, bad):
    og, img, b, R = small
    net = sp.LearnedPrecond(4)
    theta = np.full(net.num_params, np.nan if bad == "nan" else 0.0, dtype=np.float32)
    net.set_params(theta)
    g = sp.Geometry(og.rows, og.cols, og.n_angles, og.n_bins)
    kw = dict(K=K, a=A, gamma=GAMMA, mu=MU, rho=RHO, max_iter=8)
    res = sp.sp_suppcg_solve(g, cuda(b), None, precond="learned", net=net, **kw)
    ref = sp.sp_suppcg_solve(g, cuda(b), None, precond="ramp", **kw)
    assert res.trace["fallbacks"] == 1
    assert list(res.trace["ell"]) == list(ref.trace["ell"])
    assert rel_l2(res.x_half.cpu().numpy(), ref.x_half.cpu().numpy()) <= 1e-6


def test_training_gain(sp):
    # The recipe's 2000 Adam steps on 2048 Gaussian + 2048 Krylov probes at the
    # 64x64 / 90-angle geometry.  The trained network must (1) lower the loss
    # from its scaled start by 2x, and (2) reach the plain run's f(x_{100+1/2})
    # in at most half the loop bodies that the untrained network and M = I
    # need.  The paper's Fourier M is printed beside it for the record: this
    # loss does not beat it here (about 112 against 100 bodies).
    from paper_1807_10151_amd import learned_train as lt
    g = sp.Geometry(64, 64, 90, 91)
    cfg = lt.TrainConfig()
    res = lt.train(g, cfg, log_every=500)
    first, last = res.losses[0][1], res.losses[-1][1]
    print(f"loss {first:.4f} -> {last:.4f}; train {res.seconds:.2f} s", flush=True)
    assert last <= 0.5 * first
    net0 = sp.LearnedPrecond(4)
    th = lt.init_theta(4, 16, cfg.seed)
    net0.set_params(th)
    lt.scale_init(net0, th, res.extra["V"], res.extra["AV"], 16)
    seeds = [100, 101, 102, 103]
    trained = lt.time_to_target(g, res.net, seeds, cfg, max_iters=400, reps=0)
    untrained = lt.time_to_target(g, net0, seeds, cfg, max_iters=400, reps=0)
    kw = dict(K=cfg.K, a=cfg.a, gamma=cfg.gamma, mu=cfg.mu, rho=cfg.rho, graph=True)
    for r_t, r_u in zip(trained, untrained):
        _, b = lt.phantom_data(g, r_t["seed"], cfg.n_ellipses, cfg.noise)
        plain_cg = sp.sp_suppcg_solve(g, b, None, precond="none", max_iter=400, **kw)
        hit = np.nonzero(plain_cg.trace["f_half"] <= r_t["f_star"])[0]
        k_cg = int(hit[0]) + 1 if hit.size else 10 ** 6
        k_u = r_u["k_f"] or 10 ** 6
        print(f"seed {r_t['seed']}: bodies to f*: trained {r_t['k_f']}, untrained {r_u['k_f']}, "
              f"M=I {k_cg}, Fourier M 100", flush=True)
        assert r_t["fallbacks"] == 0
        assert r_t["k_f"] is not None and 2 * r_t["k_f"] <= min(k_u, k_cg)
