"""Pins of the oracle's Algorithms 1-3 (CPU only): the paper's theorems, dense
least squares, conjugacy, scale invariance and the SupTPCG equivalence."""
import math

import numpy as np
import pytest

from oracle import precond, projector, suppcg, suptpcg, tv
from oracle.geometry import Geometry
from synth import noisy_data, random_ellipses, unit_noise


def tiny_problem(seed=0, shape=(8, 8), A=16, B=13, frac=0.01, mu=1e-3, rho=0.7, M=True):
    g = Geometry(shape[0], shape[1], A, B)
    R, _ = projector.matrix(g, "siddon")
    img, rng = random_ellipses(shape[0], shape[1], 3, seed)
    b = noisy_data(R @ img.ravel(), unit_noise(rng, g.m), frac)
    pre = (lambda v: precond.apply(v, mu, rho)) if M else None
    return g, R, b, suppcg.Problem(R, b, shape, pre)


def test_pcg_reaches_dense_least_squares():
    # P14: K = 0 on a full-rank tiny system reaches numpy.linalg.lstsq
    g, R, b, prob = tiny_problem()
    Rd = R.toarray()
    assert np.linalg.matrix_rank(Rd) == g.n
    xls = np.linalg.lstsq(Rd, b, rcond=None)[0]
    res = suppcg.suppcg(prob, np.zeros(g.n), None, n_iter=g.n + 5)
    assert np.linalg.norm(res.x_last - xls) <= 1e-8 * np.linalg.norm(xls)


def test_cg_identity_preconditioner_reaches_least_squares():
    g, R, b, prob = tiny_problem(M=False)
    xls = np.linalg.lstsq(R.toarray(), b, rcond=None)[0]
    res = suppcg.suppcg(prob, np.zeros(g.n), None, n_iter=3 * g.n)
    assert np.linalg.norm(res.x_last - xls) <= 1e-7 * np.linalg.norm(xls)


def test_pcg_monotone_and_conjugate():
    # P15: f(x_k) non-increasing; p_k^T h_{k-1} = 0 and p_k^T A p_{k-1} = 0
    g, R, b, prob = tiny_problem(seed=3)
    res = suppcg.suppcg(prob, np.zeros(g.n), None, n_iter=30, record_vectors=True)
    f = [prob.f(x) for x in res.trace["x"]]
    assert all(f[i + 1] <= f[i] * (1 + 1e-12) + 1e-14 for i in range(len(f) - 1))
    ps, hs = res.trace["p"], res.trace["h"]
    for k in range(1, 20):
        scale = np.linalg.norm(ps[k]) * np.linalg.norm(hs[k - 1])
        assert abs(ps[k] @ hs[k - 1]) <= 1e-10 * scale
    # the residual f at x_{k+1/2} recorded by the loop equals f recomputed
    for k in range(5):
        assert res.trace["f_half"][k] == pytest.approx(prob.f(res.trace["x_half_v"][k + 1]), rel=1e-12)


def test_preconditioner_scale_invariance():
    # P16 / A7: M -> c M leaves every iterate unchanged (including the TV perturbation)
    g, R, b, prob = tiny_problem(seed=4)
    tvp = suppcg.TVParams(K=2, a=0.5, gamma=0.5)
    prob2 = suppcg.Problem(R, b, (8, 8), lambda v: 37.0 * precond.apply(v, 1e-3, 0.7))
    r1 = suppcg.suppcg(prob, np.zeros(g.n), tvp, n_iter=8)
    r2 = suppcg.suppcg(prob2, np.zeros(g.n), tvp, n_iter=8)
    assert r1.trace["ell"] == r2.trace["ell"]
    assert np.linalg.norm(r1.x_half - r2.x_half) <= 1e-10 * np.linalg.norm(r1.x_half)


def test_theorem1_bound_and_tv_monotone():
    # P13: ||s_k|| <= K gamma a^{(k-1)K}, l_k >= (k-1)K, TV(x_{k+1/2}) <= TV(x_k)
    g, R, b, prob = tiny_problem(seed=5, shape=(12, 12), A=20, B=19)
    for K, a, gam in ((1, 0.5, 0.5), (3, 0.8, 0.3), (2, 0.99, 0.05)):
        tvp = suppcg.TVParams(K=K, a=a, gamma=gam)
        res = suppcg.suppcg(prob, np.zeros(g.n), tvp, n_iter=15, record_vectors=True)
        for k in range(1, 16):
            s_norm = res.trace["s_norm"][k - 1]
            assert s_norm <= K * gam * a ** ((k - 1) * K) * (1 + 1e-12)
            ell_k = 0 if k == 1 else res.trace["ell"][k - 2]
            assert ell_k >= (k - 1) * K
            xk = res.trace["x"][k - 1].reshape(12, 12)
            assert res.trace["tv_half"][k - 1] <= tv.total_variation(xk) * (1 + 1e-15)


def test_s_tv_constant_image():
    out = suppcg.s_tv(np.full((6, 6), 1.5), 7, suppcg.TVParams(K=4, a=0.5, gamma=1.0))
    assert not out.s.any() and out.ell == 11 and out.trials == [1, 1, 1, 1]


def test_s_tv_trial_cap_and_replay():
    # A9: an unacceptable schedule exhausts the cap, keeps l's increments, leaves y
    rng = np.random.default_rng(2)
    x = rng.standard_normal((8, 8))
    out = suppcg.s_tv(x, 0, suppcg.TVParams(K=1, a=1 - 1e-12, gamma=1e6, max_trials=5))
    assert out.exhausted and out.ell == 5 and not out.s.any() and out.trials == [6]
    p = suppcg.TVParams(K=3, a=0.5, gamma=4.0)
    free = suppcg.s_tv(x, 0, p)
    rep = suppcg.s_tv(x, 0, p, replay=free.trials)
    assert rep.ell == free.ell and np.array_equal(rep.s, free.s)


def test_suppcg_equals_suptpcg():
    # P17, Table 2: x_k = N^T x_hat_k with N = M^{1/2}
    g, R, b, prob = tiny_problem(seed=6, shape=(6, 6), A=12, B=11)
    Md = precond.dense(6, 6, 1e-3, 0.7)
    N = suptpcg.sqrt_spd(Md)
    tvp = suppcg.TVParams(K=2, a=0.6, gamma=0.4)
    x0 = np.random.default_rng(1).standard_normal(g.n) * 0.1
    res = suppcg.suppcg(prob, x0, tvp, n_iter=10, record_vectors=True)
    k, hist = suptpcg.suptpcg(R.toarray(), b, N, (6, 6), np.linalg.solve(N.T, x0), tvp, n_iter=10)
    assert k == res.k
    for i in range(11):
        xs = N.T @ hist["x"][i]
        assert np.linalg.norm(xs - res.trace["x"][i]) <= 1e-10 * np.linalg.norm(res.trace["x"][i])
        ps = N.T @ hist["p"][i]
        assert np.linalg.norm(ps - res.trace["p"][i]) <= 1e-10 * np.linalg.norm(res.trace["p"][i])
    assert hist["ell"][1:] == res.trace["ell"]


def test_theorem2_termination():
    # P18: for eps > eps0 = min ||Rx - b||^2 the loop stops
    g, R, b, prob = tiny_problem(seed=7, frac=0.05)
    xls = np.linalg.lstsq(R.toarray(), b, rcond=None)[0]
    eps0 = float(np.sum((R @ xls - b) ** 2))
    tvp = suppcg.TVParams(K=2, a=0.7, gamma=0.5)
    res = suppcg.suppcg(prob, np.zeros(g.n), tvp, n_iter=10_000, eps=(1 + 1e-3) * eps0)
    assert res.status == "converged"
    assert prob.f(res.x_half) <= (1 + 1e-3) * eps0
    assert res.k < 10_000


def test_breakdown_on_zero_data():
    # A13: b = 0 and x0 = 0 give g0 = p0 = 0, so p^T h = 0
    g, R, b, _ = tiny_problem()
    prob = suppcg.Problem(R, np.zeros(g.m), (8, 8), lambda v: precond.apply(v, 1e-3, 0.7))
    res = suppcg.suppcg(prob, np.zeros(g.n), suppcg.TVParams(1, 0.5, 0.5), n_iter=5)
    assert res.status == "breakdown" and res.k == 1


# ---- Algorithm 1's exact step schedule on an image whose TV along t is known ----
#
# A lone interior spike of height h on a zero background: minus the TV gradient
# is nonzero only at the spike (each neighbour also enters a flat square-root
# term, so the zero rule of Section 3.1 removes it), where it equals -(2 + sqrt 2)
# times sign(h).  Hence t = -sign(h) e_spike and TV(y + lam t) = (2 + sqrt 2) |h -
# lam sign(h)|: trial step lam is accepted iff lam <= 2 |h| (equality included).
# Algorithm 1 forms gamma a^l BEFORE incrementing l, so the j-th trial of an
# inner step entered with l0 has length gamma a^(l0 + j - 1) and leaves l = l0 + j.

def _spike(h, shape=(6, 7), at=(2, 3)):
    y = np.zeros(shape)
    y[at] = h
    return y


def _first_accepted(l0, gamma, a, h):
    j = 1
    while gamma * a ** (l0 + j - 1) > 2 * abs(h):
        j += 1
    return j


@pytest.mark.parametrize("l0,gamma,a,h,want_j", [
    (0, 1.0, 0.5, 0.1, 4),       # 1, 1/2, 1/4 rejected; 1/8 <= 0.2 accepted
    (3, 1.0, 0.5, 0.1, 1),       # first trial 1/8
    (0, 20.0, 0.5, 0.3, 7),      # 20 .. 0.625 rejected, 0.3125 accepted
    (2, 3.0, 0.9, 0.05, 32),
])
def test_s_tv_step_schedule_on_spike(l0, gamma, a, h, want_j):
    assert _first_accepted(l0, gamma, a, h) == want_j
    y = _spike(h)
    out = suppcg.s_tv(y, l0, suppcg.TVParams(K=1, a=a, gamma=gamma))
    lam = gamma * a ** (l0 + want_j - 1)
    assert out.trials == [want_j] and out.ell == l0 + want_j and not out.exhausted
    want_s = np.zeros_like(y)
    want_s[2, 3] = -lam
    assert np.array_equal(out.s, want_s)
    assert np.sqrt(np.sum(out.s ** 2)) == lam
    assert out.tv_after == pytest.approx((2 + math.sqrt(2)) * abs(h - lam), rel=1e-14)


def test_s_tv_tie_accepts_and_inner_steps_carry_l():
    # lam = 2h exactly: TV(y + lam t) == TV(y) bit for bit, and "<=" accepts
    out = suppcg.s_tv(_spike(0.25), 0, suppcg.TVParams(K=1, a=0.5, gamma=1.0))
    assert out.trials == [2] and out.ell == 2 and out.s[2, 3] == -0.5
    # K = 2: the first inner step takes 1/8 (trial 4) leaving a spike of -0.025;
    # the second starts at l = 4: 1/16 > 0.05 rejected, 1/32 accepted (t now +e)
    out = suppcg.s_tv(_spike(0.1), 0, suppcg.TVParams(K=2, a=0.5, gamma=1.0))
    assert out.trials == [4, 2] and out.ell == 6
    assert out.s[2, 3] == pytest.approx(-0.125 + 1.0 / 32, abs=0)
    assert np.count_nonzero(out.s) == 1


def test_suppcg_trace_records_schedule():
    # inside Algorithm 3 the l carried between calls follows the same rule: the
    # trace's l_{k+1} minus l_k equals the trials of loop body k, every body
    g, R, b, prob = tiny_problem(seed=8)
    tvp = suppcg.TVParams(K=2, a=0.5, gamma=40.0)
    res = suppcg.suppcg(prob, np.zeros(g.n), tvp, n_iter=12)
    prev = 0
    for k in range(12):
        assert res.trace["ell"][k] - prev == sum(res.trace["trials"][k])
        prev = res.trace["ell"][k]
    assert max(max(t) for t in res.trace["trials"]) > 1    # rejections happened


def _suppcg_ray_form(prob, x0, tvp, n_iter):
    """Algorithm 3 with h = A p never formed: Algorithm 2 uses h only in
    z^T h = (R z)^T (R p) and p^T h = ||R p||^2, and R p follows the direction
    update, R p <- -R z + beta R p.  Test-local, float64, the order of
    operations of the GPU solvers (which keep q = R p)."""
    x = np.asarray(x0, dtype=np.float64).ravel()
    g = prob.RT @ (prob.R @ x - prob.b)
    z = prob.apply_M(g)
    p = -z
    q = -(prob.R @ z)
    qq = float(q @ q)
    x = x + (-float(g @ p) / qq) * p
    ell, xs, betas = 0, [], []
    for _ in range(n_iter):
        st = suppcg.s_tv(x.reshape(prob.shape), ell, tvp)
        ell = st.ell
        x_half = x + st.s.ravel()
        g = prob.RT @ (prob.R @ x_half - prob.b)
        z = prob.apply_M(g)
        w = prob.R @ z
        beta = float(w @ q) / qq
        p = -z + beta * p
        q = -w + beta * q
        qq = float(q @ q)
        x = x_half + (-float(g @ p) / qq) * p
        xs.append(x_half)
        betas.append(beta)
    return xs, betas


def test_h_enters_algorithm2_only_through_its_dot_products():
    # Algorithm 2's h = A p is needed only for beta's numerator z^T h and the
    # denominator p^T h; carrying R p instead gives the same iterates up to
    # rounding, with no drift over a superiorized run with rejections
    g, R, b, prob = tiny_problem(seed=3, shape=(12, 10), A=24, B=17)
    tvp = suppcg.TVParams(1, 0.7, 3.0)
    ref = suppcg.suppcg(prob, np.zeros(g.n), tvp, n_iter=30, record_vectors=True)
    xs, betas = _suppcg_ray_form(prob, np.zeros(g.n), tvp, 30)
    for k in range(30):
        xr = ref.trace["x_half_v"][k + 1]
        assert np.linalg.norm(xs[k] - xr) <= 1e-10 * np.linalg.norm(xr), k
        assert betas[k] == pytest.approx(ref.trace["beta"][k], rel=1e-8, abs=1e-14)
    assert sum(sum(t) for t in ref.trace["trials"]) > 30   # trials were rejected
