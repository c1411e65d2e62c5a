"""Algorithm 1's repeat-until with rejected trials, GPU against the oracle.

The GPU evaluates the trial step lengths gamma a^l, gamma a^(l+1), ... four at
a time: the first pass over the whole image in parallel, further passes (when
none of the first four is accepted) inside one workgroup.  These cases make
the acceptance land at the last trial of the first pass, in the second pass,
and after many passes, in sp_tv_perturb, in the single-slice solver and in
the batched solver; l, the trials of every inner step and the perturbed image
must match the float64 oracle.  Every case's smallest acceptance margin
|TV(trial) - TV(y)| / TV(y) was checked on the oracle to be far above the
float32 rounding of the TV direction (the printout repeats it)."""
import numpy as np
import pytest

from oracle import projector as oproj
from oracle import suppcg as osup
from oracle import tv as otv
from tests._problems import MU, RHO, oracle_precond, rel_l2, workload_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1807_10151_amd as sp_mod
    return sp_mod


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def trial_margins(y, ell, p):
    """(TV(trial) - TV(y)) / TV(y) of every trial the oracle's Algorithm 1 takes."""
    y = np.asarray(y, dtype=np.float64).copy()
    out = []
    for _ in range(p.K):
        t, _ = otv.nonascending(y)
        tvy = otv.total_variation(y)
        ms = []
        while True:
            yt = y + p.gamma * p.a ** ell * t
            ell += 1
            ms.append((otv.total_variation(yt) - tvy) / tvy)
            if ms[-1] <= 0 or len(ms) >= p.max_trials:
                break
        if ms[-1] <= 0:
            y = yt
        out.append(ms)
    return out


@pytest.fixture(scope="module")
def noisy64():
    og, img, _ = workload_problem("small64")
    rng = np.random.default_rng(3)
    return og, (img + 0.05 * rng.standard_normal(img.shape)).astype(np.float32)


@pytest.mark.parametrize("K,a,gamma,ell,want", [
    (1, 0.5, 20.0, 0, [4]),        # accepted at the last trial of the first pass
    (1, 0.5, 50.0, 0, [5]),        # first trial of the second pass
    (1, 0.9, 200.0, 0, [37]),      # ten passes
    (2, 0.5, 50.0, 0, [5, 1]),     # rejections in the first inner step, l carried on
    (3, 0.7, 30.0, 2, [5, 1, 1]),
])
def test_tv_perturb_rejections_match_oracle(sp, noisy64, K, a, gamma, ell, want):
    og, x = noisy64
    p = osup.TVParams(K, a, gamma)
    ref = osup.s_tv(x.astype(np.float64), ell, p)
    ms = trial_margins(x, ell, p)
    print(f"K={K} a={a} gamma={gamma}: trials {ref.trials}, smallest |margin| "
          f"{min(abs(m) for mm in ms for m in mm):.2e}", flush=True)
    assert ref.trials == want
    g = sp.Geometry(og.rows, og.cols, og.n_angles, og.n_bins)
    xh, ell_out, tvh, trials = sp.sp_tv_perturb(g, cuda(x), ell, K, a, gamma)
    assert trials == ref.trials and ell_out == ref.ell
    assert rel_l2(xh.cpu().numpy(), x.astype(np.float64) + ref.s) <= 1e-6
    assert tvh == pytest.approx(ref.tv_after, rel=1e-6)


@pytest.mark.parametrize("h,l0,gamma,a,want_j", [(0.1, 0, 1.0, 0.5, 4), (0.3, 0, 20.0, 0.5, 7),
                                                  (0.05, 2, 3.0, 0.9, 32)])
def test_tv_perturb_spike_closed_form(sp, h, l0, gamma, a, want_j):
    # a lone interior spike: t = -e_spike and the j-th trial is accepted iff
    # gamma a^(l0 + j - 1) <= 2 h (closed form, see the oracle's pins)
    y = np.zeros((6, 7), dtype=np.float32)
    y[2, 3] = h
    g = sp.Geometry(6, 7, 4, 9)
    xh, ell, tvh, trials = sp.sp_tv_perturb(g, cuda(y), l0, 1, a, gamma)
    lam = gamma * a ** (l0 + want_j - 1)
    assert trials == [want_j] and ell == l0 + want_j
    want = y.astype(np.float64)
    want[2, 3] -= lam
    got = xh.cpu().numpy().astype(np.float64)
    assert np.count_nonzero(got) == 1
    assert got[2, 3] == pytest.approx(want[2, 3], rel=1e-6)
    assert tvh == pytest.approx((2 + np.sqrt(2)) * abs(h - lam), rel=1e-6)


# (K, a, gamma) = (1, 0.8, 200): the first loop body rejects 14 trials (four
# passes), the fifth rejects one; the oracle's smallest acceptance margin over
# the 20 bodies is 1.2e-2.
SOLVE_TV = osup.TVParams(1, 0.8, 200.0)


@pytest.fixture(scope="module")
def solve_ref():
    og, img, b = workload_problem("small64")
    R, _ = oproj.matrix(og)
    prob = osup.Problem(R, b.astype(np.float64), (og.rows, og.cols), oracle_precond)
    ref = osup.suppcg(prob, np.zeros(og.n), SOLVE_TV, n_iter=20)
    return og, b, ref


def test_solve_with_rejections_matches_oracle(sp, solve_ref):
    og, b, ref = solve_ref
    trials = [t for tt in ref.trace["trials"] for t in tt]
    assert trials[0] == 15 and trials[4] == 2 and ref.trace["ell"][-1] == 35
    g = sp.Geometry(og.rows, og.cols, og.n_angles, og.n_bins)
    for graph in (False, True):
        res = sp.sp_suppcg_solve(g, cuda(b), None, K=1, a=0.8, gamma=200.0, mu=MU, rho=RHO,
                                 max_iter=20, graph=graph)
        assert res.k == ref.k == 21
        assert res.trace["trials"].ravel().tolist() == trials
        assert list(res.trace["ell"]) == ref.trace["ell"]
        assert rel_l2(res.x_half.cpu().numpy(), ref.x_half) <= 1e-3
        assert rel_l2(res.x_last.cpu().numpy(), ref.x_last) <= 1e-3
        np.testing.assert_allclose(res.trace["s_norm"], ref.trace["s_norm"], rtol=1e-3)
        np.testing.assert_allclose(res.trace["tv_half"], ref.trace["tv_half"], rtol=1e-3)


def test_batched_solve_with_rejections_matches_oracle(sp, solve_ref):
    # the same run as slice 0 of a batch (the batched decision kernel), next to
    # two other slices
    og, b, ref = solve_ref
    from synth import random_ellipses
    geoms = [sp.Geometry(og.rows, og.cols, og.n_angles, og.n_bins), sp.Geometry(48, 80, 60, 97),
             sp.Geometry(100, 70, 45, 123, theta0=0.1)]
    bs = [cuda(b)]
    for i, gg in enumerate(geoms[1:]):
        img, _ = random_ellipses(gg.rows, gg.cols, 5, 900 + i)
        bs.append(sp.sp_project(gg, cuda(img)).contiguous())
    got = sp.sp_suppcg_solve_batched(geoms, bs, K=1, a=0.8, gamma=200.0, mu=MU, rho=RHO,
                                     max_iter=20)
    assert got[0].k == ref.k == 21
    assert list(got[0].trace["ell"]) == ref.trace["ell"]
    assert rel_l2(got[0].x_half.cpu().numpy(), ref.x_half) <= 1e-3
    assert rel_l2(got[0].x_last.cpu().numpy(), ref.x_last) <= 1e-3
    for i in (1, 2):
        single = sp.sp_suppcg_solve(geoms[i], bs[i], None, K=1, a=0.8, gamma=200.0, mu=MU,
                                    rho=RHO, max_iter=20)
        assert np.array_equal(single.x_half.cpu().numpy(), got[i].x_half.cpu().numpy())
        assert list(single.trace["ell"]) == list(got[i].trace["ell"])
