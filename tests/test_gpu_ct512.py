"""512x512, 720-angle, 725-bin SupPCG run on the GPU against the float64
oracle's 100-iteration reference (tests/golden/ct512_oracle.npz, written by
tests/golden/make_ct512.py from the oracle only).

Bar: x_{100+1/2} and x_{101} within 1e-3 relative L2, identical l trace."""
import os

import numpy as np
import pytest

from tests._problems import A, GAMMA, K, MU, RHO, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ct512_oracle.npz")


@pytest.fixture(scope="module")
def gold():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return np.load(GOLD)


def test_ct512_100_iterations_match_oracle(gold):
    import paper_1807_10151_amd as sp
    g = sp.Geometry(512, 512, 720, 725)
    b = torch.from_numpy(np.ascontiguousarray(gold["b"])).cuda()
    res = sp.sp_suppcg_solve(g, b, None, K=K, a=A, gamma=GAMMA, mu=MU, rho=RHO, max_iter=100,
                             graph=True)
    assert res.k == int(gold["k"]) == 101
    e_half = rel_l2(res.x_half.cpu().numpy(), gold["x_half"])
    e_last = rel_l2(res.x_last.cpu().numpy(), gold["x_last"])
    print(f"ct512: rel_l2 x_half {e_half:.3e} x_last {e_last:.3e}", flush=True)
    tv_err = float(np.max(np.abs(res.trace["tv_half"] / gold["tv_half"] - 1.0)))
    f_err = float(np.max(np.abs(res.trace["f_half"] / gold["f_half"] - 1.0)))
    print(f"ct512: max rel f_half {f_err:.3e} tv_half {tv_err:.3e}", flush=True)
    assert list(res.trace["ell"]) == gold["ell"].tolist()
    assert e_half <= 1e-3 and e_last <= 1e-3
    np.testing.assert_allclose(res.trace["f_half"], gold["f_half"], rtol=1e-3)
    np.testing.assert_allclose(res.trace["tv_half"], gold["tv_half"], rtol=1e-3)
