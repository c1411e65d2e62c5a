"""GPU parity of the stored-weight R and R^T (Section 2, eqs. 2.1-2.2).

Bars: the built matrices hold the oracle's nonzero (ray, pixel) pairs with its
lengths (to the float32 rounding of the stored weight plus the conditioning
term of near-axis ramps, as in the host check of the same build); R^T is R
transposed bit for bit; the products are within 1e-5 relative L2 of the
oracle's, over the whole vector, at 64^2 x 90 x 91, on ragged geometries and
at 512^2 x 720 x 725 (tests/golden/ct512_operators.npz, oracle-written)."""
import os
import sys

import numpy as np
import pytest
import scipy.sparse as sps

from oracle import closed_form
from oracle import projector as oproj
from oracle.geometry import Geometry as OG
from oracle.geometry import angle_cos_sin
from tests._problems import rel_l2, workload_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1807_10151_amd as sp_mod
    return sp_mod


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def sp_geom(sp, og):
    return sp.Geometry(og.rows, og.cols, og.n_angles, og.n_bins, pixel=og.pixel, theta0=og.theta0,
                       dtheta=og.dtheta, bin_spacing=og.bin_spacing, bin_offset=og.bin_offset)


SMALL = [
    OG(64, 64, 90, 91),
    OG(37, 53, 45, 61),
    OG(16, 16, 8, 24, pixel=0.7, bin_spacing=0.35, bin_offset=0.091),
    OG(20, 24, 7, 33, theta0=0.1, dtheta=0.45),
    OG(41, 57, 4, 75, theta0=1e-7, dtheta=np.pi / 2),
    OG(3, 70, 1, 5),
]


@pytest.mark.parametrize("og", SMALL, ids=[f"{g.rows}x{g.cols}x{g.n_angles}x{g.n_bins}" for g in SMALL])
def test_stored_matrices_match_oracle(sp, og):
    print(f"stored matrix {og}", flush=True)
    M = sp.StoredMatrix(sp_geom(sp, og))
    nnz, nbytes = M.info()
    rp0, c0, v0 = M.export(0)
    rp1, c1, v1 = M.export(1)
    assert rp0[0] == 0 and rp0[-1] == nnz and np.all(np.diff(rp0) >= 0)
    assert rp1[0] == 0 and rp1[-1] == nnz and np.all(np.diff(rp1) >= 0)
    Rg = sps.csr_matrix((v0, c0, rp0), shape=(og.m, og.n))
    RTg = sps.csr_matrix((v1, c1, rp1), shape=(og.n, og.m))
    # R^T is R transposed, bit for bit
    T = Rg.T.tocsr()
    T.sort_indices()
    RTs = RTg.copy()
    RTs.sort_indices()
    assert np.array_equal(T.indptr, RTs.indptr) and np.array_equal(T.indices, RTs.indices)
    assert np.array_equal(T.data, RTs.data)
    # against the oracle's R, pair by pair
    R, _ = oproj.matrix(og)
    D = (Rg.astype(np.float64) - R).tocoo()
    ext = (og.rows + og.cols) * og.pixel + og.n_bins * og.bin_spacing + abs(og.bin_offset)
    tol_a = np.empty(og.n_angles)
    for ai in range(og.n_angles):
        _, co, si = angle_cos_sin(og, ai)
        ramp = min(abs(co), abs(si))
        tol_a[ai] = 1e-12 * og.pixel + (8e-16 * ext / ramp * og.pixel if ramp > 0 else 0.0)
    Rd = R.tocsr()
    ref = np.asarray(abs(Rd[D.row, D.col])).ravel() if D.nnz else np.zeros(0)
    bound = tol_a[D.row // og.n_bins] + 6e-8 * ref
    assert np.all(np.abs(D.data) <= bound), float(np.max(np.abs(D.data) / bound))
    # the products, whole vectors
    rng = np.random.default_rng(og.n)
    x = rng.standard_normal((og.rows, og.cols)).astype(np.float32)
    y = rng.standard_normal((og.n_angles, og.n_bins)).astype(np.float32)
    Rx = M.project(cuda(x)).cpu().numpy().ravel()
    RTy = M.backproject(cuda(y)).cpu().numpy().ravel()
    assert rel_l2(Rx, R @ x.astype(np.float64).ravel()) <= 1e-5
    assert rel_l2(RTy, R.T @ y.astype(np.float64).ravel()) <= 1e-5
    # adjoint identity between the two stored products
    lhs = float(np.dot(Rx.astype(np.float64), y.ravel().astype(np.float64)))
    rhs = float(np.dot(x.ravel().astype(np.float64), RTy.astype(np.float64)))
    assert abs(lhs - rhs) <= 1e-6 * max(abs(lhs), 1.0)
    M.close()


@pytest.fixture(scope="module")
def gold():
    sys.path.insert(0, os.path.join(HERE, "golden"))
    from make_ct512_operators import inputs
    d = dict(np.load(os.path.join(HERE, "golden", "ct512_operators.npz")))
    d["x_ell"], d["x_gauss"], d["y_gauss"] = inputs()
    return d


def test_stored_ct512_whole_vectors(sp, gold):
    print("stored matrix 512x512x720x725", flush=True)
    g = sp.Geometry(512, 512, 720, 725)
    M = sp.StoredMatrix(g)
    nnz, nbytes = M.info()
    print(f"nnz {nnz} (oracle {int(gold['nnz'])}), {nbytes / 1e9:.3f} GB", flush=True)
    # Whole angle blocks of R against the oracle's closed form, pair by pair,
    # for sampled angles (axis-parallel, 45 and 135 degrees, neighbours of
    # each, and random ones).  Pairs present on one side only are grazing
    # contacts whose exact length is 0 (a central ray at 45 degrees touching
    # pixel corners): their stored weight must be below 1e-12.
    rp, col, val = M.export(0)
    og = OG(512, 512, 720, 725)
    sample = sorted({0, 1, 179, 180, 181, 359, 360, 361, 539, 540, 541, 719}
                    | set(np.random.default_rng(7).integers(0, 720, 8).tolist()))
    extra = 0
    for a in sample:
        blk = closed_form.angle_block(og, a).tocsr()
        lo, hi = rp[a * 725], rp[(a + 1) * 725]
        Rg = sps.csr_matrix((val[lo:hi].astype(np.float64), col[lo:hi], rp[a * 725:(a + 1) * 725 + 1] - lo),
                            shape=(725, og.n))
        D = (Rg - blk).tocoo()
        ref = np.asarray(abs(blk[D.row, D.col])).ravel() if D.nnz else np.zeros(0)
        assert np.all(np.abs(D.data) <= 1e-12 + 6e-8 * ref), (a, float(np.max(np.abs(D.data) - 6e-8 * ref)))
        extra += Rg.nnz - blk.nnz
    print(f"sampled angles {sample}: {extra} stored pairs beyond the oracle's", flush=True)
    # every other nonzero is the oracle's: the totals differ by grazing pairs only
    assert abs(nnz - int(gold["nnz"])) <= 2 * 725 * 2
    for name in ("ell", "gauss"):
        got = M.project(cuda(gold[f"x_{name}"])).cpu().numpy().ravel()
        e = rel_l2(got, gold[f"Rx_{name}"])
        print(f"stored R x_{name}: rel_l2 {e:.3e}", flush=True)
        assert e <= 1e-5
    got = M.backproject(cuda(gold["y_gauss"])).cpu().numpy().ravel()
    e = rel_l2(got, gold["RTy_gauss"])
    print(f"stored R^T y_gauss: rel_l2 {e:.3e}", flush=True)
    assert e <= 1e-5
    # the stored and the matrix-free products agree with each other too
    mf = sp.sp_project(g, cuda(gold["x_ell"])).cpu().numpy().ravel()
    assert rel_l2(M.project(cuda(gold["x_ell"])).cpu().numpy().ravel(), mf) <= 2e-5
    M.close()


def test_stored_solve_inputs_match_matrix_free(sp):
    """The stored R of the 64^2 workload applied to its phantom gives the
    matrix-free sinogram to 1e-6."""
    og, img, b = workload_problem("small64")
    g = sp_geom(sp, og)
    M = sp.StoredMatrix(g)
    a = M.project(cuda(img)).cpu().numpy()
    m = sp.sp_project(g, cuda(img)).cpu().numpy()
    assert rel_l2(a, m) <= 1e-6
    M.close()
