"""Writes whole-vector references of R, R^T and the gradient R^T (R x - b) at
the 512x512, 720-angle, 725-bin geometry to ct512_operators.npz (float32).

Calls only the oracle (R assembled from the closed-form chord lengths, which
the oracle's tests pin to the per-ray crossing merge) and the shared input
generator.  Inputs, regenerated identically by the tests:
  x_ell   the 20-ellipse phantom of seed 1 (scale 8), rounded to float32;
  x_gauss default_rng(41).standard_normal((512, 512)) rounded to float32;
  y_gauss default_rng(42).standard_normal((720, 725)) rounded to float32;
  b       the float32 data of ct512_oracle.npz (x_ell's rays + 0.5% noise).
Outputs: R x_ell, R x_gauss, R^T y_gauss, R^T (R x_ell - b) and
R^T (R x_gauss - b), each computed in float64 from the float32 inputs.

    python tests/golden/make_ct512_operators.py      (a few minutes, ~8 GB RAM)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import projector  # noqa: E402
from oracle.geometry import Geometry  # noqa: E402
from synth import WORKLOADS, random_ellipses  # noqa: E402

OUT = os.path.join(HERE, "ct512_operators.npz")


def inputs():
    w = WORKLOADS["ct512"]
    x_ell = random_ellipses(w.rows, w.cols, w.n_ellipses, w.seed)[0].astype(np.float32)
    x_gauss = np.random.default_rng(41).standard_normal((w.rows, w.cols)).astype(np.float32)
    y_gauss = np.random.default_rng(42).standard_normal((w.n_angles, w.n_bins)).astype(np.float32)
    return x_ell, x_gauss, y_gauss


def main():
    w = WORKLOADS["ct512"]
    g = Geometry(w.rows, w.cols, w.n_angles, w.n_bins)
    t0 = time.time()
    R, RT = projector.matrix(g, "closed")
    print(f"R assembled: nnz={R.nnz} ({time.time() - t0:.0f} s)", flush=True)
    x_ell, x_gauss, y_gauss = inputs()
    b = np.load(os.path.join(HERE, "ct512_oracle.npz"))["b"].astype(np.float64).ravel()
    Rx_ell = R @ x_ell.astype(np.float64).ravel()
    Rx_gauss = R @ x_gauss.astype(np.float64).ravel()
    out = dict(
        Rx_ell=Rx_ell.astype(np.float32), Rx_gauss=Rx_gauss.astype(np.float32),
        RTy_gauss=(RT @ y_gauss.astype(np.float64).ravel()).astype(np.float32),
        grad_ell=(RT @ (Rx_ell - b)).astype(np.float32),
        grad_gauss=(RT @ (Rx_gauss - b)).astype(np.float32),
        nnz=R.nnz)
    np.savez_compressed(OUT, **out)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
