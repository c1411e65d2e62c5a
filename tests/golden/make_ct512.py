"""Writes the float64 oracle's reference run for the 512x512, 720-angle,
725-bin workload (100 SupPCG iterations) to ct512_oracle.npz.

Calls only the oracle and the shared input generator:
  phantom: 20 random ellipses, seed 1 (scale 8); b = R x + 0.5% Gaussian noise,
  stored as float32 (the GPU receives exactly these values);
  SupPCG with K = 1, a = 0.5, gamma = 0.5 (first trial step 0.5^k),
  ramp-Hamming preconditioner mu = 1e-5, rho = 0.8, x0 = 0, 100 loop bodies.

    python tests/golden/make_ct512.py        (about 10 minutes, ~8 GB RAM)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import precond, projector, suppcg  # noqa: E402
from oracle.geometry import Geometry  # noqa: E402
from synth import WORKLOADS, noisy_data, random_ellipses, unit_noise  # noqa: E402

OUT = os.path.join(HERE, "ct512_oracle.npz")


def main(n_iter=100):
    w = WORKLOADS["ct512"]
    g = Geometry(w.rows, w.cols, w.n_angles, w.n_bins)
    t0 = time.time()
    R, _ = projector.matrix(g, "closed")
    print(f"R assembled: nnz={R.nnz} ({time.time() - t0:.0f} s)", flush=True)
    img, rng = random_ellipses(w.rows, w.cols, w.n_ellipses, w.seed)
    b32 = noisy_data(R @ img.ravel(), unit_noise(rng, g.m), w.noise_frac).astype(np.float32)
    prob = suppcg.Problem(R, b32.astype(np.float64), (w.rows, w.cols),
                          lambda v: precond.apply(v, 1e-5, 0.8))
    t1 = time.time()
    res = suppcg.suppcg(prob, np.zeros(g.n), suppcg.TVParams(K=1, a=0.5, gamma=0.5), n_iter=n_iter)
    print(f"SupPCG {n_iter} iterations: {time.time() - t1:.0f} s, k={res.k}", flush=True)
    tr = res.trace
    np.savez_compressed(
        OUT, b=b32.reshape(w.n_angles, w.n_bins), x_half=res.x_half.astype(np.float32),
        x_last=res.x_last.astype(np.float32), k=res.k,
        ell=np.array(tr["ell"], dtype=np.int32),
        trials=np.array([t[0] for t in tr["trials"]], dtype=np.int32),
        f_half=np.array(tr["f_half"]), tv_half=np.array(tr["tv_half"]),
        alpha=np.array(tr["alpha"]), beta=np.array(tr["beta"]), f0=tr["f0"],
        nnz=R.nnz)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
