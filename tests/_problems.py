"""Seeded test problems built from the shared input generator and the oracle.

Every expected value and every data vector b comes from the oracle; the GPU
side receives the same float32 arrays.
"""
from __future__ import annotations

import functools
import math

import numpy as np

from oracle import precond as oprecond
from oracle import projector as oproj
from oracle.geometry import Geometry as OGeometry
from synth import WORKLOADS, noisy_data, random_ellipses, unit_noise

# Preconditioner and perturbation settings used by the parity runs: the
# paper's SupPCG preset for (mu, rho) and the step schedule gamma_k = 0.5^k
# (K = 1, a = 0.5, gamma = 0.5).
MU, RHO = 1e-5, 0.8
K, A, GAMMA = 1, 0.5, 0.5


def ogeom(w):
    return OGeometry(w.rows, w.cols, w.n_angles, w.n_bins)


@functools.lru_cache(maxsize=4)
def workload_problem(name: str):
    """(oracle geometry, phantom float32 [rows, cols], b float32 [A, B])."""
    w = WORKLOADS[name]
    g = ogeom(w)
    img, rng = random_ellipses(w.rows, w.cols, w.n_ellipses, w.seed)
    b_exact = oproj.project(g, img)
    b = noisy_data(b_exact, unit_noise(rng, g.m), w.noise_frac)
    return g, img.astype(np.float32), b.astype(np.float32).reshape(w.n_angles, w.n_bins)


def oracle_precond(v):
    return oprecond.apply(v, MU, RHO)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def random_geometries(n, seed=2024):
    """Seeded random parallel-beam geometries: image sizes 1-160 a side, 1-120
    angles with a random start and (half the time) a random step, bin counts
    from 0.3 to 1.2 of the diagonal, spacings 0.6-1.6 pixels, offsets within
    three spacings, and non-unit pixels half the time."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        rows, cols = (int(v) for v in rng.integers(1, 161, 2))
        n_angles = int(rng.integers(1, 121))
        pixel = 1.0 if rng.random() < 0.5 else float(rng.uniform(0.5, 1.5))
        spacing = pixel * float(rng.uniform(0.6, 1.6))
        diag = math.hypot(rows, cols) * pixel
        n_bins = int(rng.integers(max(1, int(0.3 * diag / spacing)), int(1.2 * diag / spacing) + 3))
        theta0 = float(rng.uniform(0.0, math.pi))
        dtheta = math.pi / n_angles if rng.random() < 0.5 else float(rng.uniform(0.01, 0.5))
        offset = float(rng.uniform(-3.0, 3.0)) * spacing
        out.append(OGeometry(rows, cols, n_angles, n_bins, pixel=pixel, theta0=theta0, dtheta=dtheta,
                             bin_spacing=spacing, bin_offset=offset))
    return out
