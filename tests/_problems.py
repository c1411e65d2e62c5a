"""Seeded test problems built from the shared input generator and the oracle.

Every expected value and every data vector b comes from the oracle; the GPU
side receives the same float32 arrays.
"""
from __future__ import annotations

import functools

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
