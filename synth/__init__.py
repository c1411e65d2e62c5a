"""Seeded synthetic inputs shared by the CPU oracle's tests and the GPU path.

This module holds none of the reconstruction method's arithmetic: no projector,
no preconditioner, no total variation, no solver step.  It only draws the
random inputs (random-ellipse phantoms, unit Gaussian noise vectors, probe
vectors) and states the workload geometries, so that both sides of a parity
test start from bit-identical inputs.

Coordinates follow the pixel convention of the paper's total-variation
definition (Section 3.1): pixel (i, j) with 0-based row i counted from the top
and column j from the left; its centre is at
    x_j = (j - (cols - 1) / 2) * pixel,  y_i = ((rows - 1) / 2 - i) * pixel,
so the image is centred at the origin.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Workload",
    "random_ellipses",
    "unit_noise",
    "noisy_data",
    "WORKLOADS",
    "batched_slices",
    "large_batch",
]


def random_ellipses(rows: int, cols: int, n_ellipses: int, seed: int,
                    scale: float | None = None, pixel: float = 1.0):
    """Random-ellipse phantom.

    Per ellipse, drawn in this order from ``numpy.random.default_rng(seed)``:
    centre cx, cy ~ U(-24S, 24S); semi-axes a, b ~ U(4S, 20S); rotation
    phi ~ U(0, pi); density rho ~ U(0.1, 1); with S = side / 64 (side = max
    of rows and cols) unless ``scale`` is given.  A pixel's value is the sum of
    rho over the ellipses that contain the pixel centre (overlaps add).

    Returns ``(image[rows, cols] float64, rng)``; the generator is returned so
    that the caller can draw the noise right after the ellipses.
    """
    if scale is None:
        scale = max(rows, cols) / 64.0
    rng = np.random.default_rng(seed)
    xs = (np.arange(cols, dtype=np.float64) - (cols - 1) / 2.0) * pixel
    ys = ((rows - 1) / 2.0 - np.arange(rows, dtype=np.float64)) * pixel
    X, Y = np.meshgrid(xs, ys)
    img = np.zeros((rows, cols), dtype=np.float64)
    for _ in range(n_ellipses):
        cx = rng.uniform(-24.0 * scale, 24.0 * scale)
        cy = rng.uniform(-24.0 * scale, 24.0 * scale)
        ea = rng.uniform(4.0 * scale, 20.0 * scale)
        eb = rng.uniform(4.0 * scale, 20.0 * scale)
        phi = rng.uniform(0.0, math.pi)
        rho = rng.uniform(0.1, 1.0)
        dx, dy = X - cx, Y - cy
        u = dx * math.cos(phi) + dy * math.sin(phi)
        v = -dx * math.sin(phi) + dy * math.cos(phi)
        img += rho * ((u / ea) ** 2 + (v / eb) ** 2 <= 1.0)
    return img, rng


def unit_noise(rng, m: int):
    """m standard-normal draws from ``rng`` (the phantom's generator)."""
    return rng.standard_normal(m)


def noisy_data(b_exact, noise, frac: float):
    """b = b_exact + sigma * noise with sigma = frac * max(b_exact)."""
    b_exact = np.asarray(b_exact, dtype=np.float64)
    sigma = frac * float(np.max(b_exact))
    return b_exact + sigma * np.asarray(noise, dtype=np.float64)


@dataclass(frozen=True)
class Workload:
    """One reconstruction workload: geometry, phantom recipe, noise, iterations."""
    name: str
    rows: int
    cols: int
    n_angles: int
    n_bins: int
    n_ellipses: int
    seed: int
    noise_frac: float
    iterations: int

    @property
    def n(self) -> int:
        return self.rows * self.cols

    @property
    def m(self) -> int:
        return self.n_angles * self.n_bins


# The reconstruction workloads.  Angles are uniform over [0, pi) and bins sit at
# unit spacing, centred on the rotation axis; pixels are unit squares.
WORKLOADS = {
    # 64x64 image, 90 angles, 91 bins, 5 ellipses, 1% noise, 20 iterations.
    "small64": Workload("small64", 64, 64, 90, 91, 5, 0, 0.01, 20),
    # 512x512 image, 720 angles, 725 bins, 20 ellipses (scale 8), 0.5% noise,
    # 100 iterations.
    "ct512": Workload("ct512", 512, 512, 720, 725, 20, 1, 0.005, 100),
    # Paper-shaped stand-in: 243x243 pixels, 360 angles, 345 rays.
    "paper243": Workload("paper243", 243, 243, 360, 345, 20, 3, 0.01, 20),
    # 2048x2048 image, 2048 angles, 2899 bins, 50 ellipses.
    "ct2048": Workload("ct2048", 2048, 2048, 2048, 2899, 50, 5000, 0.005, 200),
}


def batched_slices(count: int = 64, seed: int = 2):
    """Mixed-size slice batch: sides from {256, 384, 512, 768, 1024}.

    From ``default_rng(seed)``: sides = choice(count), then noise fractions
    uniform in [0.2%, 2%).  Angles = 8 * round(1.4 * side / 8) over [0, pi);
    bins = ceil(side * sqrt(2)) + 1; slice i uses phantom seed 1000 + i with 20
    ellipses.
    """
    rng = np.random.default_rng(seed)
    sides = rng.choice(np.array([256, 384, 512, 768, 1024]), count)
    fracs = rng.uniform(0.002, 0.02, count)
    out = []
    for i, (side, frac) in enumerate(zip(sides.tolist(), fracs.tolist())):
        A = 8 * int(round(1.4 * side / 8))
        B = int(math.ceil(side * math.sqrt(2.0))) + 1
        out.append(Workload(f"slice{i}", side, side, A, B, 20, 1000 + i, frac, 50))
    return out


def large_batch(count: int = 8):
    """2048 x 2048 slices, 2048 angles over [0, pi), 2899 bins, 50 ellipses
    (scale 32), phantom seeds 5000 + i, noise fractions 0.25%, 0.25%, 0.5%,
    0.5%, 1%, 1%, 2%, 2% (two slices each), 200 iterations."""
    fracs = [0.0025, 0.0025, 0.005, 0.005, 0.01, 0.01, 0.02, 0.02]
    return [Workload(f"large{i}", 2048, 2048, 2048, 2899, 50, 5000 + i, fracs[i % len(fracs)], 200)
            for i in range(count)]
