"""Counts the nonzero entries of R (strictly positive chord lengths) with the
oracle's closed form, angle block by angle block.

    python tests/golden/count_nnz.py 512 720 725      # 240,840,802
    python tests/golden/count_nnz.py 2048 2048 2899   # 10,945,428,176 (minutes)

bench.py uses these counts as the algorithmic work of R and R^T.
"""
import os
import sys
from multiprocessing import Pool

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

from oracle import closed_form  # noqa: E402
from oracle.geometry import Geometry  # noqa: E402


def _count(args):
    g, a = args
    return closed_form.angle_block(g, a).nnz


def count(side: int, n_angles: int, n_bins: int, workers: int = 6) -> int:
    g = Geometry(side, side, n_angles, n_bins)
    with Pool(workers) as p:
        return sum(p.map(_count, [(g, a) for a in range(n_angles)], chunksize=8))


if __name__ == "__main__":
    side, n_angles, n_bins = (int(v) for v in sys.argv[1:4])
    print(count(side, n_angles, n_bins))
