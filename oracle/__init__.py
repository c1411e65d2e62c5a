"""CPU FP64 oracle for superiorized preconditioned conjugate gradients.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
GPU path is checked against.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the GPU library never does, and
this package shares no code with it.

Everything is float64 NumPy/SciPy, written from the paper
(Helou, Herman, Lin, Zibetti: "Superiorization of preconditioned conjugate
gradient algorithms for tomographic image reconstruction"):

* ``geometry``     parallel-beam geometry of Section 4.1 (readings G1-G7)
* ``siddon``       R as line-in-pixel intersection lengths, per ray (Section 2)
* ``closed_form``  the same lengths from the closed-form trapezoid (reading G8)
* ``projector``    R and its transpose as sparse matrices (eqs. 2.1-2.2)
* ``precond``      M = F^-1 D F with the ramp-Hamming window of eq. (3.2)
* ``tv``           total variation and its nonascending vector (Section 3.1)
* ``suppcg``       Algorithms 1 (S_TV), 2 (U_PCG) and 3 (SupPCG)
* ``suptpcg``      Algorithms 4 and 5 (transformed PCG; dense, tiny grids)
* ``learned``      a learned SPD preconditioner C^T diag(softplus(d)) C

Pinned by the ``-m "not gpu"`` tests under ``tests/`` against closed forms,
brute force and the paper's theorems.  Parts with no pin say "parity unpinned"
in their own module docstring.
"""
