"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds input construction only: random orthonormal factors, spectra
and the matrices built from them, the Gaussian test matrix handed to both sides
when a run compares them, and the request lists of the batched and served
workloads.  None of the CoR-UTV arithmetic (sketches, orthonormalisation,
compression, QRCP, assembly) lives here.

Recipes (the paper's constructions, Sec. "Numerical Experiments"):

* random orthonormal factors: Q of the QR of an i.i.d. N(0,1) matrix with the
  columns multiplied by sign(diag R), which makes Q Haar distributed
  (Mezzadri 2007); the paper only asks for "random orthonormal" factors;
* low-rank-plus-tail matrices A = U diag(sigma) V^T (+ optional noise);
* NoisyLowRank-I/II of the singular-value comparison (Fig. 1 / Fig. 2);
* the robust-PCA low-rank plus sparse matrices of the synthetic recovery
  experiment (Tables I and II).
"""

from .gen import (  # noqa: F401
    gaussian,
    haar,
    lowrank,
    spectrum,
    config_matrix,
    noisy_lowrank,
    rpca_matrix,
    gaussian_omega,
    batched_problems,
    served_requests,
    CONFIGS,
)
