"""Pins of the oracle's ALM-CoRUTV (robust PCA with CoR-UTV as the low-rank
step; Sec. V and the synthetic recovery experiment of Sec. VI-D).

The paper's Tables I and II report, for n = 1000, rank 50, outliers of
magnitude 80 on 5 % (10 %) of the entries, with l = 2k and q = 1: the exact
rank 50 recovered, zeta = ||M - L - S||_F / ||M||_F below the 1e-5 stopping
threshold, 12 (14) iterations.  The inputs here are the seeded synthetic
matrices of the same construction (L = G1 G2^T with standard Gaussian
factors, +-80 outliers at uniformly drawn positions).
"""

import numpy as np
import pytest

import inputs as I


@pytest.mark.parametrize("frac,iters", [(0.05, (12, 12)), (0.10, (13, 14))])
def test_rpca_recovers_the_synthetic_low_rank_plus_sparse(orc, frac, iters):
    n, rk = 1000, 50
    low, s = I.rpca_matrix(n, n, rk, frac, seed=1)
    out = orc.rpca_alm(low + s, rk, rk, 1, omega_seed=77)
    lerr = np.linalg.norm(out["L"] - low) / np.linalg.norm(low)
    serr = np.linalg.norm(out["S"] - s) / np.linalg.norm(s)
    print(f"[rpca {frac}] iters {out['iters']} rank {out['rank']} zeta {out['zeta']:.2e} "
          f"L err {lerr:.2e} S err {serr:.2e} ranks {out['ranks']}")
    assert out["rank"] == rk                       # exact numerical rank
    assert out["zeta"] < 1e-5                      # the stopping rule
    assert iters[0] <= out["iters"] <= iters[1]    # Tables I / II: 12 and 14
    assert lerr < 1e-4 and serr < 1e-4             # the components themselves


def test_rpca_shrinkage_is_the_soft_threshold(orc):
    """A matrix with no outliers and rank below l: the sparse part stays
    (numerically) zero and L reproduces M."""
    n, rk = 300, 8
    low, _ = I.rpca_matrix(n, n, rk, 0.0, seed=3)
    out = orc.rpca_alm(low, rk, rk, 1, omega_seed=5)
    assert out["rank"] == rk
    assert np.linalg.norm(out["S"]) <= 1e-4 * np.linalg.norm(low)
    assert np.linalg.norm(out["L"] - low) <= 1e-5 * np.linalg.norm(low)
