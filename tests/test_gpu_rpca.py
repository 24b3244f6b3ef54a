"""GPU parity of robust PCA by ALM with CoR-UTV as the low-rank step
(cor_rpca_alm, Sec. V) against the oracle's rpca_alm on the same seeded
L + S matrices (the construction of the synthetic recovery experiment of
Sec. VI-D) and the same Gaussian test matrix (seed).

The iteration is a fixed-point map with a soft threshold, so FP64 rounding
differences between the two sides (CoR-UTV factors agree to ~1e-14) can only
move an entry across the threshold when it sits within rounding of it; on
these inputs both sides take the same path: the same iteration count and
rank, L and S equal to a relative 1e-11 of their largest entries (measured
3e-15 to 7e-14).
"""

import numpy as np
import pytest

import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    import paper_1810_07323_amd as cu

    cu.lib()
    return cu


@pytest.fixture(scope="module")
def dev():
    import torch

    return torch.device("cuda:0")


@pytest.mark.parametrize("m,n,rk,frac,k,p,q,seed,recovers", [
    (1000, 1000, 50, 0.05, 50, 50, 1, 77, True),  # Table I's shape: rank 50, 5 % outliers, l = 2k
    (1000, 1000, 50, 0.10, 50, 50, 1, 78, True),  # Table II's: 10 % outliers
    (700, 451, 20, 0.08, 20, 12, 2, 79, True),    # ragged tiles, m > n, two power steps
    # m < n, q = 0 and little oversampling: the method itself settles at rank
    # l = 16 with L off by ~0.4 (both sides alike); a parity case, not a recovery
    (333, 610, 12, 0.05, 12, 4, 0, 80, False),
])
def test_rpca_f64_matches_oracle(cu, dev, orc, m, n, rk, frac, k, p, q, seed, recovers):
    import torch

    low, s = I.rpca_matrix(m, n, rk, frac, seed=seed)
    M = low + s
    ref = orc.rpca_alm(M, k, p, q, omega_seed=seed)
    L, S, info = cu.rpca(torch.from_numpy(M).to(dev), k, p, q, seed=seed)
    torch.cuda.synchronize()
    L, S = L.cpu().numpy(), S.cpu().numpy()
    dL = np.abs(L - ref["L"]).max() / np.abs(ref["L"]).max()
    dS = np.abs(S - ref["S"]).max() / max(np.abs(ref["S"]).max(), 1e-300)
    lerr = np.linalg.norm(L - low) / np.linalg.norm(low)
    print(f"[rpca f64 {m}x{n} r={rk} {frac}] iters {info.iters} (oracle {ref['iters']}) rank "
          f"{info.rank} ({ref['rank']}) zeta {info.zeta:.3e} ({ref['zeta']:.3e}) |dL| {dL:.1e} "
          f"|dS| {dS:.1e} L err {lerr:.1e} {info.ms:.1f} ms")
    assert info.iters == ref["iters"] and info.rank == ref["rank"]
    assert info.zeta < 1e-5
    assert abs(info.zeta - ref["zeta"]) <= 1e-6 * ref["zeta"] + 1e-14
    assert dL <= 1e-11 and dS <= 1e-11
    if recovers:
        assert info.rank == rk and lerr < 1e-4
    # S's support: the sparse part's nonzeros agree except where the shrunk
    # value sits within rounding of zero on one side
    diff = (S != 0) != (ref["S"] != 0)
    assert np.all(np.abs(np.where(diff, S - ref["S"], 0.0)) <= 1e-11 * np.abs(ref["S"]).max())


def test_rpca_iteration_cap_matches_oracle(cu, dev, orc):
    """max_iter stops both sides after the same iterate (an unconverged state)."""
    import torch

    low, s = I.rpca_matrix(600, 500, 30, 0.1, seed=5)
    M = low + s
    ref = orc.rpca_alm(M, 30, 20, 1, omega_seed=6, max_iter=4)
    L, S, info = cu.rpca(torch.from_numpy(M).to(dev), 30, 20, 1, seed=6, max_iter=4)
    torch.cuda.synchronize()
    assert info.iters == 4 and ref["iters"] == 4
    assert info.rank == ref["rank"]
    assert abs(info.zeta - ref["zeta"]) <= 1e-9 * ref["zeta"]
    assert np.abs(L.cpu().numpy() - ref["L"]).max() <= 1e-9 * np.abs(ref["L"]).max()
    assert np.abs(S.cpu().numpy() - ref["S"]).max() <= 1e-9 * np.abs(ref["S"]).max()


def test_rpca_f32_recovers(cu, dev, orc):
    """B and the passes over it in FP32 (the ALM state and L stay FP64): the
    rank and the recovery of L and S as in FP64."""
    import torch

    low, s = I.rpca_matrix(1000, 1000, 50, 0.05, seed=77)
    L, S, info = cu.rpca(torch.from_numpy(low + s).to(dev), 50, 50, 1, seed=77,
                         prec=cu.COR_F32)
    torch.cuda.synchronize()
    L, S = L.cpu().numpy(), S.cpu().numpy()
    lerr = np.linalg.norm(L - low) / np.linalg.norm(low)
    serr = np.linalg.norm(S - s) / np.linalg.norm(s)
    print(f"[rpca f32] iters {info.iters} rank {info.rank} zeta {info.zeta:.2e} L err {lerr:.1e} "
          f"S err {serr:.1e}")
    assert info.rank == 50 and info.zeta < 1e-5 and info.iters <= 20
    assert lerr < 1e-4 and serr < 1e-4


def test_rpca_rejects_bad_input(cu, dev):
    import torch

    Z = torch.zeros((300, 200), dtype=torch.float64, device=dev)
    L = torch.empty_like(Z)
    S = torch.empty_like(Z)
    st, _ = cu.cor_rpca_alm(Z, 300, 200, 200, cu.cor_rpca_opts(10, 5, 1, cu.COR_F64, 1), L, S)
    assert st == cu.COR_E_NUMERIC           # M = 0: no penalty scale
    st, _ = cu.cor_rpca_alm(Z, 300, 200, 200, cu.cor_rpca_opts(10, 5, 1, cu.COR_BF16, 1), L, S)
    assert st == cu.COR_E_INVAL
    st, _ = cu.cor_rpca_alm(Z, 300, 200, 200, cu.cor_rpca_opts(150, 60, 1, cu.COR_F64, 1), L, S)
    assert st == cu.COR_E_INVAL             # l >= min(m, n)
    st, _ = cu.cor_rpca_alm(Z, 300, 200, 100, cu.cor_rpca_opts(10, 5, 1, cu.COR_F64, 1), L, S)
    assert st == cu.COR_E_INVAL             # ldm < n
