"""GPU parity of the fused power step (cor_opts.fused_power): the q power
steps before the final pair read A once each, forming A^T (A X) as the loop
of Alg. 3 prints it, with the first sketch's Gram taken as X^T (A^T A X) and
Y R1^{-1} = A^T Q1 formed on the small side.  In exact arithmetic Q2 after
each step is the same as the two-pass step's, so the result is the oracle's
(which orthonormalises after every product) to the same rules as the
two-pass path: FP64 |d eps| <= 1e-12, orthogonality <= 1e-13, U, T, V
elementwise to 1e-10 where the pivots are unique; FP32 |d eps| <= 1e-5.
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


def _host(*ts):
    return [t.cpu().numpy() for t in ts]


@pytest.mark.parametrize("m,n,k,p,q,lda_pad", [
    (20000, 1000, 8, 4, 2, 0),   # tall, l = 12, n at the FP64 limit: two fused steps
    (20000, 500, 20, 4, 2, 0),   # tall, l = 24
    (3001, 291, 33, 7, 1, 5),    # ragged rows and columns, lda > n, l = 40 (three column tiles)
    (1500, 190, 50, 14, 3, 0),   # l = 64 (four column tiles)
    (900, 300, 6, 4, 1, 0),      # l = 10, a single split
])
def test_fused_f64_matches_oracle(cu, dev, orc, m, n, k, p, q, lda_pad):
    import torch

    a, _ = I.lowrank(m, n, np.exp(-np.arange(1, n + 1) / 25.0), seed=m + n)
    om = I.gaussian_omega(n, k + p, 61)
    if lda_pad:
        buf = torch.zeros((m, n + lda_pad), dtype=torch.float64, device=dev)
        buf[:, :n] = torch.from_numpy(a).to(dev)
        A = buf[:, :n]
    else:
        A = torch.from_numpy(a).to(dev)
    U, T, V, perm, info = cu.decompose(A, k, p, q, omega=om, report=True, fused=True)
    U0, T0, V0, perm0, _ = cu.decompose(A, k, p, q, omega=om, report=True)
    torch.cuda.synchronize()
    U, T, V, perm, T0 = *_host(U, T, V, perm), T0.cpu().numpy()
    ref = orc.cor_utv(a, k, p, q, om)
    mg = orc.metrics(a, U, T, V, k)
    mo = orc.metrics(a, ref["U"], ref["T"], ref["V"], k)
    scale = np.abs(ref["T"]).max()
    dT = np.abs(T - ref["T"]).max() / scale
    dU, dV = np.abs(U - ref["U"]).max(), np.abs(V - ref["V"]).max()
    print(f"[fused f64 {m}x{n} l={k + p} q={q}] d eps_l {abs(mg['err_l'] - mo['err_l']):.1e} "
          f"d eps_k {abs(mg['err_k'] - mo['err_k']):.1e} orth {mg['orth_u']:.1e} "
          f"{mg['orth_v']:.1e}; |dT|/|T| {dT:.1e} |dU| {dU:.1e} |dV| {dV:.1e}; vs two-pass "
          f"|dT| {np.abs(T - T0).max() / scale:.1e}; gap {ref['diag'][1]:.1e} flags {info.flags}")
    assert abs(mg["err_l"] - mo["err_l"]) <= 1e-12
    assert abs(mg["err_k"] - mo["err_k"]) <= 1e-12
    assert mg["orth_u"] <= 1e-13 and mg["orth_v"] <= 1e-13
    assert abs(info.err_l ** 2 - mg["err_l"] ** 2) <= 1e-14 + 1e-11 * mg["err_l"] ** 2
    assert np.array_equal(np.tril(T, -1), np.zeros_like(T))
    if ref["diag"][1] > 1e-8:
        assert np.array_equal(perm, ref["perm"])
        assert dT <= 1e-10 and dU <= 1e-10 and dV <= 1e-10


def test_fused_f32_tall_matches_oracle(cu, dev, orc):
    """The tall robust-PCA request shape scaled down (FP32, rank 5 plus
    outliers, l = 13, q = 2): where the fused step pays."""
    import torch

    m, n, k, p, q = 30000, 2000, 5, 8, 2
    low, s = I.rpca_matrix(m, n, 5, 0.05, seed=7)
    a = low + s
    om = I.gaussian_omega(n, k + p, 62)
    A = torch.from_numpy(a.astype(np.float32)).to(dev)
    U, T, V, perm, info = cu.decompose(A, k, p, q, omega=om, report=True, fused=True)
    U0, T0, V0, _, _ = cu.decompose(A, k, p, q, omega=om, report=True)
    torch.cuda.synchronize()
    U, T, V, U0, T0, V0 = _host(U, T, V, U0, T0, V0)
    ref = orc.cor_utv(a, k, p, q, om)
    mg = orc.metrics(a, U, T, V, k)
    m0 = orc.metrics(a, U0, T0, V0, k)
    mo = orc.metrics(a, ref["U"], ref["T"], ref["V"], k)
    print(f"[fused f32 {m}x{n} l={k + p} q={q}] eps_l fused {mg['err_l']:.10e} two-pass "
          f"{m0['err_l']:.10e} oracle {mo['err_l']:.10e}; orth {mg['orth_u']:.1e} {mg['orth_v']:.1e}")
    assert abs(mg["err_l"] - mo["err_l"]) <= 1e-5
    assert abs(mg["err_k"] - mo["err_k"]) <= 1e-5
    assert mg["orth_u"] <= 1e-13 and mg["orth_v"] <= 1e-13


def test_fused_ulv_matches_oracle_of_transpose(cu, dev, orc):
    """ULV of a wide matrix with the fused step: the passes read A^T, whose
    column count is the caller's m."""
    import torch

    m, n, k, p, q = 400, 12000, 12, 4, 2
    a, _ = I.lowrank(m, n, np.exp(-np.arange(1, m + 1) / 20.0), seed=5)
    om = I.gaussian_omega(m, k + p, 63)
    A = torch.from_numpy(a).to(dev)
    U, L, V, perm, info = cu.decompose(A, k, p, q, omega=om, orient=cu.COR_ULV, fused=True)
    torch.cuda.synchronize()
    U, L, V = _host(U, L, V)
    ref = orc.cor_utv(np.ascontiguousarray(a.T), k, p, q, om)
    mg = orc.metrics(a, U, L, V, k)
    mo = orc.metrics(a, ref["V"], ref["T"].T, ref["U"], k)
    print(f"[fused ulv {m}x{n}] d eps_l {abs(mg['err_l'] - mo['err_l']):.1e}")
    assert abs(mg["err_l"] - mo["err_l"]) <= 1e-12
    assert mg["orth_u"] <= 1e-13 and mg["orth_v"] <= 1e-13
    if ref["diag"][1] > 1e-8:
        assert np.abs(L - ref["T"].T).max() <= 1e-10 * np.abs(ref["T"]).max()


def test_fused_batched_equals_single(cu, dev):
    import torch

    shapes = [(5000, 500, 20, 6), (2200, 300, 8, 4), (9000, 1000, 8, 4)]
    q = 2
    opts = cu.cor_opts(0, 0, cu.COR_M_R2T, cu.COR_URV, 1)
    probs, outs, mats = [], [], []
    for i, (m, n, k, p) in enumerate(shapes):
        a, _ = I.lowrank(m, n, np.exp(-np.arange(1, n + 1) / 30.0), seed=40 + i)
        A = torch.from_numpy(a).to(dev)
        l = k + p
        o = (torch.empty((m, l), dtype=torch.float64, device=dev),
             torch.empty((l, l), dtype=torch.float64, device=dev),
             torch.empty((n, l), dtype=torch.float64, device=dev),
             torch.empty((l,), dtype=torch.int32, device=dev))
        probs.append(cu.make_problem(A, k, p, q, 70 + i, *o))
        outs.append(o)
        mats.append(A)
    st, _ = cu.cor_utv_batched(probs, opts)
    cu.check(st, "batched fused")
    torch.cuda.synchronize()
    for i, (m, n, k, p) in enumerate(shapes):
        l = k + p
        o1 = (torch.empty((m, l), dtype=torch.float64, device=dev),
              torch.empty((l, l), dtype=torch.float64, device=dev),
              torch.empty((n, l), dtype=torch.float64, device=dev),
              torch.empty((l,), dtype=torch.int32, device=dev))
        st, _ = cu.cor_utv_ex(cu.make_problem(mats[i], k, p, q, 70 + i, *o1), opts)
        cu.check(st, "single fused")
        torch.cuda.synchronize()
        for x, y in zip(outs[i], o1):
            assert torch.equal(x, y), f"problem {i} differs from its single call"


def test_fused_rejects_what_it_cannot_run(cu, dev):
    import torch

    def call(A, k, p, q, colscale=None):
        m, n = A.shape
        l = k + p
        U = torch.empty((m, l), dtype=torch.float64, device=dev)
        T = torch.empty((l, l), dtype=torch.float64, device=dev)
        V = torch.empty((n, l), dtype=torch.float64, device=dev)
        pr = cu.make_problem(A, k, p, q, 1, U, T, V, colscale=colscale)
        st, _ = cu.cor_utv_ex(pr, cu.cor_opts(0, 0, 0, 0, 1))
        return st

    A16 = torch.zeros((600, 500), dtype=torch.bfloat16, device=dev)
    assert call(A16, 10, 4, 1) == cu.COR_E_INVAL           # BF16 passes
    A = torch.zeros((600, 500), dtype=torch.float64, device=dev)
    assert call(A, 60, 20, 1) == cu.COR_E_INVAL            # l = 80 > 64
    A = torch.zeros((600, 3000), dtype=torch.float32, device=dev)
    assert call(A, 10, 4, 1) == cu.COR_E_INVAL             # n = 3000 > 2400 (FP32)
    # one q per batched call
    B = [torch.randn((500, 300), dtype=torch.float64, device=dev) for _ in range(2)]
    probs = []
    for i, Bi in enumerate(B):
        probs.append(cu.make_problem(Bi, 8, 4, 1 + i, 3,
                                     torch.empty((500, 12), dtype=torch.float64, device=dev),
                                     torch.empty((12, 12), dtype=torch.float64, device=dev),
                                     torch.empty((300, 12), dtype=torch.float64, device=dev)))
    st, _ = cu.cor_utv_batched(probs, cu.cor_opts(0, 0, 0, 0, 1))
    assert st == cu.COR_E_INVAL
    # q = 0 has no power step to fuse: same result as without the option
    A = torch.from_numpy(np.random.default_rng(3).standard_normal((800, 400))).to(dev)
    r1 = cu.decompose(A, 10, 5, 0, seed=9, fused=True)
    r0 = cu.decompose(A, 10, 5, 0, seed=9)
    torch.cuda.synchronize()
    for x, y in zip(r1[:4], r0[:4]):
        assert torch.equal(x, y)
