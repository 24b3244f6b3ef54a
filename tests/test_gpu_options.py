"""GPU parity of the compression and orientation options.

* COR_M_EXPLICIT: M = Q1^T (A Q2) formed with one more pass over A, as
  eq. (14) prints it.  The oracle forms D the same way, so U, T, V agree
  elementwise where the pivots are unique; the library's m_check reports
  ||M - R2^T|| / ||M|| (the identity behind the default compression).
* COR_M_APPROX: eq. (18), M = Q1^T Y1 (Q2^T X)^+ with X the last power
  step's input.  D_approx = D in exact arithmetic (Q1^T A (I - Q2 Q2^T) = 0
  since Q2 spans A^T Q1), so the oracle's explicit D is the reference.
* COR_ULV: A = U L V^T with L lower triangular (Sec. III, the other
  orientation), computed as the URV of A^T; the oracle's URV of A^T,
  transposed back, is the reference (U = V', L = T'^T, V = U').
FP64 rules as in test_gpu_core.py (|d eps| <= 1e-12, orthogonality 1e-13,
factors to 1e-10 where the oracle's smallest pivot gap exceeds 1e-8); FP32
|d eps| <= 1e-5.
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


@pytest.mark.parametrize("mode", ["explicit", "approx"])
@pytest.mark.parametrize("m,n,k,p,q", [
    (900, 700, 32, 8, 0),     # l = 40: register QRCP; q = 0 (X = Omega in eq. (18))
    (1037, 613, 60, 9, 2),    # ragged, two power steps
    (800, 760, 140, 10, 1),   # l = 150: the l > 128 kernels, eq. (18) solve at l = 150
])
def test_compression_modes_f64(cu, dev, orc, mode, m, n, k, p, q):
    import torch

    a, _ = I.lowrank(m, n, np.exp(-np.arange(1, min(m, n) + 1) / 35.0), seed=m + 3 * n)
    om = I.gaussian_omega(n, k + p, 21)
    A = torch.from_numpy(a).to(dev)
    cm = cu.COR_M_EXPLICIT if mode == "explicit" else cu.COR_M_APPROX
    U, T, V, perm, info = cu.decompose(A, k, p, q, omega=om, report=True, compress=cm)
    U0, T0, V0, perm0, info0 = cu.decompose(A, k, p, q, omega=om, report=True)
    torch.cuda.synchronize()
    U, T, V, perm, T0 = *_host(U, T, V, perm), T0.cpu().numpy()
    ref = orc.cor_utv(a, k, p, q, om)
    mg = orc.metrics(a, U, T, V, k)
    mo = orc.metrics(a, ref["U"], ref["T"], ref["V"], k)
    scale = np.abs(ref["T"]).max()
    dT = np.abs(T - ref["T"]).max() / scale
    dU, dV = np.abs(U - ref["U"]).max(), np.abs(V - ref["V"]).max()
    print(f"[{mode} {m}x{n} l={k + p} q={q}] eps_l d {abs(mg['err_l'] - mo['err_l']):.1e}; "
          f"m_check {info.m_check:.1e}; |dT|/|T| {dT:.1e} |dU| {dU:.1e} |dV| {dV:.1e}; "
          f"vs default |dT| {np.abs(T - T0).max() / scale:.1e}; gap {ref['diag'][1]:.1e}")
    assert abs(mg["err_l"] - mo["err_l"]) <= 1e-12
    assert abs(mg["err_k"] - mo["err_k"]) <= 1e-12
    assert mg["orth_u"] <= 1e-13 and mg["orth_v"] <= 1e-13
    assert np.array_equal(np.tril(T, -1), np.zeros_like(T))
    # the identity M = R2^T that the default compression relies on
    assert info.m_check <= (1e-13 if mode == "explicit" else 1e-11)
    assert info0.m_check == 0.0
    if ref["diag"][1] > 1e-8:
        assert np.array_equal(perm, ref["perm"])
        assert dT <= (1e-10 if mode == "explicit" else 1e-9)
        assert dU <= 1e-10 and dV <= 1e-10


def test_explicit_compression_f32(cu, dev, orc):
    import torch

    m, n, k, p, q = 1200, 1000, 50, 10, 1
    a, _ = I.lowrank(m, n, np.exp(-np.arange(1, 301) / 30.0), seed=77)
    om = I.gaussian_omega(n, k + p, 22)
    A = torch.from_numpy(a.astype(np.float32)).to(dev)
    U, T, V, perm, info = cu.decompose(A, k, p, q, omega=om, report=True,
                                       compress=cu.COR_M_EXPLICIT)
    torch.cuda.synchronize()
    U, T, V = _host(U, T, V)
    ref = orc.cor_utv(a, k, p, q, om)
    mg = orc.metrics(a, U, T, V, k)
    mo = orc.metrics(a, ref["U"], ref["T"], ref["V"], k)
    print(f"[explicit f32] eps_l {mg['err_l']:.8e} oracle {mo['err_l']:.8e}; "
          f"m_check {info.m_check:.1e}")
    assert abs(mg["err_l"] - mo["err_l"]) <= 1e-5
    # the pass A Q2 runs in FP32: M agrees with R2^T to the FP32 rounding
    assert info.m_check <= 1e-5


@pytest.mark.parametrize("m,n,k,p,q,fmt", [
    (500, 900, 24, 6, 1, "f64"),    # m < n: the case the paper gives ULV for
    (777, 431, 40, 8, 2, "f64"),    # m > n works as well
    (700, 1300, 100, 40, 0, "f64"), # l = 140
    (640, 1100, 30, 6, 1, "f32"),
    (640, 1100, 30, 6, 1, "bf16"),
])
def test_ulv_matches_oracle_of_transpose(cu, dev, orc, m, n, k, p, q, fmt):
    import torch

    l = k + p
    a, _ = I.lowrank(m, n, np.exp(-np.arange(1, min(m, n) + 1) / 30.0), seed=m * n % 997)
    om = I.gaussian_omega(m, l, 23)  # the URV of A^T draws an m x l test matrix
    A = torch.from_numpy(a).to(dev)
    if fmt == "f32":
        A = A.float().contiguous()
    elif fmt == "bf16":
        A = A.to(torch.bfloat16).contiguous()
    U, L, V, perm, info = cu.decompose(A, k, p, q, omega=om, report=True, orient=cu.COR_ULV)
    torch.cuda.synchronize()
    U, L, V, perm = _host(U, L, V, perm)
    assert U.shape == (m, l) and V.shape == (n, l)
    ref = orc.cor_utv(np.ascontiguousarray(a.T), k, p, q, om)
    mg = orc.metrics(a, U, L, V, k)
    mo = orc.metrics(a, ref["V"], ref["T"].T, ref["U"], k)
    print(f"[ulv {fmt} {m}x{n} l={l} q={q}] eps_l gpu {mg['err_l']:.12e} oracle "
          f"{mo['err_l']:.12e}; orth {mg['orth_u']:.1e} {mg['orth_v']:.1e}; report orth "
          f"{info.orth_u:.1e} {info.orth_v:.1e}; gap {ref['diag'][1]:.1e}")
    assert np.array_equal(np.triu(L, 1), np.zeros_like(L))  # lower triangular
    assert np.all(np.diag(L) >= 0)
    assert mg["orth_u"] <= 1e-13 and mg["orth_v"] <= 1e-13
    assert abs(info.orth_u - mg["orth_u"]) <= 1e-13 and abs(info.orth_v - mg["orth_v"]) <= 1e-13
    if fmt == "f64":  # the report measures against the stored matrix
        assert abs(info.err_l ** 2 - mg["err_l"] ** 2) <= 1e-14 + 1e-11 * mg["err_l"] ** 2
        assert abs(mg["err_l"] - mo["err_l"]) <= 1e-12
        if ref["diag"][1] > 1e-8:
            assert np.array_equal(perm, ref["perm"])
            assert np.abs(L - ref["T"].T).max() <= 1e-10 * np.abs(ref["T"]).max()
            assert np.abs(U - ref["V"]).max() <= 1e-10
            assert np.abs(V - ref["U"]).max() <= 1e-10
    elif fmt == "f32":
        assert abs(mg["err_l"] - mo["err_l"]) <= 1e-5
    else:
        assert mg["err_l"] <= 1.05 * mo["err_l"]


def test_options_batched_equal_single(cu, dev):
    """Grouped launches with the options: each problem equals its single call."""
    import torch

    shapes = [(600, 500, 20, 5, 1), (450, 800, 12, 4, 2), (900, 300, 40, 8, 0)]
    for opts in [cu.cor_opts(1, 0, cu.COR_M_EXPLICIT, 0), cu.cor_opts(1, 0, cu.COR_M_APPROX, 0),
                 cu.cor_opts(1, 0, cu.COR_M_R2T, cu.COR_ULV)]:
        probs, outs, mats = [], [], []
        for i, (m, n, k, p, q) in enumerate(shapes):
            a, _ = I.lowrank(m, n, np.exp(-np.arange(1, min(m, n) + 1) / 20.0), seed=300 + i)
            A = torch.from_numpy(a).to(dev)
            l = k + p
            o = (torch.empty((m, l), dtype=torch.float64, device=dev),
                 torch.empty((l, l), dtype=torch.float64, device=dev),
                 torch.empty((n, l), dtype=torch.float64, device=dev),
                 torch.empty((l,), dtype=torch.int32, device=dev))
            probs.append(cu.make_problem(A, k, p, q, 900 + i, *o))
            outs.append(o)
            mats.append(A)
        st, infos = cu.cor_utv_batched(probs, opts)
        cu.check(st, "batched")
        torch.cuda.synchronize()
        for i, (m, n, k, p, q) in enumerate(shapes):
            l = k + p
            o1 = (torch.empty((m, l), dtype=torch.float64, device=dev),
                  torch.empty((l, l), dtype=torch.float64, device=dev),
                  torch.empty((n, l), dtype=torch.float64, device=dev),
                  torch.empty((l,), dtype=torch.int32, device=dev))
            st, info1 = cu.cor_utv_ex(cu.make_problem(mats[i], k, p, q, 900 + i, *o1), opts)
            cu.check(st, "single")
            torch.cuda.synchronize()
            for x, y in zip(outs[i], o1):
                assert torch.equal(x, y), f"problem {i} differs (compress {opts.compress}, " \
                                          f"orient {opts.orient})"
            assert infos[i].m_check == info1.m_check


def test_ulv_rejects_fp8(cu, dev):
    import torch

    A = torch.zeros((50, 80), dtype=torch.uint8, device=dev)
    s = torch.ones(80, dtype=torch.float32, device=dev)
    U = torch.empty((50, 10), dtype=torch.float64, device=dev)
    T = torch.empty((10, 10), dtype=torch.float64, device=dev)
    V = torch.empty((80, 10), dtype=torch.float64, device=dev)
    pr = cu.make_problem(A, 8, 2, 0, 1, U, T, V, colscale=s)
    st, _ = cu.cor_utv_ex(pr, cu.cor_opts(0, 0, 0, cu.COR_ULV))
    assert st == cu.COR_E_INVAL
    st, _ = cu.cor_utv_ex(pr, cu.cor_opts(0, 0, 7, 0))
    assert st == cu.COR_E_INVAL
