"""GPU parity of cor_utv_host: A in host memory, every pass streaming it in
row panels through device staging buffers (the pass model of Sec. III with A
stored outside the fast memory).  The result is the oracle's to the FP64
rules (|d eps| <= 1e-12, orthogonality <= 1e-13, U, T, V elementwise to
1e-10 where the pivots are unique) and the in-HBM call's to the order of the
K-split partial sums: pinned and pageable host memory, lda > n, a last
panel shorter than the others, one panel, the fused power step, and the
BF16 format.
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


def _outputs(dev, m, n, l):
    import torch

    return (torch.empty((m, l), dtype=torch.float64, device=dev),
            torch.empty((l, l), dtype=torch.float64, device=dev),
            torch.empty((n, l), dtype=torch.float64, device=dev),
            torch.empty((l,), dtype=torch.int32, device=dev))


def _host_run(cu, dev, Ah, k, p, q, om, panel_rows, opts=None, lda=None, prec=None):
    import torch

    m, n = Ah.shape
    o = _outputs(dev, m, n, k + p)
    omd = torch.from_numpy(om).to(dev)
    pr = cu.make_problem(Ah, k, p, q, 0, *o, omega=omd, lda=lda, prec=prec)
    st, info = cu.cor_utv_host(pr, opts, panel_rows)
    cu.check(st, "cor_utv_host")
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in o], info


@pytest.mark.parametrize("m,n,k,p,q,panel_rows,pinned,fused", [
    (20000, 600, 20, 4, 2, 3000, True, False),   # 7 panels of 3072 rows, the last shorter
    (9000, 700, 30, 10, 1, 0, True, False),      # default panels: one panel
    (30000, 1000, 8, 4, 2, 4096, True, True),    # fused power step: q + 2 streams of A
    (6000, 500, 16, 8, 0, 1000, False, False),   # pageable memory, q = 0, panels of 1024
])
def test_host_f64_matches_oracle(cu, dev, orc, m, n, k, p, q, panel_rows, pinned, fused):
    import torch

    a, _ = I.lowrank(m, n, np.exp(-np.arange(1, n + 1) / 30.0), seed=m + 11)
    om = I.gaussian_omega(n, k + p, 81)
    Ah = torch.from_numpy(a)
    if pinned:
        Ah = Ah.pin_memory()
    opts = cu.cor_opts(0, 0, 0, 0, 1 if fused else 0)
    (U, T, V, perm), info = _host_run(cu, dev, Ah, k, p, q, om, panel_rows, opts)
    Ud, Td, Vd, _, _ = cu.decompose(torch.from_numpy(a).to(dev), k, p, q, omega=om, fused=fused)
    torch.cuda.synchronize()
    Td = Td.cpu().numpy()
    ref = orc.cor_utv(a, k, p, q, om)
    mg = orc.metrics(a, U, T, V, k)
    mo = orc.metrics(a, ref["U"], ref["T"], ref["V"], k)
    scale = np.abs(ref["T"]).max()
    dT = np.abs(T - ref["T"]).max() / scale
    dU, dV = np.abs(U - ref["U"]).max(), np.abs(V - ref["V"]).max()
    print(f"[host f64 {m}x{n} l={k + p} q={q} panels {panel_rows} pinned {pinned} fused {fused}] "
          f"d eps_l {abs(mg['err_l'] - mo['err_l']):.1e}; |dT|/|T| {dT:.1e} |dU| {dU:.1e} "
          f"|dV| {dV:.1e}; vs in-HBM |dT| {np.abs(T - Td).max() / scale:.1e}; "
          f"{info.device_ms:.2f} ms")
    assert abs(mg["err_l"] - mo["err_l"]) <= 1e-12
    assert abs(mg["err_k"] - mo["err_k"]) <= 1e-12
    assert mg["orth_u"] <= 1e-13 and mg["orth_v"] <= 1e-13
    assert np.abs(T - Td).max() <= 1e-12 * scale
    if ref["diag"][1] > 1e-8:
        assert np.array_equal(perm, ref["perm"])
        assert dT <= 1e-10 and dU <= 1e-10 and dV <= 1e-10


def test_host_lda_and_formats(cu, dev, orc):
    """lda > n in host memory (a 2-D copy per panel), FP32 and BF16 passes."""
    import torch

    m, n, k, p, q = 7000, 900, 24, 8, 1
    a, _ = I.lowrank(m, n, np.exp(-np.arange(1, n + 1) / 40.0), seed=3)
    om = I.gaussian_omega(n, k + p, 82)
    ref = orc.cor_utv(a, k, p, q, om)
    mo = orc.metrics(a, ref["U"], ref["T"], ref["V"], k)
    for dt, tol in [(torch.float32, 1e-5), (torch.bfloat16, None)]:
        buf = torch.zeros((m, n + 7), dtype=dt).pin_memory()
        buf[:, :n] = torch.from_numpy(a).to(dt)
        (U, T, V, _), _ = _host_run(cu, dev, buf[:, :n], k, p, q, om, 2048, lda=n + 7)
        # the same stored matrix in HBM
        Ad = buf[:, :n].contiguous().to(dev)
        Ud, Td, Vd, _, _ = cu.decompose(Ad, k, p, q, omega=om)
        torch.cuda.synchronize()
        mg = orc.metrics(a, U, T, V, k)
        md = orc.metrics(a, Ud.cpu().numpy(), Td.cpu().numpy(), Vd.cpu().numpy(), k)
        print(f"[host {dt} lda {n + 7}] eps_l host {mg['err_l']:.10e} in-HBM {md['err_l']:.10e} "
              f"oracle {mo['err_l']:.10e}")
        if tol is not None:
            assert abs(mg["err_l"] - mo["err_l"]) <= tol
        else:
            assert mg["err_l"] <= 1.05 * mo["err_l"]
        assert abs(mg["err_l"] - md["err_l"]) <= 1e-6 * md["err_l"]
        assert mg["orth_u"] <= 1e-13 and mg["orth_v"] <= 1e-13


def test_host_rejects_options_it_cannot_stream(cu, dev):
    import torch

    Ah = torch.zeros((3000, 400), dtype=torch.float64).pin_memory()
    o = _outputs(dev, 3000, 400, 12)
    pr = cu.make_problem(Ah, 8, 4, 1, 0, *o)
    for opts in [cu.cor_opts(1, 0, 0, 0), cu.cor_opts(0, 0, cu.COR_M_EXPLICIT, 0),
                 cu.cor_opts(0, 0, 0, cu.COR_ULV)]:
        st, _ = cu.cor_utv_host(pr, opts, 1024)
        assert st == cu.COR_E_INVAL
