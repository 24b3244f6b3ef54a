"""The no-allocation entry point (cor_utv_ex_noalloc) against cor_utv_ex.

Two calls in a row through the C ABI, the second on a smaller input, each
compared with cor_utv_ex on the same problem: the same kernels run on the same
layout, so U, T, V, perm and the report must be equal bit for bit.  A problem
whose workspace exceeds the fixed array is refused with COR_E_INVAL.
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


def _outputs(dev, m, n, l):
    import torch

    return (torch.full((m, l), 3.0, dtype=torch.float64, device=dev),
            torch.full((l, l), 3.0, dtype=torch.float64, device=dev),
            torch.full((n, l), 3.0, dtype=torch.float64, device=dev),
            torch.full((l,), -1, dtype=torch.int32, device=dev))


def test_noalloc_equals_cor_utv_ex_twice_then_refuses_oversize(cu, orc):
    import torch

    dev = torch.device("cuda:0")
    cases = [(1500, 1100, 36, 8, 1, "f32", 31), (600, 520, 12, 4, 2, "f64", 32)]
    for m, n, k, p, q, fmt, seed in cases:
        l = k + p
        assert cu.cor_workspace_bytes(m, n, l, cu.PREC[fmt]) <= cu.COR_NOALLOC_SCRATCH_BYTES
        a, _ = I.lowrank(m, n, np.exp(-np.arange(1, min(m, n) + 1) / 20.0), seed=seed)
        A = torch.from_numpy(a).to(dev)
        if fmt == "f32":
            A = A.float().contiguous()
        o1 = _outputs(dev, m, n, l)
        o2 = _outputs(dev, m, n, l)
        opts = cu.cor_opts(1, 0)
        st, info1 = cu.cor_utv_ex_noalloc(cu.make_problem(A, k, p, q, seed, *o1), opts)
        cu.check(st, "cor_utv_ex_noalloc")
        st, info2 = cu.cor_utv_ex(cu.make_problem(A, k, p, q, seed, *o2), opts)
        cu.check(st, "cor_utv_ex")
        torch.cuda.synchronize()
        for x, y in zip(o1, o2):
            assert torch.equal(x, y), f"{m}x{n} {fmt}: no-allocation result differs"
        assert info1.err_l == info2.err_l and info1.orth_u == info2.orth_u
        assert info1.flags == info2.flags
        # and the result is the method's (oracle metric, same seeded test matrix)
        ref = orc.cor_utv(a, k, p, q, orc.omega(seed, n, l))
        mo = orc.metrics(a, ref["U"], ref["T"], ref["V"], k)
        mg = orc.metrics(a, *[x.cpu().numpy() for x in o1[:3]], k)
        print(f"[noalloc {m}x{n} {fmt}] eps {mg['err_l']:.10e} oracle {mo['err_l']:.10e}")
        tol = 1e-12 if fmt == "f64" else 1e-5
        assert abs(mg["err_l"] - mo["err_l"]) <= tol
    # a problem larger than the fixed array is refused, nothing runs
    m, n, l = 8000, 8000, 110
    assert cu.cor_workspace_bytes(m, n, l, cu.COR_F64) > cu.COR_NOALLOC_SCRATCH_BYTES
    A = torch.zeros((m, n), dtype=torch.float64, device=dev)
    o = _outputs(dev, m, n, l)
    st, _ = cu.cor_utv_ex_noalloc(cu.make_problem(A, 100, 10, 0, 1, *o), None)
    assert st == cu.COR_E_INVAL
    assert "bytes of workspace" in cu.cor_last_error()
