"""GPU checks of the split tuner (cor_tune): it measures candidate split
counts of the two passes on the caller's matrix, keeps the fastest, and the
decompositions of the tuned shape still match the oracle; a table written
to JSON and loaded again gives the same plans (bitwise equal results)."""

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


def test_tuned_splits_keep_parity_and_round_trip(cu, orc, tmp_path):
    import torch

    dev = torch.device("cuda:0")
    m, n, k, p, q = 6000, 3000, 40, 8, 1
    a, _ = I.lowrank(m, n, np.exp(-np.arange(1, n + 1) / 40.0), seed=91)
    om = I.gaussian_omega(n, k + p, 92)
    A = torch.from_numpy(a.astype(np.float32)).to(dev)
    omd = torch.from_numpy(om).to(dev)
    assert cu.cor_tune_clear() == cu.COR_OK

    def run():
        o = (torch.empty((m, k + p), dtype=torch.float64, device=dev),
             torch.empty((k + p, k + p), dtype=torch.float64, device=dev),
             torch.empty((n, k + p), dtype=torch.float64, device=dev),
             torch.empty((k + p,), dtype=torch.int32, device=dev))
        st, _ = cu.cor_utv_ex(cu.make_problem(A, k, p, q, 0, *o, omega=omd))
        cu.check(st, "cor_utv_ex")
        torch.cuda.synchronize()
        return [x.cpu().numpy() for x in o]

    U0, T0, V0, _ = run()
    pr = cu.make_problem(A, k, p, q, 0,
                         torch.empty((m, k + p), dtype=torch.float64, device=dev),
                         torch.empty((k + p, k + p), dtype=torch.float64, device=dev),
                         torch.empty((n, k + p), dtype=torch.float64, device=dev), omega=omd)
    st, s_ax, s_atx = cu.cor_tune(pr, 3)
    cu.check(st, "cor_tune")
    print(f"[tune {m}x{n} l={k + p} FP32] s_ax {s_ax} s_atx {s_atx}")
    assert 1 <= s_ax <= 64 and 1 <= s_atx <= 64
    U1, T1, V1, _ = run()
    ref = orc.cor_utv(a, k, p, q, om)
    mo = orc.metrics(a, ref["U"], ref["T"], ref["V"], k)
    for U, T, V in [(U0, T0, V0), (U1, T1, V1)]:
        mg = orc.metrics(a, U, T, V, k)
        assert abs(mg["err_l"] - mo["err_l"]) <= 1e-5
        assert mg["orth_u"] <= 1e-13 and mg["orth_v"] <= 1e-13
    path = tmp_path / "tune.json"
    assert cu.cor_tune_save(str(path)) == cu.COR_OK
    assert cu.cor_tune_clear() == cu.COR_OK
    assert cu.cor_tune_load(str(path)) == cu.COR_OK
    U2, T2, V2, _ = run()
    assert np.array_equal(T1, T2) and np.array_equal(U1, U2) and np.array_equal(V1, V2)
    assert cu.cor_tune_clear() == cu.COR_OK
