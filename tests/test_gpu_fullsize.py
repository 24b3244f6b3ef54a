"""GPU results at the full sizes of the benchmark workloads against stored
oracle results.

The oracle needs minutes at these sizes, so tests/golden/make_oracle_golden.py
ran it once on the host (it calls only the oracle and the seeded input
generators) and stored its errors, QRCP permutation, diag(T) and sampled rows
of U and V.  The device builds the same matrices from the same seeded
Gaussians (its QR and products differ from the host's by rounding only; the
stored fingerprint confirms it), and the decomposition draws the same test
matrix from the documented counter-based stream (device twin of the oracle's
generator, equal to a few ulp).

Rules (relative Frobenius errors against the FP64 matrix):
  FP64 : |eps_gpu - eps_oracle| <= 1e-12 (eps_l and eps_k), orthogonality
         <= 1e-13, permutation and factors elementwise (pivot gap > 1e-8)
  FP32 : |eps_gpu - eps_oracle| <= 1e-5
  BF16 : eps_gpu <= 1.05 eps_oracle; and within 5 % of the oracle's stored-
         format run (same storage, exact products) both ways
  FP8  : within 5 % of the oracle's stored-format run both ways; against the
         FP64 oracle the E4M3 storage noise exceeds sigma_l at this size, so
         the 1.05x rule is not met (recorded as an expected failure)
"""

import json
import os

import numpy as np
import pytest

import inputs as I

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated")
    with open(path) as f:
        return json.load(f)


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


def _build(name, dev, gold):
    import torch

    print(f"[build] {name} on the device", flush=True)
    a, sig = I.config_matrix(name, backend="torch", device=dev)
    torch.cuda.synchronize()
    fp = gold["fingerprint"]
    fro = float(torch.linalg.norm(a))
    row0 = a[0, :6].cpu().numpy()
    tail = a[-1, -6:].cpu().numpy()
    cs = a[:, :4].sum(dim=0).cpu().numpy()
    d = max(abs(fro - fp["fro"]) / fp["fro"],
            np.abs(row0 - fp["row0_head"]).max() / np.abs(fp["row0_head"]).max(),
            np.abs(tail - fp["last_row_tail"]).max() / np.abs(fp["last_row_tail"]).max(),
            np.abs(cs - fp["col_sums_head"]).max() / np.abs(fp["col_sums_head"]).max())
    print(f"[build] {name}: fingerprint relative difference {d:.2e}", flush=True)
    assert d <= 1e-11, "the device matrix is not the one the oracle saw"
    return a, sig


@pytest.fixture(scope="module")
def c3(dev):
    gold = _golden("c3_oracle.json")
    a, sig = _build("c3", dev, gold)
    yield a, gold
    del a


@pytest.fixture(scope="module")
def c2(dev):
    gold = _golden("c2_oracle.json")
    a, sig = _build("c2", dev, gold)
    yield a, gold
    del a


def _errors(a64, U, T, V, k):
    """eps_l, eps_k and orthogonality of a device result against the device
    FP64 matrix (plain FP64 products; the same definitions as the oracle's
    metric routine)."""
    import torch

    l = T.shape[0]
    nA = torch.linalg.norm(a64)
    W = T @ V.T
    err_l = float(torch.linalg.norm(a64 - U @ W) / nA)
    err_k = float(torch.linalg.norm(a64 - U[:, :k] @ W[:k]) / nA)
    eye = torch.eye(l, dtype=torch.float64, device=U.device)
    orth_u = float(torch.linalg.norm(U.T @ U - eye))
    orth_v = float(torch.linalg.norm(V.T @ V - eye))
    return dict(err_l=err_l, err_k=err_k, orth_u=orth_u, orth_v=orth_v)


def _run(cu, A, gold, colscale=None, report=True):
    import torch

    k, p, q = gold["k"], gold["p"], gold["q"]
    U, T, V, perm, info = cu.decompose(A, k, p, q, seed=gold["omega_seed"], colscale=colscale,
                                       report=report)
    torch.cuda.synchronize()
    return U, T, V, perm, info


def _quantise(cu, dev, a64, fmt):
    import torch

    A32 = a64.float().contiguous()
    if fmt == "f32":
        return A32, None
    if fmt == "bf16":
        out = torch.empty(A32.shape, dtype=torch.bfloat16, device=dev)
        cu.check(cu.cor_quantize(A32, cu.COR_BF16, out), "quantize")
        del A32
        return out, None
    out = torch.empty(A32.shape, dtype=torch.uint8, device=dev)
    s = torch.empty(A32.shape[1], dtype=torch.float32, device=dev)
    cu.check(cu.cor_quantize(A32, cu.COR_FP8, out, s), "quantize")
    del A32
    return out, s


def _check_f64(cu, a64, gold, tag):
    U, T, V, perm, info = _run(cu, a64, gold)
    e = _errors(a64, U, T, V, gold["k"])
    dl, dk = abs(e["err_l"] - gold["err_l"]), abs(e["err_k"] - gold["err_k"])
    Tn = T.cpu().numpy()
    dT = np.abs(np.diag(Tn) - np.asarray(gold["T_diag"])).max() / max(gold["T_diag"])
    Un, Vn = U.cpu().numpy(), V.cpu().numpy()
    dU = max(np.abs(Un[int(i)] - np.asarray(r)).max() for i, r in gold["U_rows"].items())
    dV = max(np.abs(Vn[int(i)] - np.asarray(r)).max() for i, r in gold["V_rows"].items())
    dR = np.abs(Tn[0] - np.asarray(gold["T_row0"])).max() / max(gold["T_diag"])
    print(f"[{tag} f64] eps_l {e['err_l']:.15e} (oracle {gold['err_l']:.15e}, d {dl:.1e}); "
          f"eps_k d {dk:.1e}; orth {e['orth_u']:.1e} {e['orth_v']:.1e}; "
          f"report eps_l {info.err_l:.6e} eps_k {info.err_k:.6e}; max |d diag T| {dT:.1e}, "
          f"|d T row0| {dR:.1e}, |dU| {dU:.1e}, |dV| {dV:.1e}", flush=True)
    assert dl <= 1e-12 and dk <= 1e-12
    assert e["orth_u"] <= 1e-13 and e["orth_v"] <= 1e-13
    assert abs(info.err_l ** 2 - e["err_l"] ** 2) <= 1e-14 + 1e-11 * e["err_l"] ** 2
    assert abs(info.err_k ** 2 - e["err_k"] ** 2) <= 1e-14 + 1e-11 * e["err_k"] ** 2
    assert abs(info.orth_u - e["orth_u"]) <= 1e-13 and abs(info.orth_v - e["orth_v"]) <= 1e-13
    assert np.array_equal(np.tril(Tn, -1), np.zeros_like(Tn))
    assert gold["min_pivot_gap"] > 1e-8  # the factors are unique: compare them
    assert np.array_equal(perm.cpu().numpy(), np.asarray(gold["perm"]))
    assert dT <= 1e-10 and dR <= 1e-10
    assert dU <= 1e-10 and dV <= 1e-10


def test_c3_f64_matches_stored_oracle(cu, dev, c3):
    """20000 x 10000, sigma_i = i^-1.5, k = 200, l = 220, q = 2 in FP64."""
    a64, gold = c3
    _check_f64(cu, a64, gold, "c3")


def test_c2_f64_matches_stored_oracle(cu, dev, c2):
    """8000 x 8000 rank 500, sigma_i = exp(-i/40), k = 100, l = 110, q = 2 in FP64."""
    a64, gold = c2
    _check_f64(cu, a64, gold, "c2")


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_f32_full_size_matches_stored_oracle(cu, dev, c2, c3, name):
    a64, gold = {"c2": c2, "c3": c3}[name]
    A32, _ = _quantise(cu, dev, a64, "f32")
    U, T, V, perm, info = _run(cu, A32, gold)
    del A32
    e = _errors(a64, U, T, V, gold["k"])
    dl, dk = abs(e["err_l"] - gold["err_l"]), abs(e["err_k"] - gold["err_k"])
    print(f"[{name} f32] eps_l {e['err_l']:.10e} (oracle {gold['err_l']:.10e}, d {dl:.1e}); "
          f"eps_k d {dk:.1e}; orth {e['orth_u']:.1e} {e['orth_v']:.1e}", flush=True)
    assert dl <= 1e-5 and dk <= 1e-5
    assert e["orth_u"] <= 1e-13 and e["orth_v"] <= 1e-13


_RESULTS = {}


def _quantised(cu, dev, c3, fmt):
    if fmt in _RESULTS:
        return _RESULTS[fmt]
    a64, gold = c3
    gq = _golden(f"c3_oracle_{fmt}.json")
    Aq, cs = _quantise(cu, dev, a64, fmt)
    U, T, V, perm, info = _run(cu, Aq, gold, colscale=cs)
    del Aq
    e = _errors(a64, U, T, V, gold["k"])
    r64 = e["err_l"] / gold["err_l"]
    rk64 = e["err_k"] / gold["err_k"]
    rq = e["err_l"] / gq["err_l"]
    rkq = e["err_k"] / gq["err_k"]
    print(f"[c3 {fmt}] eps_l {e['err_l']:.6e}: / FP64 oracle {r64:.4f}, / stored-format oracle "
          f"{rq:.4f} (format's own error {gq['format_error']:.2e}); eps_k / FP64 oracle "
          f"{rk64:.4f}, / stored-format {rkq:.4f}; orth {e['orth_u']:.1e} {e['orth_v']:.1e}",
          flush=True)
    assert e["orth_u"] <= 1e-13 and e["orth_v"] <= 1e-13
    assert np.array_equal(np.tril(T.cpu().numpy(), -1), np.zeros((gold["k"] + gold["p"],) * 2))
    _RESULTS[fmt] = (e, gold, gq)
    return e, gold, gq


def test_c3_bf16_within_rule(cu, dev, c3):
    e, gold, gq = _quantised(cu, dev, c3, "bf16")
    assert e["err_l"] <= 1.05 * gold["err_l"]
    assert e["err_k"] <= 1.05 * gold["err_k"]
    assert abs(e["err_l"] / gq["err_l"] - 1.0) <= 0.05
    assert abs(e["err_k"] / gq["err_k"] - 1.0) <= 0.05


def test_c3_fp8_matches_stored_format_oracle(cu, dev, c3):
    e, gold, gq = _quantised(cu, dev, c3, "fp8")
    assert abs(e["err_l"] / gq["err_l"] - 1.0) <= 0.05
    assert abs(e["err_k"] / gq["err_k"] - 1.0) <= 0.05


@pytest.mark.xfail(reason="E4M3 storage noise (about 3 % of each entry) has a spectral norm above "
                          "sigma_220 of the 20000 x 10000 matrix: the error of any method that "
                          "reads only the FP8 matrix is several times the FP64 oracle's",
                   strict=True)
def test_c3_fp8_within_fp64_rule(cu, dev, c3):
    e, gold, gq = _quantised(cu, dev, c3, "fp8")
    assert e["err_l"] <= 1.05 * gold["err_l"]
