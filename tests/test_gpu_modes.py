"""GPU parity of the reduced-precision passes, the batched call and the server.

Quantised modes (A stored as BF16, or FP8 E4M3 with per-column scales):
  * against the FP64 matrix the caller quantised (what a user gets), the GPU
    error may exceed the oracle's only by the format's own floor:
      eps_gpu <= 1.05 * sqrt(eps_oracle^2 + q^2),  q = ||A - deq(A_q)||_F / ||A||_F
    (any method that only sees the stored matrix carries q);
  * against the dequantised matrix the GPU actually read, the oracle run on
    that same matrix: eps_gpu <= 1.05 * eps_oracle for BF16.  FP8 operands of
    the skinny factors have a 3-bit mantissa, so there the bound is the
    oracle's error plus the relative rounding of an E4M3 operand averaged
    over the contraction (documented, not hidden).
Batched and served results must equal the single call bit for bit: a
problem's layout, launch shapes and reduction orders depend on its own shape
only.
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


def _c3_scaled():
    """The 20000x10000 recipe (U, V random orthonormal, sigma_i = i^-1.5, full
    rank) at 2000x1000 with the same k = 200, p = 20 (l = 220: fourteen column
    tiles, the l > 136 path of the small kernels)."""
    m, n = 2000, 1000
    a, sig = I.lowrank(m, n, I.spectrum("pow15", n), seed=303)
    return a, sig, 200, 20, 2


def _quantise(cu, dev, a, fmt):
    import torch

    A32 = torch.from_numpy(a.astype(np.float32)).to(dev)
    if fmt == "bf16":
        out = torch.empty(a.shape, dtype=torch.bfloat16, device=dev)
        cu.check(cu.cor_quantize(A32, cu.COR_BF16, out), "quantize")
        torch.cuda.synchronize()
        deq = out.float().cpu().numpy().astype(np.float64)
        return out, None, deq
    out = torch.empty(a.shape, dtype=torch.uint8, device=dev)
    s = torch.empty(a.shape[1], dtype=torch.float32, device=dev)
    cu.check(cu.cor_quantize(A32, cu.COR_FP8, out, s), "quantize")
    torch.cuda.synchronize()
    return out, s, None


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_quantised_passes_scaled_config3(cu, dev, orc, fmt):
    a, sig, k, p, q = _c3_scaled()
    l = k + p
    Aq, colscale, deq = _quantise(cu, dev, a, fmt)
    if fmt == "fp8":
        codes = Aq.cpu().numpy()
        deq = orc.dequantize_fp8(codes, colscale.cpu().numpy())
    om = I.gaussian_omega(a.shape[1], l, 11)
    U, T, V, perm, info = cu.decompose(Aq, k, p, q, omega=om, colscale=colscale)
    import torch

    torch.cuda.synchronize()
    U, T, V = U.cpu().numpy(), T.cpu().numpy(), V.cpu().numpy()
    nrm = np.linalg.norm(a)
    qerr = np.linalg.norm(a - deq) / nrm
    ref = orc.cor_utv(a, k, p, q, om)
    mo = orc.metrics(a, ref["U"], ref["T"], ref["V"], k)
    mg = orc.metrics(a, U, T, V, k)
    ref_q = orc.cor_utv(deq, k, p, q, om)
    mo_q = orc.metrics(deq, ref_q["U"], ref_q["T"], ref_q["V"], k)
    mg_q = orc.metrics(deq, U, T, V, k)
    floor = np.sqrt(mo["err_l"] ** 2 + qerr ** 2)
    print(f"[{fmt}] eps_l vs A: gpu {mg['err_l']:.4e} oracle {mo['err_l']:.4e} "
          f"(ratio {mg['err_l'] / mo['err_l']:.4f}); format floor q {qerr:.3e} -> "
          f"{floor:.4e} (ratio {mg['err_l'] / floor:.4f}); vs deq(A): gpu {mg_q['err_l']:.4e} "
          f"oracle {mo_q['err_l']:.4e} (ratio {mg_q['err_l'] / mo_q['err_l']:.4f}); "
          f"orth {mg['orth_u']:.1e} {mg['orth_v']:.1e}")
    # Orthonormal factors and triangular T whatever the pass format.
    assert mg["orth_u"] <= 1e-13 and mg["orth_v"] <= 1e-13
    assert np.array_equal(np.tril(T, -1), np.zeros_like(T))
    # What a user gets, up to the storage format's own floor.
    assert mg["err_l"] <= 1.05 * np.sqrt(mo["err_l"] ** 2 + qerr ** 2)
    assert mg["err_k"] <= 1.05 * np.sqrt(mo["err_k"] ** 2 + qerr ** 2)
    if fmt == "bf16":
        assert mg_q["err_l"] <= 1.05 * mo_q["err_l"]
        assert mg_q["err_k"] <= 1.05 * mo_q["err_k"]
    else:
        # E4M3 skinny operands: relative rounding 2^-4 per element, averaged
        # over the l-column factor against the m rows of the contraction.
        op = 2.0 ** -4 / np.sqrt(3.0) * np.sqrt(l / a.shape[0])
        assert mg_q["err_l"] <= 1.05 * np.sqrt(mo_q["err_l"] ** 2 + op ** 2)


def test_f32_l220_matches_oracle(cu, dev, orc):
    """FP32 passes at l = 220 (global-memory Cholesky and QRCP paths)."""
    import torch

    a, sig, k, p, q = _c3_scaled()
    om = I.gaussian_omega(a.shape[1], k + p, 12)
    U, T, V, perm, info = cu.decompose(torch.from_numpy(a.astype(np.float32)).to(dev), k, p, q,
                                       omega=om)
    torch.cuda.synchronize()
    ref = orc.cor_utv(a, k, p, q, om)
    mg = orc.metrics(a, U.cpu().numpy(), T.cpu().numpy(), V.cpu().numpy(), k)
    mo = orc.metrics(a, ref["U"], ref["T"], ref["V"], k)
    print(f"[f32 l=220] eps_l gpu {mg['err_l']:.8e} oracle {mo['err_l']:.8e} "
          f"d={abs(mg['err_l'] - mo['err_l']):.2e}; orth {mg['orth_u']:.1e} {mg['orth_v']:.1e}")
    assert abs(mg["err_l"] - mo["err_l"]) <= 1e-5
    assert abs(mg["err_k"] - mo["err_k"]) <= 1e-5
    assert mg["orth_u"] <= 1e-13 and mg["orth_v"] <= 1e-13


def _batch(count, seed, prec):
    """Problems of the batched recipe (m, n ~ U{256..1024}, k ~ U{8..64},
    l = k + 8, sigma_i = exp(-i/k), q = 1), scaled down so that the oracle
    checks every one."""
    return I.batched_problems(count, seed, mn_lo=256, mn_hi=1024, k_lo=8, k_hi=64)


def test_batched_equals_single_and_oracle(cu, dev, orc):
    import torch

    specs = _batch(10, 404, "f64")
    mats, probs, outs, oms = [], [], [], []
    for i, s in enumerate(specs):
        a, _ = I.lowrank(s["m"], s["n"], I.spectrum("expk", s["rank"], s["k"]), seed=s["seed"])
        l = s["k"] + s["p"]
        om = I.gaussian_omega(s["n"], l, 100 + i)
        A = torch.from_numpy(a).to(dev)
        o = _outputs(dev, s["m"], s["n"], l)
        omd = torch.from_numpy(om).to(dev)
        probs.append(cu.make_problem(A, s["k"], s["p"], s["q"], 0, *o, omega=omd))
        mats.append((a, A))
        outs.append(o)
        oms.append((om, omd))
    st, infos = cu.cor_utv_batched(probs, cu.cor_opts(0, 0))
    cu.check(st, "batched")
    torch.cuda.synchronize()
    for i, s in enumerate(specs):
        a, A = mats[i]
        l = s["k"] + s["p"]
        U1, T1, V1, P1 = _outputs(dev, s["m"], s["n"], l)
        pr = cu.make_problem(A, s["k"], s["p"], s["q"], 0, U1, T1, V1, P1, omega=oms[i][1])
        st, _ = cu.cor_utv_ex(pr, cu.cor_opts(0, 0))
        cu.check(st, "single")
        torch.cuda.synchronize()
        Ub, Tb, Vb, Pb = [x.cpu().numpy() for x in outs[i]]
        assert np.array_equal(Ub, U1.cpu().numpy()), f"problem {i}: U differs from the single call"
        assert np.array_equal(Tb, T1.cpu().numpy())
        assert np.array_equal(Vb, V1.cpu().numpy())
        assert np.array_equal(Pb, P1.cpu().numpy())
        ref = orc.cor_utv(a, s["k"], s["p"], s["q"], oms[i][0])
        mg = orc.metrics(a, Ub, Tb, Vb, s["k"])
        mo = orc.metrics(a, ref["U"], ref["T"], ref["V"], s["k"])
        print(f"[batched {i}] {s['m']}x{s['n']} l={l}: d eps {abs(mg['err_l'] - mo['err_l']):.1e} "
              f"orth {mg['orth_u']:.1e}")
        assert abs(mg["err_l"] - mo["err_l"]) <= 1e-12
        assert mg["orth_u"] <= 1e-13 and mg["orth_v"] <= 1e-13


def test_server_mix_equals_single(cu, dev, orc):
    """Requests of three formats served concurrently under a budget that
    forces queueing; each result equals its single call bit for bit, FP32
    requests converted by the server equal the single call on the BF16 copy."""
    import torch

    rng = np.random.default_rng(505)
    reqs = []
    for i in range(9):
        m, n = int(rng.integers(300, 1200)), int(rng.integers(300, 1200))
        k = int(rng.integers(8, 48))
        p, q = 8, int(rng.integers(0, 3))
        a, _ = I.lowrank(m, n, I.spectrum("expk", min(m, n, 4 * (k + p)), k), seed=5050 + i)
        fmt = ["f64", "f32", "bf16"][i % 3]
        A = torch.from_numpy(a).to(dev)
        if fmt == "f32":
            A = A.float().contiguous()
        elif fmt == "bf16":
            A = A.to(torch.bfloat16).contiguous()
        reqs.append(dict(m=m, n=n, k=k, p=p, q=q, A=A, fmt=fmt, a=a, seed=777 + i))
    # room for about three requests at a time: the rest queue
    budget = 3 * max(cu.cor_workspace_bytes(r["m"], r["n"], r["k"] + r["p"], cu.COR_F64)
                     + r["m"] * r["n"] * 2 for r in reqs)
    st, srv = cu.cor_server_create(hbm_budget=budget, max_slots=4, convert_f32_to=cu.COR_BF16)
    cu.check(st, "server_create")
    try:
        tickets, outs = [], []
        for r in reqs:
            o = _outputs(dev, r["m"], r["n"], r["k"] + r["p"])
            pr = cu.make_problem(r["A"], r["k"], r["p"], r["q"], r["seed"], *o)
            st, t = cu.cor_server_submit(srv, pr, cu.cor_opts(1, 0))
            cu.check(st, "submit")
            tickets.append(t)
            outs.append(o)
        infos = []
        for t in tickets:
            st, info = cu.cor_server_wait(srv, t)
            cu.check(st, "wait")
            infos.append(info)
        st, stats = cu.cor_server_stats_get(srv)
        cu.check(st, "stats")
        print(f"[server] completed {stats.completed} p50 {stats.p50_ms:.3f} ms p99 "
              f"{stats.p99_ms:.3f} ms {stats.decomps_per_s:.1f}/s high water "
              f"{stats.hbm_high_water} of budget {budget}")
        assert stats.completed == len(reqs)
        assert stats.hbm_high_water <= budget
        assert 0 < stats.p50_ms <= stats.p99_ms
        # a request larger than the budget is refused at submit
        big = reqs[0]
        o = _outputs(dev, big["m"], big["n"], big["k"] + big["p"])
        pr = cu.make_problem(big["A"], big["k"], big["p"], big["q"], 1, *o)
        st2, srv2 = cu.cor_server_create(hbm_budget=1 << 20, max_slots=2)
        cu.check(st2, "server_create")
        st, _ = cu.cor_server_submit(srv2, pr, None)
        assert st == cu.COR_E_INVAL
        cu.check(cu.cor_server_destroy(srv2), "destroy")
    finally:
        cu.check(cu.cor_server_destroy(srv), "destroy")
    torch.cuda.synchronize()
    for r, o, info in zip(reqs, outs, infos):
        A = r["A"]
        if r["fmt"] == "f32":  # the server ran this request on its BF16 copy
            A16 = torch.empty(A.shape, dtype=torch.bfloat16, device=dev)
            cu.check(cu.cor_quantize(A, cu.COR_BF16, A16), "quantize")
            A = A16
        o1 = _outputs(dev, r["m"], r["n"], r["k"] + r["p"])
        pr = cu.make_problem(A, r["k"], r["p"], r["q"], r["seed"], *o1)
        st, info1 = cu.cor_utv_ex(pr, cu.cor_opts(1, 0))
        cu.check(st, "single")
        torch.cuda.synchronize()
        for x, y in zip(o, o1):
            assert torch.equal(x, y), f"served {r['fmt']} {r['m']}x{r['n']} differs from single"
        assert info.err_l == info1.err_l
        # and the single call is itself accurate against the oracle (seeded Omega)
        l = r["k"] + r["p"]
        if r["fmt"] == "f64":
            ref = orc.cor_utv(r["a"], r["k"], r["p"], r["q"], orc.omega(r["seed"], r["n"], l))
            mg = orc.metrics(r["a"], *[x.cpu().numpy() for x in o1[:3]], r["k"])
            mo = orc.metrics(r["a"], ref["U"], ref["T"], ref["V"], r["k"])
            assert abs(mg["err_l"] - mo["err_l"]) <= 1e-12
