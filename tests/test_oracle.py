"""Pins of the FP64 CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: values the
paper prints (Fig. 1), LAPACK routines on tiny inputs, closed forms, exact
recovery, the Eckart-Young optimum and structural invariants.  No test here
needs a GPU.
"""

import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.stats as st

import inputs as I

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig1_noisylowrank1.txt")


def _signfix_qr(y):
    q, r = np.linalg.qr(y)
    s = np.sign(np.diag(r))
    s[s == 0] = 1
    return q * s, r * s[:, None]


# --------------------------------------------------------------------------
# Gaussian test matrix (Alg. 2 / Alg. 3 first step)
# --------------------------------------------------------------------------
def test_splitmix64_reference_output(orc):
    # First output of SplitMix64 started from state 0, as produced by the
    # reference implementation of Steele, Lea & Flood.
    assert orc.splitmix64(0, 0) == 0xE220A8397B1DCDAF


def test_omega_is_standard_gaussian(orc):
    z = orc.omega(12345, 50_000, 20).ravel()
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    assert abs(st.kurtosis(z, fisher=False) - 3.0) < 0.05
    assert st.kstest(z, "norm").pvalue > 1e-4
    # Box-Muller pairs are independent: no correlation between the two halves.
    ev, od = z[0::2], z[1::2]
    assert abs(np.corrcoef(ev, od)[0, 1]) < 5 / np.sqrt(n / 2)


def test_omega_is_counter_based(orc):
    # Element t of the row-major array depends on t only, not on the shape.
    a = orc.omega(7, 30, 4).ravel()
    b = orc.omega(7, 12, 10).ravel()
    assert np.array_equal(a[:120], b[:120])
    c = orc.omega(8, 30, 4).ravel()
    assert not np.array_equal(a, c)


# --------------------------------------------------------------------------
# Orthonormalisation (QR of C1 and C2)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(40, 7), (65, 16), (9, 9), (300, 33)])
def test_qr_matches_lapack(orc, shape):
    y = np.random.default_rng(shape[0]).standard_normal(shape)
    q, r = orc.qr(y)
    q0, r0 = _signfix_qr(y)
    assert np.abs(q - q0).max() < 1e-12
    assert np.abs(r - r0).max() < 1e-12 * np.abs(r0).max()
    assert np.linalg.norm(q.T @ q - np.eye(shape[1])) < 1e-13
    assert np.all(np.diag(r) >= 0)
    assert np.array_equal(np.tril(r, -1), np.zeros_like(r))


def test_qr_rank_deficient(orc):
    rng = np.random.default_rng(3)
    y = rng.standard_normal((50, 4)) @ rng.standard_normal((4, 8))  # rank 4
    q, r = orc.qr(y)
    assert np.linalg.norm(q @ r - y) < 1e-12 * np.linalg.norm(y)
    assert np.linalg.norm(q.T @ q - np.eye(8)) < 1e-12


# --------------------------------------------------------------------------
# QRCP of the compressed matrix
# --------------------------------------------------------------------------
def _graded(l, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((l, l)) * (0.7 ** np.arange(l))[None, rng.permutation(l)]


@pytest.mark.parametrize("l,seed", [(6, 1), (15, 2), (40, 3)])
def test_qrcp_matches_geqp3(orc, l, seed):
    m = _graded(l, seed)
    qt, t, perm, gap = orc.qrcp(m)
    q0, r0, p0 = sla.qr(m, pivoting=True)
    assert gap > 1e-3
    assert np.array_equal(perm, p0)
    s = np.sign(np.diag(r0))
    assert np.abs(t - r0 * s[:, None]).max() < 1e-12 * np.abs(m).max()
    assert np.abs(qt - q0 * s[None, :]).max() < 1e-12


@pytest.mark.parametrize("l,seed", [(5, 11), (24, 12), (64, 13)])
def test_qrcp_invariants(orc, l, seed):
    m = np.random.default_rng(seed).standard_normal((l, l))
    qt, t, perm, _ = orc.qrcp(m)
    assert sorted(perm.tolist()) == list(range(l))
    assert np.array_equal(np.tril(t, -1), np.zeros_like(t))  # exact zeros
    d = np.diag(t)
    assert np.all(d >= 0)
    assert np.all(np.diff(d) <= 1e-12 * d[0])  # |T_jj| non-increasing
    # Businger-Golub dominance: T_jj^2 >= sum_{i=j..c} T_ic^2 for every c > j.
    for j in range(l):
        for c in range(j + 1, l):
            assert d[j] ** 2 >= (t[j : c + 1, c] ** 2).sum() * (1 - 1e-12)
    assert np.linalg.norm(qt.T @ qt - np.eye(l)) < 1e-13
    assert np.linalg.norm(m[:, perm] - qt @ t) < 1e-13 * np.linalg.norm(m)
    # Singular values of T are those of M.
    assert np.allclose(np.linalg.svd(t, compute_uv=False), np.linalg.svd(m, compute_uv=False),
                       rtol=1e-12, atol=1e-14)


def test_qrcp_ties_take_lowest_index(orc):
    m = np.eye(4) * 2.0  # every column has the same norm at step 0
    _, t, perm, gap = orc.qrcp(m)
    assert perm.tolist() == [0, 1, 2, 3]
    assert gap == 0.0
    assert np.allclose(np.diag(t), 2.0)


# --------------------------------------------------------------------------
# Whole method
# --------------------------------------------------------------------------
def _run(orc, a, k, p, q, seed=0, inter=False):
    om = I.gaussian_omega(a.shape[1], k + p, seed)
    return orc.cor_utv(a, k, p, q, om, want_intermediates=inter)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_exact_recovery_when_rank_le_l(orc, q):
    # rank(A) <= l: the sketch captures the whole range, so A = U T V^T exactly.
    a, _ = I.lowrank(120, 90, np.linspace(3, 1, 12), seed=5)
    r = _run(orc, a, 12, 4, q)
    met = orc.metrics(a, r["U"], r["T"], r["V"], 12)
    assert met["err_l"] < 1e-13
    assert met["orth_u"] < 1e-13 and met["orth_v"] < 1e-13


@pytest.mark.parametrize("m,n,q", [(150, 100, 0), (100, 150, 1), (200, 200, 2)])
def test_errors_above_eckart_young_floor(orc, m, n, q):
    a = np.random.default_rng(m + n).standard_normal((m, n)) * (0.93 ** np.arange(n))[None, :]
    k, p = 10, 6
    r = _run(orc, a, k, p, q)
    met = orc.metrics(a, r["U"], r["T"], r["V"], k)
    s = np.linalg.svd(a, compute_uv=False)
    tot = (s ** 2).sum()
    opt_l = np.sqrt((s[k + p :] ** 2).sum() / tot)
    opt_k = np.sqrt((s[k:] ** 2).sum() / tot)
    assert met["err_l"] >= opt_l * (1 - 1e-12)
    assert met["err_k"] >= opt_k * (1 - 1e-12)
    # singular values of T never exceed those of A (interlacing)
    st_ = np.linalg.svd(r["T"], compute_uv=False)
    assert np.all(st_ <= s[: k + p] * (1 + 1e-12))


def test_structure_of_outputs(orc):
    a = np.random.default_rng(9).standard_normal((130, 70))
    r = _run(orc, a, 8, 5, 1, inter=True)
    l = 13
    assert r["U"].shape == (130, l) and r["V"].shape == (70, l) and r["T"].shape == (l, l)
    assert np.array_equal(np.tril(r["T"], -1), np.zeros((l, l)))
    assert np.all(np.diag(r["T"]) >= 0)
    assert np.linalg.norm(r["U"].T @ r["U"] - np.eye(l)) < 1e-13
    assert np.linalg.norm(r["V"].T @ r["V"] - np.eye(l)) < 1e-13
    # V = Q2 P (columns of Q2 in pivot order)
    assert np.array_equal(r["V"], r["Q2"][:, r["perm"]])


def test_metrics_identity_with_exact_compression(orc):
    # With M = Q1^T A Q2 formed explicitly, T = U^T A V, hence
    # ||A - U T V^T||_F^2 = ||A||_F^2 - ||T||_F^2 (Pythagoras on projections).
    a = np.random.default_rng(4).standard_normal((90, 60)) * (0.9 ** np.arange(60))[None, :]
    r = _run(orc, a, 6, 4, 1)
    met = orc.metrics(a, r["U"], r["T"], r["V"], 6)
    na2 = (a ** 2).sum()
    ident = np.sqrt(max(0.0, 1 - (r["T"] ** 2).sum() / na2))
    assert abs(met["err_l"] - ident) < 1e-12
    assert np.allclose(r["T"], r["U"].T @ a @ r["V"], atol=1e-13)


def test_compression_equals_r2_transpose_and_d_approx(orc):
    # Alg. 2 as printed (q = 0): C1 = A Psi, C2 = A^T C1, QR of both, explicit
    # D = Q1^T A Q2 and the single-pass D_approx = Q1^T C1 (Q2^T Psi)^+.
    # The oracle instead forms C2 = A^T Q1.  Closed forms: Q2 is the same,
    # D = D_approx = R1^-T R2'^T and D = R2^T (R2 of A^T Q1).
    rng = np.random.default_rng(21)
    a = rng.standard_normal((80, 60)) * (0.85 ** np.arange(60))[None, :]
    k, p = 6, 4
    om = I.gaussian_omega(60, k + p, 3)
    r = orc.cor_utv(a, k, p, 0, om, want_intermediates=True)
    c1 = a @ om
    c2 = a.T @ c1
    q1, r1 = _signfix_qr(c1)
    q2, r2p = _signfix_qr(c2)
    d = q1.T @ a @ q2
    d_approx = q1.T @ c1 @ np.linalg.pinv(q2.T @ om)
    assert np.abs(r["Q1"] - q1).max() < 1e-10
    assert np.abs(r["Q2"] - q2).max() < 1e-8
    scale = np.abs(d).max()
    assert np.abs(r["M"] - d).max() < 1e-9 * scale
    assert np.abs(d_approx - d).max() < 1e-9 * scale
    assert np.abs(np.linalg.solve(r1.T, r2p.T) - d).max() < 1e-9 * scale
    assert np.abs(r["M"] - r["R2"].T).max() < 1e-12 * scale
    assert r["diag"][0] < 1e-13


@pytest.mark.parametrize("q", [1, 2])
def test_power_loop_matches_literal_alg3(orc, q):
    # Alg. 3 as printed: C2 = Psi; q + 1 times C1 = A C2, C2 = A^T C1 (no QR
    # inside the loop); then QR of C1 and C2, D = Q1^T A Q2 and the single-pass
    # D_approx = Q1^T C1 (Q2^T C2_old)^+ with the C2 that produced the last C1.
    # On a well-conditioned matrix (singular values in [1, 3]) the loop
    # without re-orthonormalisation loses nothing, so the oracle's form
    # (orthonormalise after every product, second sketch A^T Q1) must give
    # the same sign-fixed Q1, Q2, the same D and the same T.
    rng = np.random.default_rng(70 + q)
    m, n, k, p = 40, 30, 4, 2
    l = k + p
    sig = np.linspace(3.0, 1.0, n)
    u, _ = np.linalg.qr(rng.standard_normal((m, n)))
    v, _ = np.linalg.qr(rng.standard_normal((n, n)))
    a = (u * sig) @ v.T
    om = I.gaussian_omega(n, l, 40 + q)
    c2 = om.copy()
    for _ in range(q + 1):
        c2_old = c2
        c1 = a @ c2
        c2 = a.T @ c1
    q1, _ = _signfix_qr(c1)
    q2, _ = _signfix_qr(c2)
    d = q1.T @ a @ q2
    d_approx = q1.T @ c1 @ np.linalg.pinv(q2.T @ c2_old)
    r = orc.cor_utv(a, k, p, q, om, want_intermediates=True)
    assert np.abs(r["Q1"] - q1).max() < 1e-10
    assert np.abs(r["Q2"] - q2).max() < 1e-10
    assert np.abs(r["M"] - d).max() < 1e-10 * np.abs(d).max()
    assert np.abs(d_approx - d).max() < 1e-10 * np.abs(d).max()
    # T of the QRCP of the literal D (LAPACK geqp3, sign-fixed)
    qd, td, pd = sla.qr(d, pivoting=True)
    td = td * np.sign(np.diag(td))[:, None]
    assert np.array_equal(r["perm"], pd)
    assert np.abs(r["T"] - td).max() < 1e-10 * np.abs(td).max()


def test_err_k_closed_form(orc):
    # With M = Q1^T A Q2 formed explicitly, U^T A V = T, so the rank-k
    # truncation U[:, :k] T[:k, :] V^T = P_k A P_V (P_k the projector on the
    # first k columns of U, P_V on V) and, by Pythagoras,
    # ||A - U[:, :k] T[:k, :] V^T||_F^2 = ||A||_F^2 - ||T[:k, :]||_F^2.
    # The test matrix makes the k x (l - k) block T[:k, k:] large enough that
    # truncating to T[:k, :k] instead would fail by a wide margin.
    a, _ = I.lowrank(300, 200, 1.0 / np.arange(1, 201) ** 0.5, seed=31)
    k, p = 10, 15
    r = _run(orc, a, k, p, 0, seed=6)
    met = orc.metrics(a, r["U"], r["T"], r["V"], k)
    na2 = (a ** 2).sum()
    t = r["T"]
    closed = np.sqrt(1.0 - (t[:k, :] ** 2).sum() / na2)
    wrong = np.sqrt(1.0 - (t[:k, :k] ** 2).sum() / na2)
    assert abs(met["err_k"] - closed) < 1e-12
    assert abs(wrong - closed) > 1e4 * 1e-12
    # and the rank-l error by the same identity with all of T
    assert abs(met["err_l"] - np.sqrt(1.0 - (t ** 2).sum() / na2)) < 1e-12


def _torch_operand(x, fmt, rowscale=None):
    """Decoded operand and column scales of a stored-format pass, from torch's
    own format conversions (independent of the oracle's)."""
    import torch

    if rowscale is not None:
        x = x * rowscale[:, None]
    xf = x.astype(np.float32)
    if fmt == "bf16":
        return torch.from_numpy(xf).to(torch.bfloat16).double().numpy(), np.ones(x.shape[1])
    mx = np.abs(xf).max(axis=0)
    t = np.where(mx > 0, mx / np.float32(448.0), np.float32(1.0)).astype(np.float32)
    y = np.clip(xf / t[None, :], -448.0, 448.0).astype(np.float32)
    dec = torch.from_numpy(y).to(torch.float8_e4m3fn).double().numpy()
    return dec, t.astype(np.float64)


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_stored_format_passes_match_torch_conversions(orc, fmt):
    # q = 0: span(U) = span(Aq Xq diag(t)) and span(V) = span of the second
    # sketch diag(s) Aq^T Q1q diag(t), with the operands quantised by torch.
    rng = np.random.default_rng(5 if fmt == "bf16" else 6)
    m, n, k, p = 60, 40, 4, 2
    l = k + p
    a = rng.standard_normal((m, n)) * (0.8 ** np.arange(n))[None, :]
    a32 = a.astype(np.float32)
    if fmt == "bf16":
        aq = orc.bf16_to_f64(orc.quantize_bf16(a32))
        cs = None
        rs = None
    else:
        codes, cs = orc.quantize_fp8(a32)
        aq = orc.fp8_to_f64(codes).reshape(codes.shape)
        rs = cs.astype(np.float64)
    om = I.gaussian_omega(n, l, 9)
    r = orc.cor_utv_fmt(aq, fmt, k, p, 0, om, colscale=cs)
    xq, t = _torch_operand(om, fmt, rs)
    q1, _ = _signfix_qr(aq @ xq * t[None, :])
    assert np.abs(r["U"] @ r["U"].T - q1 @ q1.T).max() < 1e-12
    q1q, t1 = _torch_operand(q1, fmt)
    y2 = aq.T @ q1q * t1[None, :]
    if rs is not None:
        y2 = y2 * rs[:, None]
    q2, _ = _signfix_qr(y2)
    assert np.abs(r["V"] @ r["V"].T - q2 @ q2.T).max() < 1e-12
    # the operand rounding is really there: FP64 passes give another span
    r64 = orc.cor_utv(aq * (rs[None, :] if rs is not None else 1.0), k, p, 0, om)
    assert np.abs(r64["U"] @ r64["U"].T - q1 @ q1.T).max() > 1e-6


def test_stored_format_fp64_is_the_plain_method(orc):
    a = np.random.default_rng(8).standard_normal((70, 50))
    om = I.gaussian_omega(50, 9, 2)
    r = orc.cor_utv(a, 6, 3, 1, om)
    f = orc.cor_utv_fmt(a, "f64", 6, 3, 1, om)
    for key in ("U", "T", "V", "perm"):
        assert np.array_equal(r[key], f[key])


def test_power_iteration_improves_accuracy(orc):
    # Slowly decaying spectrum: q = 1 beats q = 0, and q = 2 gives a rank-k
    # error within 1% of the optimum (Sec. VI-B observations).
    a, sig = I.lowrank(400, 300, 1.0 / np.sqrt(np.arange(1, 301)), seed=11)
    k, p = 20, 5
    errs = []
    for q in (0, 1, 2):
        r = _run(orc, a, k, p, q, seed=4)
        errs.append(orc.metrics(a, r["U"], r["T"], r["V"], k))
    assert errs[1]["err_l"] < errs[0]["err_l"]
    assert errs[2]["err_l"] <= errs[1]["err_l"] * 1.001
    tot = (sig ** 2).sum()
    opt_k = np.sqrt((sig[k:] ** 2).sum() / tot)
    assert errs[2]["err_k"] < 1.01 * opt_k


def test_rejects_invalid_arguments(orc):
    a = np.zeros((20, 10))
    with pytest.raises(ValueError):
        orc.cor_utv(a, 8, 2, 0, np.zeros((10, 10)))  # l = 10 = min(m, n)
    with pytest.raises(ValueError):
        orc.cor_utv(a, 0, 3, 0, np.zeros((10, 3)))  # k < 1
    with pytest.raises(ValueError):
        orc.cor_utv(a, 1, 0, 0, np.zeros((10, 1)))  # l < 2


def test_zero_matrix_is_handled(orc):
    a = np.zeros((30, 20))
    r = _run(orc, a, 3, 2, 1)
    assert np.all(r["T"] == 0)
    assert np.linalg.norm(r["U"].T @ r["U"] - np.eye(5)) < 1e-13


# --------------------------------------------------------------------------
# Fig. 1: the only printed output of the method itself
# --------------------------------------------------------------------------
def test_fig1_noisylowrank1_diagonal_of_T(orc):
    tab = np.loadtxt(GOLDEN)
    j, cor, svd = tab[:, 0].astype(int), tab[:, 1], tab[:, 2]
    a = I.noisy_lowrank(0.01, seed=1)
    s = np.linalg.svd(a, compute_uv=False)
    # The construction reproduces the printed SVD curve.
    assert np.all(np.abs(s[:20] - svd[:20]) / svd[:20] < 5e-3)
    assert np.all(np.abs(s[20:40] - svd[20:40]) / svd[20:40] < 5e-2)
    k, l = 20, 40
    acc = np.zeros(l)
    for trial in range(20):
        om = I.gaussian_omega(1000, l, 100 + trial)
        r = orc.cor_utv(a, k, l - k, 0, om)
        acc += np.abs(np.diag(r["T"]))
    mean = acc / 20
    rel = np.abs(mean - cor) / cor
    assert np.all(rel[:20] < 0.01), rel[:20]
    assert np.all(rel[20:] < 0.05), rel[20:]
    # The gap at j = k is revealed: T_21,21 / T_20,20 ~ 7e-3.
    assert mean[20] / mean[19] < 0.02


# --------------------------------------------------------------------------
# Storage formats of the reduced-precision modes
# --------------------------------------------------------------------------
def test_bf16_rounding_matches_torch(orc):
    import torch

    rng = np.random.default_rng(1)
    x = np.concatenate([
        rng.standard_normal(2000).astype(np.float32) * np.float32(1e3),
        # exact ties: bf16 value + half an ulp
        (np.arange(1, 200, dtype=np.uint32) << 16 | 0x8000).view(np.float32),
        (np.arange(0x3F80, 0x3FA0, dtype=np.uint32) << 16 | 0x8000).view(np.float32),
        np.array([0.0, -0.0, 3.4e38, -3.4e38, 1e-40, 65504.0], dtype=np.float32),
    ])
    ours = orc.bf16_from_f32(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)


def test_fp8_e4m3fn_format(orc):
    import torch

    # Decoding table: fixed points of the OCP E4M3FN format.
    assert orc.fp8_to_f64([0x7E])[0] == 448.0
    assert orc.fp8_to_f64([0x38])[0] == 1.0
    assert orc.fp8_to_f64([0x08])[0] == 2.0 ** -6
    assert orc.fp8_to_f64([0x01])[0] == 2.0 ** -9
    assert orc.fp8_to_f64([0xFE])[0] == -448.0
    assert np.isnan(orc.fp8_to_f64([0x7F])[0])
    rng = np.random.default_rng(2)
    x = np.concatenate([
        (rng.standard_normal(3000) * 50).astype(np.float32),
        (rng.standard_normal(500) * 1e-2).astype(np.float32),
        np.array([0.0, 448.0, -448.0, 2.0 ** -10, 1.0625, 1.1875, 240.0], dtype=np.float32),
    ])
    x = x[np.abs(x) <= 448]
    ours = orc.fp8_from_f32(x)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(ours, ref)
    # Saturation beyond the largest finite value.
    assert orc.fp8_from_f32(np.array([1e4, -500.0], dtype=np.float32)).tolist() == [0x7E, 0xFE]


def test_fp8_columnwise_quantisation(orc):
    rng = np.random.default_rng(5)
    a = (rng.standard_normal((40, 12)) * np.logspace(-3, 2, 12)[None, :]).astype(np.float32)
    a[:, 3] = 0.0
    codes, s = orc.quantize_fp8(a)
    assert s[3] == 1.0 and np.all(codes[:, 3] == 0)
    colmax = np.abs(a).max(axis=0)
    nz = colmax > 0
    assert np.array_equal(s[nz], (colmax[nz] / np.float32(448)).astype(np.float32))
    deq = orc.dequantize_fp8(codes, s)
    # E4M3 has a 3-bit mantissa: relative error <= 2^-4 for normal values.
    big = np.abs(a) > s[None, :] * 2.0 ** -6
    assert np.all(np.abs(deq - a)[big] <= np.abs(a)[big] * 2.0 ** -4 * (1 + 1e-6))
    # each column's largest element maps to the largest code
    assert np.all(np.abs(deq).max(axis=0)[nz] == pytest.approx(colmax[nz], rel=1e-6))
