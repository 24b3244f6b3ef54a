"""ctypes view of the FP64 CPU oracle (oracle.c) -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark load this module.  The GPU library never imports it and never
falls back to it.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
        os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "oracle.h"))
    ):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-shared",
             "-fPIC", _SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        d = C.POINTER(C.c_double)
        i32 = C.POINTER(C.c_int32)
        _lib.orc_omega.argtypes = [C.c_uint64, C.c_int64, C.c_int32, d]
        _lib.orc_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        _lib.orc_splitmix64.restype = C.c_uint64
        _lib.orc_qr.argtypes = [d, C.c_int64, C.c_int32, C.c_int64, d, d]
        _lib.orc_qrcp.argtypes = [d, C.c_int32, d, d, i32, d]
        _lib.orc_cor_utv.argtypes = [d, C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_int32,
                                     C.c_int32, d, d, d, d, i32, d, d, d, d, d]
        _lib.orc_cor_utv_fmt.argtypes = [d, C.c_int64, C.c_int64, C.c_int64, C.c_int32,
                                         C.POINTER(C.c_float), C.c_int32, C.c_int32, C.c_int32,
                                         d, d, d, d, i32, d]
        _lib.orc_metrics.argtypes = [d, C.c_int64, C.c_int64, C.c_int64, d, d, d, C.c_int32,
                                     C.c_int32, d]
        _lib.orc_gemm_nn.argtypes = [d, C.c_int64, C.c_int64, C.c_int64, d, C.c_int64,
                                     C.c_int64, d]
        _lib.orc_gemm_tn.argtypes = [d, C.c_int64, C.c_int64, C.c_int64, d, C.c_int64,
                                     C.c_int64, d]
        _lib.orc_bf16_from_f32.argtypes = [C.c_float]
        _lib.orc_bf16_from_f32.restype = C.c_uint16
        _lib.orc_fp8_from_f32.argtypes = [C.c_float]
        _lib.orc_fp8_from_f32.restype = C.c_uint8
        _lib.orc_fp8_to_f64.argtypes = [C.c_uint8]
        _lib.orc_fp8_to_f64.restype = C.c_double
        _lib.orc_bf16_to_f64.argtypes = [C.c_uint16]
        _lib.orc_bf16_to_f64.restype = C.c_double
        _lib.orc_quantize_bf16.argtypes = [C.POINTER(C.c_float), C.c_int64, C.c_int64,
                                           C.c_int64, C.POINTER(C.c_uint16)]
        _lib.orc_quantize_fp8.argtypes = [C.POINTER(C.c_float), C.c_int64, C.c_int64,
                                          C.c_int64, C.POINTER(C.c_uint8),
                                          C.POINTER(C.c_float)]
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def omega(seed: int, n: int, l: int) -> np.ndarray:
    out = np.empty((n, l), dtype=np.float64)
    lib().orc_omega(C.c_uint64(seed), n, l, _dp(out))
    return out


def splitmix64(seed: int, index: int) -> int:
    return int(lib().orc_splitmix64(C.c_uint64(seed), C.c_uint64(index)))


def qr(y):
    y = _f64(y)
    r, c = y.shape
    q = np.empty((r, c))
    rr = np.empty((c, c))
    st = lib().orc_qr(_dp(y), r, c, c, _dp(q), _dp(rr))
    if st:
        raise ValueError("orc_qr status %d" % st)
    return q, rr


def qrcp(m):
    m = _f64(m)
    l = m.shape[0]
    qt = np.empty((l, l))
    t = np.empty((l, l))
    perm = np.empty(l, dtype=np.int32)
    gap = np.zeros(1)
    st = lib().orc_qrcp(_dp(m), l, _dp(qt), _dp(t),
                        perm.ctypes.data_as(C.POINTER(C.c_int32)), _dp(gap))
    if st:
        raise ValueError("orc_qrcp status %d" % st)
    return qt, t, perm, float(gap[0])


def cor_utv(a, k: int, p: int, q: int, omega_arr, want_intermediates: bool = False):
    """Run the oracle.  Returns dict(U, T, V, perm, diag[, Q1, Q2, M, R2])."""
    a = _f64(a)
    m, n = a.shape
    l = k + p
    om = _f64(omega_arr)
    if om.shape != (n, l):
        raise ValueError("omega must be n x l")
    U = np.empty((m, l))
    T = np.empty((l, l))
    V = np.empty((n, l))
    perm = np.empty(l, dtype=np.int32)
    diag = np.zeros(4)
    if want_intermediates:
        Q1 = np.empty((m, l)); Q2 = np.empty((n, l)); M = np.empty((l, l)); R2 = np.empty((l, l))
        ptrs = [_dp(Q1), _dp(Q2), _dp(M), _dp(R2)]
    else:
        ptrs = [None, None, None, None]
    st = lib().orc_cor_utv(_dp(a), m, n, n, k, p, q, _dp(om), _dp(U), _dp(T), _dp(V),
                           perm.ctypes.data_as(C.POINTER(C.c_int32)), *ptrs, _dp(diag))
    if st:
        raise ValueError("orc_cor_utv status %d" % st)
    out = dict(U=U, T=T, V=V, perm=perm, diag=diag)
    if want_intermediates:
        out.update(Q1=Q1, Q2=Q2, M=M, R2=R2)
    return out


FMT = {"f64": 0, "f32": 1, "bf16": 2, "fp8": 3}


def cor_utv_fmt(aq, fmt: str, k: int, p: int, q: int, omega_arr, colscale=None):
    """The method with the passes over A read in a storage format (orc_cor_utv_fmt).

    aq: decoded stored values of A (FP8: decoded codes, A = aq diag(colscale)).
    Returns dict(U, T, V, perm, diag)."""
    aq = _f64(aq)
    m, n = aq.shape
    l = k + p
    om = _f64(omega_arr)
    if om.shape != (n, l):
        raise ValueError("omega must be n x l")
    cs = None
    if fmt == "fp8":
        cs_arr = np.ascontiguousarray(colscale, dtype=np.float32)
        cs = cs_arr.ctypes.data_as(C.POINTER(C.c_float))
    U = np.empty((m, l))
    T = np.empty((l, l))
    V = np.empty((n, l))
    perm = np.empty(l, dtype=np.int32)
    diag = np.zeros(4)
    st = lib().orc_cor_utv_fmt(_dp(aq), m, n, n, FMT[fmt], cs, k, p, q, _dp(om), _dp(U),
                               _dp(T), _dp(V), perm.ctypes.data_as(C.POINTER(C.c_int32)),
                               _dp(diag))
    if st:
        raise ValueError("orc_cor_utv_fmt status %d" % st)
    return dict(U=U, T=T, V=V, perm=perm, diag=diag)


def metrics(a, U, T, V, k: int):
    a = _f64(a)
    m, n = a.shape
    l = T.shape[0]
    out = np.zeros(4)
    lib().orc_metrics(_dp(a), m, n, n, _dp(_f64(U)), _dp(_f64(T)), _dp(_f64(V)), l, k, _dp(out))
    return dict(err_l=out[0], err_k=out[1], orth_u=out[2], orth_v=out[3])


def gemm_nn(a, b):
    a = _f64(a); b = _f64(b)
    r, kk = a.shape
    c = b.shape[1]
    out = np.empty((r, c))
    lib().orc_gemm_nn(_dp(a), r, kk, kk, _dp(b), c, c, _dp(out))
    return out


def gemm_tn(a, b):
    a = _f64(a); b = _f64(b)
    r, kk = a.shape
    c = b.shape[1]
    out = np.empty((kk, c))
    lib().orc_gemm_tn(_dp(a), r, kk, kk, _dp(b), c, c, _dp(out))
    return out


def bf16_from_f32(x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32).ravel()
    return np.array([lib().orc_bf16_from_f32(float(v)) for v in x], dtype=np.uint16)


def fp8_from_f32(x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32).ravel()
    return np.array([lib().orc_fp8_from_f32(float(v)) for v in x], dtype=np.uint8)


def fp8_to_f64(codes) -> np.ndarray:
    return np.array([lib().orc_fp8_to_f64(int(c)) for c in np.asarray(codes).ravel()])


def quantize_bf16(a32) -> np.ndarray:
    a32 = np.ascontiguousarray(a32, dtype=np.float32)
    m, n = a32.shape
    out = np.empty((m, n), dtype=np.uint16)
    lib().orc_quantize_bf16(a32.ctypes.data_as(C.POINTER(C.c_float)), m, n, n,
                            out.ctypes.data_as(C.POINTER(C.c_uint16)))
    return out


def quantize_fp8(a32):
    a32 = np.ascontiguousarray(a32, dtype=np.float32)
    m, n = a32.shape
    out = np.empty((m, n), dtype=np.uint8)
    s = np.empty(n, dtype=np.float32)
    lib().orc_quantize_fp8(a32.ctypes.data_as(C.POINTER(C.c_float)), m, n, n,
                           out.ctypes.data_as(C.POINTER(C.c_uint8)),
                           s.ctypes.data_as(C.POINTER(C.c_float)))
    return out, s


def bf16_to_f64(h) -> np.ndarray:
    h = np.asarray(h, dtype=np.uint16)
    return (h.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def dequantize_fp8(codes, colscale) -> np.ndarray:
    table = fp8_to_f64(np.arange(256))
    return table[np.asarray(codes, dtype=np.uint8)] * np.asarray(colscale, dtype=np.float64)[None, :]


def rpca_alm(M, k: int, p: int, q: int, omega_seed: int, lam=None, rho: float = 1.5,
             mubar_ratio: float = 1e7, tol: float = 1e-5, max_iter: int = 100):
    """Robust PCA by ALM with CoR-UTV as the low-rank step (Sec. V, the
    ALM-CoRUTV algorithm; termination and tests of Sec. VI-D), in plain FP64
    numpy around the oracle's CoR-UTV.

    Iteration j (mu_j the penalty):
      B      = M - S_j + Y_j / mu_j
      U T V  = CoR-UTV(B)  (k, l = k + p, q; the same Gaussian test matrix
               every iteration, from the documented stream at omega_seed)
      r      = number of diagonal entries of T greater than delta = 1 / mu_j
      L_j+1  = U[:, :r] (T[:r, :] - delta [I_r 0]) V^T  (the operator C_delta)
      S_j+1  = shrink(M - L_j+1 + Y_j / mu_j, lam / mu_j),
               shrink(x, d) = sgn(x) max(|x| - d, 0)
      Y_j+1  = Y_j + mu_j (M - L_j+1 - S_j+1)
      mu_j+1 = min(rho mu_j, mu_bar)
    until zeta = ||M - L - S||_F / ||M||_F < tol.  Readings (the paper leaves
    them to a cited reference or prints them garbled): C_delta shrinks the r
    kept diagonal entries of T by delta, as the singular value thresholding
    it stands in for shrinks the singular values (the printed form keeps
    U[:, :r] T[:r, :] V^T unshrunk, which on the synthetic L + S matrices
    stalls at a wrong rank); lam = 1/sqrt(max(m, n));
    mu_0 = 1.25 / ||M||_2 with ||M||_2 taken as T_11 of the first
    decomposition (whose input is M itself, S_0 = Y_0 = 0); mu_bar = 1e7 mu_0;
    rho = 1.5; the penalty grows to its cap (the printed max(rho mu_j, mu_bar)
    would jump to the cap at once); the S step uses Y_j.
    Returns dict(L, S, iters, rank, zeta, ranks)."""
    M = _f64(M)
    m, n = M.shape
    l = k + p
    lam = 1.0 / np.sqrt(max(m, n)) if lam is None else lam
    om = omega(omega_seed, n, l)
    nM = np.linalg.norm(M)
    S = np.zeros_like(M)
    Y = np.zeros_like(M)
    mu = None
    mubar = None
    ranks = []
    it = 0
    while True:
        B = M if mu is None else M - S + Y / mu
        out = cor_utv(B, k, p, q, om)
        T = out["T"]
        if mu is None:
            mu = 1.25 / T[0, 0]
            mubar = mu * mubar_ratio
        delta = 1.0 / mu
        r = int(np.sum(np.diag(T) > delta))
        Tr = T[:r, :].copy()
        Tr[np.arange(r), np.arange(r)] -= delta
        L = out["U"][:, :r] @ (Tr @ out["V"].T)
        Z = M - L + Y / mu
        d = lam / mu
        S = np.sign(Z) * np.maximum(np.abs(Z) - d, 0.0)
        R = M - L - S
        Y = Y + mu * R
        zeta = np.linalg.norm(R) / nM
        ranks.append(r)
        it += 1
        mu = min(rho * mu, mubar)
        if zeta < tol or it >= max_iter:
            break
    return dict(L=L, S=S, iters=it, rank=r, zeta=zeta, ranks=ranks)
