"""Python binding of libcorutv (CoR-UTV on MI355X / gfx950).

Argument marshalling only: every step of the decomposition runs in the HIP
kernels of ``libcorutv.so``.  PyTorch provides device memory and streams.
The names mirror the C ABI of ``include/cor_utv.h``.  Importing this module
fails loudly if the library has not been built (``python -m
paper_1810_07323_amd.build``); there is no CPU fallback.
"""

from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcorutv.so")

COR_OK, COR_E_INVAL, COR_E_NOMEM, COR_E_DEVICE, COR_E_NUMERIC, COR_E_BUSY, COR_E_NOTFOUND = range(7)
COR_F64, COR_F32, COR_BF16, COR_FP8 = range(4)
COR_FLAG_RANK_DEFICIENT, COR_FLAG_NONFINITE, COR_FLAG_SYNC_TIMEOUT = 2, 4, 8
COR_NOALLOC_SCRATCH_BYTES = 64 << 20
COR_M_R2T, COR_M_EXPLICIT, COR_M_APPROX = 0, 1, 2
COR_URV, COR_ULV = 0, 1
PREC = {"f64": COR_F64, "f32": COR_F32, "bf16": COR_BF16, "fp8": COR_FP8}


class cor_info(C.Structure):
    _fields_ = [("err_l", C.c_double), ("err_k", C.c_double), ("orth_u", C.c_double),
                ("orth_v", C.c_double), ("device_ms", C.c_double), ("flags", C.c_int32),
                ("l", C.c_int32), ("m_check", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class cor_problem(C.Structure):
    _fields_ = [("A", C.c_void_p), ("colscale", C.c_void_p), ("m", C.c_int64), ("n", C.c_int64),
                ("lda", C.c_int64), ("k", C.c_int32), ("p", C.c_int32), ("q", C.c_int32),
                ("prec", C.c_int32), ("seed", C.c_uint64), ("omega", C.c_void_p),
                ("U", C.c_void_p), ("T", C.c_void_p), ("V", C.c_void_p), ("perm", C.c_void_p)]


class cor_opts(C.Structure):
    _fields_ = [("report", C.c_int32), ("cholqr2_all", C.c_int32), ("compress", C.c_int32),
                ("orient", C.c_int32), ("fused_power", C.c_int32)]


class cor_rpca_opts(C.Structure):
    _fields_ = [("k", C.c_int32), ("p", C.c_int32), ("q", C.c_int32), ("prec", C.c_int32),
                ("seed", C.c_uint64), ("lam", C.c_double), ("rho", C.c_double),
                ("mu_bar_ratio", C.c_double), ("tol", C.c_double), ("max_iter", C.c_int32)]


class cor_rpca_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("rank", C.c_int32), ("zeta", C.c_double),
                ("mu", C.c_double), ("ms", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class cor_server_cfg(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("max_slots", C.c_int32),
                ("convert_f32_to", C.c_int32)]


class cor_server_stats(C.Structure):
    _fields_ = [("p50_ms", C.c_double), ("p99_ms", C.c_double), ("mean_ms", C.c_double),
                ("decomps_per_s", C.c_double), ("completed", C.c_int64), ("queued", C.c_int64),
                ("active", C.c_int64), ("rejected", C.c_int64), ("hbm_in_use", C.c_size_t),
                ("hbm_high_water", C.c_size_t)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# Every symbol the header declares, with its ctypes signature.
_P = C.c_void_p
_SIGS = {
    "cor_utv": (C.c_int, [_P, C.c_int64, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_uint64,
                          C.c_int32, _P, _P, _P, C.POINTER(cor_info), _P]),
    "cor_utv_ex": (C.c_int, [C.POINTER(cor_problem), C.POINTER(cor_opts), C.POINTER(cor_info), _P]),
    "cor_utv_ex_noalloc": (C.c_int, [C.POINTER(cor_problem), C.POINTER(cor_opts),
                                     C.POINTER(cor_info), _P]),
    "cor_tune": (C.c_int, [C.POINTER(cor_problem), C.c_int32, C.POINTER(C.c_int32),
                           C.POINTER(C.c_int32), _P]),
    "cor_tune_save": (C.c_int, [C.c_char_p]),
    "cor_tune_load": (C.c_int, [C.c_char_p]),
    "cor_tune_clear": (C.c_int, []),
    "cor_utv_host": (C.c_int, [C.POINTER(cor_problem), C.POINTER(cor_opts), C.c_int64,
                               C.POINTER(cor_info), _P]),
    "cor_utv_batched": (C.c_int, [C.POINTER(cor_problem), C.c_int32, C.POINTER(cor_opts),
                                  C.POINTER(cor_info), _P]),
    "cor_rpca_alm": (C.c_int, [_P, C.c_int64, C.c_int64, C.c_int64, C.POINTER(cor_rpca_opts),
                               _P, _P, C.POINTER(cor_rpca_info), _P]),
    "cor_plan_create": (C.c_int, [C.POINTER(cor_problem), C.c_int32, C.POINTER(cor_opts),
                                  C.POINTER(_P)]),
    "cor_plan_run": (C.c_int, [_P, _P]),
    "cor_plan_capture": (C.c_int, [_P, _P]),
    "cor_plan_info": (C.c_int, [_P, C.POINTER(cor_info), _P]),
    "cor_plan_destroy": (C.c_int, [_P]),
    "cor_server_create": (C.c_int, [C.POINTER(cor_server_cfg), C.POINTER(_P)]),
    "cor_server_submit": (C.c_int, [_P, C.POINTER(cor_problem), C.POINTER(cor_opts),
                                    C.POINTER(C.c_uint64)]),
    "cor_server_poll": (C.c_int, [_P, C.c_uint64, C.POINTER(cor_info)]),
    "cor_server_wait": (C.c_int, [_P, C.c_uint64, C.POINTER(cor_info)]),
    "cor_server_stats_get": (C.c_int, [_P, C.POINTER(cor_server_stats)]),
    "cor_server_destroy": (C.c_int, [_P]),
    "cor_workspace_bytes": (C.c_size_t, [C.c_int64, C.c_int64, C.c_int32, C.c_int32]),
    "cor_quantize": (C.c_int, [_P, C.c_int64, C.c_int64, C.c_int64, C.c_int32, _P, _P, _P]),
    "cor_omega": (C.c_int, [C.c_uint64, C.c_int64, C.c_int32, _P, _P]),
    "cor_profile_enable": (C.c_int, [C.c_int32]),
    "cor_profile_read": (C.c_int, [C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "cor_status_string": (C.c_char_p, [C.c_int32]),
    "cor_last_error": (C.c_char_p, []),
    "cor_release": (C.c_int, []),
}

_lib = None


def lib():
    """Load libcorutv.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1810_07323_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class CorError(RuntimeError):
    def __init__(self, status, where):
        L = lib()
        msg = L.cor_last_error().decode()
        super().__init__(f"{where}: {L.cor_status_string(status).decode()} ({msg})")
        self.status = status


def check(status, where="cor"):
    if status != COR_OK:
        raise CorError(status, where)
    return status


# ---------------------------------------------------------------------------
# Marshalling helpers (torch tensors -> device pointers, streams)
# ---------------------------------------------------------------------------
def ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def stream_handle(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _prec_of(A):
    import torch

    return {torch.float64: COR_F64, torch.float32: COR_F32, torch.bfloat16: COR_BF16,
            torch.uint8: COR_FP8, torch.float8_e4m3fn: COR_FP8}[A.dtype]


# ---------------------------------------------------------------------------
# Entry points with the C names
# ---------------------------------------------------------------------------
def cor_utv(A, m, n, k, p, q, seed, prec, U, T, V, stream=None):
    info = cor_info()
    st = lib().cor_utv(ptr(A), m, n, k, p, q, C.c_uint64(seed), prec, ptr(U), ptr(T), ptr(V),
                       C.byref(info), stream_handle(stream))
    return st, info


def make_problem(A, k, p, q, seed=0, U=None, T=None, V=None, perm=None, omega=None,
                 colscale=None, prec=None, lda=None):
    m, n = A.shape
    pr = cor_problem()
    pr.A = A.data_ptr()
    pr.colscale = colscale.data_ptr() if colscale is not None else None
    pr.m, pr.n = m, n
    pr.lda = lda if lda is not None else A.stride(0)
    pr.k, pr.p, pr.q = k, p, q
    pr.prec = prec if prec is not None else _prec_of(A)
    pr.seed = seed
    pr.omega = omega.data_ptr() if omega is not None else None
    pr.U = U.data_ptr() if U is not None else None
    pr.T = T.data_ptr() if T is not None else None
    pr.V = V.data_ptr() if V is not None else None
    pr.perm = perm.data_ptr() if perm is not None else None
    return pr


def cor_utv_ex(problem, opts=None, stream=None):
    info = cor_info()
    st = lib().cor_utv_ex(C.byref(problem), C.byref(opts) if opts is not None else None,
                          C.byref(info), stream_handle(stream))
    return st, info


def cor_utv_ex_noalloc(problem, opts=None, stream=None):
    info = cor_info()
    st = lib().cor_utv_ex_noalloc(C.byref(problem), C.byref(opts) if opts is not None else None,
                                  C.byref(info), stream_handle(stream))
    return st, info


def cor_tune(problem, reps=5, stream=None):
    """Returns (status, s_ax, s_atx)."""
    a, b = C.c_int32(0), C.c_int32(0)
    st = lib().cor_tune(C.byref(problem), reps, C.byref(a), C.byref(b), stream_handle(stream))
    return st, a.value, b.value


def cor_tune_save(path):
    return lib().cor_tune_save(os.fsencode(path))


def cor_tune_load(path):
    return lib().cor_tune_load(os.fsencode(path))


def cor_tune_clear():
    return lib().cor_tune_clear()


def cor_utv_host(problem, opts=None, panel_rows=0, stream=None):
    """problem.A is a host address (e.g. a pinned torch tensor's data_ptr())."""
    info = cor_info()
    st = lib().cor_utv_host(C.byref(problem), C.byref(opts) if opts is not None else None,
                            panel_rows, C.byref(info), stream_handle(stream))
    return st, info


def cor_utv_batched(problems, opts=None, stream=None):
    arr = (cor_problem * len(problems))(*problems)
    infos = (cor_info * len(problems))()
    st = lib().cor_utv_batched(arr, len(problems), C.byref(opts) if opts is not None else None,
                               infos, stream_handle(stream))
    return st, list(infos)


def cor_rpca_alm(M, m, n, ldm, opts, L, S, stream=None):
    """M, L, S: device FP64 tensors or addresses; returns (status, cor_rpca_info)."""
    info = cor_rpca_info()
    st = lib().cor_rpca_alm(ptr(M), m, n, ldm, C.byref(opts), ptr(L), ptr(S), C.byref(info),
                            stream_handle(stream))
    return st, info


def rpca(M, k, p, q, seed=0, prec=COR_F64, lam=0.0, rho=0.0, mu_bar_ratio=0.0, tol=0.0,
         max_iter=0, stream=None):
    """Robust PCA of device FP64 matrix M (torch tensor): returns (L, S, info)."""
    import torch

    m, n = M.shape
    assert M.dtype == torch.float64 and M.stride(1) == 1
    L = torch.empty((m, n), dtype=torch.float64, device=M.device)
    S = torch.empty((m, n), dtype=torch.float64, device=M.device)
    o = cor_rpca_opts(k, p, q, prec, seed, lam, rho, mu_bar_ratio, tol, max_iter)
    st, info = cor_rpca_alm(M, m, n, M.stride(0), o, L, S, stream)
    check(st, "cor_rpca_alm")
    return L, S, info


def cor_plan_create(problems, opts=None):
    arr = (cor_problem * len(problems))(*problems)
    h = C.c_void_p()
    st = lib().cor_plan_create(arr, len(problems), C.byref(opts) if opts is not None else None,
                               C.byref(h))
    return st, h


def cor_plan_run(plan, stream=None):
    return lib().cor_plan_run(plan, stream_handle(stream))


def cor_plan_capture(plan, stream=None):
    return lib().cor_plan_capture(plan, stream_handle(stream))


def cor_plan_info(plan, count, stream=None):
    infos = (cor_info * count)()
    st = lib().cor_plan_info(plan, infos, stream_handle(stream))
    return st, list(infos)


def cor_plan_destroy(plan):
    return lib().cor_plan_destroy(plan)


def cor_server_create(hbm_budget=0, max_slots=0, convert_f32_to=0):
    cfg = cor_server_cfg(hbm_budget, max_slots, convert_f32_to)
    h = C.c_void_p()
    st = lib().cor_server_create(C.byref(cfg), C.byref(h))
    return st, h


def cor_server_submit(server, problem, opts=None):
    t = C.c_uint64()
    st = lib().cor_server_submit(server, C.byref(problem),
                                 C.byref(opts) if opts is not None else None, C.byref(t))
    return st, t.value


def cor_server_poll(server, ticket):
    info = cor_info()
    st = lib().cor_server_poll(server, C.c_uint64(ticket), C.byref(info))
    return st, info


def cor_server_wait(server, ticket):
    info = cor_info()
    st = lib().cor_server_wait(server, C.c_uint64(ticket), C.byref(info))
    return st, info


def cor_server_stats_get(server):
    s = cor_server_stats()
    st = lib().cor_server_stats_get(server, C.byref(s))
    return st, s


def cor_server_destroy(server):
    return lib().cor_server_destroy(server)


def cor_workspace_bytes(m, n, l, prec):
    return lib().cor_workspace_bytes(m, n, l, prec)


def cor_quantize(A32, to, out, colscale=None, stream=None):
    m, n = A32.shape
    return lib().cor_quantize(ptr(A32), m, n, A32.stride(0), to, ptr(out), ptr(colscale),
                              stream_handle(stream))


def cor_omega(seed, n, l, out, stream=None):
    return lib().cor_omega(C.c_uint64(seed), n, l, ptr(out), stream_handle(stream))


def cor_profile_enable(on=True):
    """on: False/0 off, True/1 the two-pass kernels, 2 the fused power step, 3 both."""
    return lib().cor_profile_enable(int(on))


def cor_profile_read():
    ms, n, b, f = C.c_double(), C.c_int64(), C.c_double(), C.c_double()
    check(lib().cor_profile_read(C.byref(ms), C.byref(n), C.byref(b), C.byref(f)), "profile")
    return dict(ms=ms.value, launches=n.value, bytes=b.value, flops=f.value)


def cor_status_string(st):
    return lib().cor_status_string(st).decode()


def cor_last_error():
    return lib().cor_last_error().decode()


def cor_release():
    return lib().cor_release()


# ---------------------------------------------------------------------------
# Convenience: allocate outputs with torch and run one decomposition.
# ---------------------------------------------------------------------------
def decompose(A, k, p, q, seed=0, omega=None, colscale=None, report=False, stream=None,
              compress=COR_M_R2T, orient=COR_URV, fused=False):
    """Return (U, T, V, perm, info) for device matrix A (torch tensor on cuda)."""
    import torch

    m, n = A.shape
    l = k + p
    dev = A.device
    U = torch.empty((m, l), dtype=torch.float64, device=dev)
    T = torch.empty((l, l), dtype=torch.float64, device=dev)
    V = torch.empty((n, l), dtype=torch.float64, device=dev)
    perm = torch.empty((l,), dtype=torch.int32, device=dev)
    om = None
    if omega is not None:
        om = torch.as_tensor(omega, dtype=torch.float64, device=dev).contiguous()
    pr = make_problem(A, k, p, q, seed, U, T, V, perm, om, colscale)
    st, info = cor_utv_ex(pr, cor_opts(1 if report else 0, 0, compress, orient, 1 if fused else 0),
                          stream)
    check(st, "cor_utv_ex")
    return U, T, V, perm, info
