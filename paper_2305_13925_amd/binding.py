"""ctypes binding of libjacpcg.so with the names of its C ABI.

Argument marshalling only: torch tensors supply device memory and the stream;
every step of the precoder runs in the library's HIP kernels. Layout rules
(see include/jacpcg.h):

  H  complex64 [batch, K, M]   (each instance column-major M x K)
  A  complex64 [batch, K, K]   (row-major, both triangles)
  B, X complex64 [batch, n, K] (column-major K x n)
  W  complex64 [batch, n, M]   (column-major M x n)

There is no fallback: when the library is missing or no GPU is present the
calls raise.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libjacpcg.so")

# status codes
OK = 0
NOT_CONVERGED = 1
NOT_READY = 2
E_INVALID_ARG = -1
E_UNSUPPORTED = -2
E_NO_DEVICE = -3
E_OUT_OF_MEMORY = -4
E_BREAKDOWN = -5
E_HIP = -6
E_BUDGET = -7
E_CANCELLED = -8
E_TIMEOUT = -9

GRAM_FP32 = 0
GRAM_BF16X3 = 1
GRAM_BF16X6 = 2
GRAM_FP64_ROUNDED = 3
REFINE_FP64 = 0x100
PRECOND_JACOBI = 0
PRECOND_NONE = 1
EPILOGUE_FP32 = 0x10

PHASES = ("gram", "solve", "epilogue", "gram64", "residual")

_i64 = C.c_int64
_vp = C.c_void_p


class JacpcgStats(C.Structure):
    _fields_ = [
        ("max_rel_residual", C.c_double),
        ("max_refine_residual", C.c_double),
        ("max_iters", C.c_int32),
        ("refine_steps", C.c_int32),
        ("worst_status", C.c_int32),
        ("reserved", C.c_int32),
        ("beta_pow_min", C.c_double),
        ("beta_pow_max", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class JacpcgRequest(C.Structure):
    _fields_ = [("M", C.c_int), ("K", C.c_int), ("n_sub", C.c_int), ("H", C.c_void_p), ("W", C.c_void_p),
                ("xi", C.c_double), ("power", C.c_double), ("tol", C.c_double), ("max_iter", C.c_int),
                ("precision", C.c_int), ("flags", C.c_int), ("user_tag", C.c_uint64), ("stream", C.c_void_p)]


class JacpcgResult(C.Structure):
    _fields_ = [("status", C.c_int), ("max_iters", C.c_int32), ("t_submit_us", C.c_double),
                ("t_admit_us", C.c_double), ("t_done_us", C.c_double), ("user_tag", C.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class JacpcgError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"{status_string(code)} ({code}): {message}")
        self.code = code


_lib = None


def _declare(lib):
    lib.jacpcg_version.restype = C.c_int
    lib.jacpcg_last_error.restype = C.c_char_p
    lib.jacpcg_last_error.argtypes = [_vp]
    lib.jacpcg_status_string.restype = C.c_char_p
    lib.jacpcg_status_string.argtypes = [C.c_int]
    lib.jacpcg_session_create.argtypes = [C.c_int, C.c_size_t, C.c_char_p, C.POINTER(_vp)]
    lib.jacpcg_session_destroy.argtypes = [_vp]
    lib.jacpcg_session_destroy.restype = None
    lib.jacpcg_session_set_profiling.argtypes = [_vp, C.c_int]
    lib.jacpcg_session_phase_times.argtypes = [_vp, C.POINTER(C.c_double), C.POINTER(_i64), C.c_int]
    lib.jacpcg_gram.argtypes = [_vp, _vp, C.c_int, C.c_int, C.c_int, _vp, _i64, _i64, C.c_float, C.c_int,
                                _vp, _i64, _i64, _vp]
    lib.jacpcg_solve.argtypes = [_vp, _vp, C.c_int, C.c_int, C.c_int, _vp, _i64, _i64, _vp, _i64, _i64,
                                 _vp, _i64, _i64, C.c_double, C.c_int, C.c_int, _vp, _vp, _vp]
    lib.rzf_precoder.argtypes = [_vp, _vp, C.c_int, C.c_int, C.c_int, _vp, _i64, _i64, C.c_double, C.c_double,
                                 C.c_double, C.c_int, C.c_int, C.c_int, C.c_double, _vp, _i64, _i64, _vp, _vp,
                                 C.POINTER(JacpcgStats)]
    lib.rzf_precoder_noalloc.argtypes = [_vp, _vp, C.c_int, C.c_int, C.c_int, _vp, _i64, _i64, C.c_double,
                                         C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, _vp, _i64, _i64, _vp]
    lib.rzf_precoder_plain.argtypes = [_vp, _vp, C.c_int, C.c_int, C.c_int, _vp, _i64, _i64, C.c_double,
                                       C.c_double, C.c_double, C.c_int, C.c_int, _vp, _i64, _i64, _vp,
                                       C.POINTER(JacpcgStats)]
    lib.rzf_transmit.argtypes = [_vp, _vp, C.c_int, C.c_int, C.c_int, C.c_int, _vp, C.c_int64, C.c_int64, _vp,
                                 C.c_int64, C.c_int64, C.c_double, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int,
                                 _vp, C.c_int64, C.c_int64, _vp, C.POINTER(JacpcgStats)]
    lib.rzf_precoder_vr.argtypes = [_vp, _vp, C.c_int, C.c_int, C.c_int, _vp, C.c_int64, C.c_int64, _vp, C.c_double,
                                    C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, C.c_double, _vp, C.c_int64,
                                    C.c_int64, _vp, C.POINTER(JacpcgStats)]
    lib.rzf_block_precoder.argtypes = [_vp, _vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _vp,
                                       C.c_int64, C.c_int64, C.c_double, C.c_double, C.c_double, C.c_int, C.c_int,
                                       C.c_int, C.c_double, _vp, C.c_int64, C.c_int64, C.POINTER(JacpcgStats)]
    lib.rzf_sinr.argtypes = [_vp, _vp, C.c_int, C.c_int, C.c_int, _vp, C.c_int64, C.c_int64, _vp, C.c_int64,
                             C.c_int64, C.c_double, _vp, _vp]
    lib.jacpcg_mfma_peaks.argtypes = [_vp, _vp, C.POINTER(C.c_double)]
    lib.jacpcg_mfma_peaks.restype = C.c_int
    lib.jacpcg_tune_set.argtypes = [_vp, C.c_char_p, C.c_int, C.c_int, C.c_int, C.c_int]
    lib.jacpcg_tune_set.restype = C.c_int
    lib.jacpcg_tune_get.argtypes = [_vp, C.c_char_p, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int)]
    lib.jacpcg_tune_get.restype = C.c_int
    lib.jacpcg_session_set_graphs.argtypes = [_vp, C.c_int]
    lib.jacpcg_autotune.argtypes = [_vp, _vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]
    lib.jacpcg_submit.argtypes = [_vp, C.POINTER(JacpcgRequest), C.POINTER(C.c_uint64)]
    lib.jacpcg_poll.argtypes = [_vp, C.c_uint64, C.POINTER(JacpcgResult)]
    lib.jacpcg_wait.argtypes = [_vp, C.c_uint64, C.c_int, C.POINTER(JacpcgResult)]
    lib.jacpcg_cancel.argtypes = [_vp, C.c_uint64]
    lib.jacpcg_session_clock_us.argtypes = [_vp]
    lib.jacpcg_session_clock_us.restype = C.c_double
    for name in ("jacpcg_session_create", "jacpcg_session_set_profiling", "jacpcg_session_phase_times",
                 "jacpcg_gram", "jacpcg_solve", "rzf_precoder", "rzf_precoder_noalloc", "rzf_precoder_plain", "rzf_transmit", "rzf_sinr",
                 "rzf_block_precoder", "rzf_precoder_vr", "jacpcg_submit", "jacpcg_session_set_graphs",
                 "jacpcg_autotune",
                 "jacpcg_poll", "jacpcg_wait", "jacpcg_cancel"):
        getattr(lib, name).restype = C.c_int
    return lib


def lib():
    """The loaded library (raises if it has not been built).

    torch is imported first: torch ships its own HIP runtime under the same
    soname (libamdhip64.so.7), and whichever copy is loaded first serves the
    whole process. Loading torch's first keeps one HIP runtime for torch's
    allocations and streams and this library's kernels."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2305_13925_amd.build`")
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        _lib = _declare(C.CDLL(LIB_PATH))
    return _lib


def status_string(code):
    return lib().jacpcg_status_string(int(code)).decode()


def last_error():
    return lib().jacpcg_last_error(None).decode()


def _check(rc):
    if rc < 0:
        raise JacpcgError(rc, last_error())
    return rc


# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _require(t, name, dtype, shape=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


class Session:
    """jacpcg_session_create / jacpcg_session_destroy."""

    def __init__(self, device=0, hbm_budget_bytes=0, tune_cache_path=None):
        h = _vp()
        path = tune_cache_path.encode() if tune_cache_path else None
        _check(lib().jacpcg_session_create(int(device), int(hbm_budget_bytes), path, C.byref(h)))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            lib().jacpcg_session_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_profiling(self, enable=True):
        _check(lib().jacpcg_session_set_profiling(self.handle, int(bool(enable))))

    def set_graphs(self, enable=True):
        _check(lib().jacpcg_session_set_graphs(self.handle, int(bool(enable))))

    def autotune(self, batch, M, K, precision=GRAM_FP32, flags=PRECOND_JACOBI, stream=None):
        """jacpcg_autotune: time the launch variants of one shape and keep the fastest."""
        _check(lib().jacpcg_autotune(self.handle, _stream(stream), int(batch), int(M), int(K), int(precision),
                                     int(flags)))

    def tune_set(self, knob, M, K, variant, value):
        """jacpcg_tune_set: pin one launch choice (value 0: the default rule)."""
        _check(lib().jacpcg_tune_set(self.handle, knob.encode(), int(M), int(K), int(variant), int(value)))

    def tune_get(self, knob, M, K, variant):
        """jacpcg_tune_get: the chosen value of one knob (0: not tuned)."""
        v = C.c_int()
        _check(lib().jacpcg_tune_get(self.handle, knob.encode(), int(M), int(K), int(variant), C.byref(v)))
        return v.value

    def phase_times(self, reset=False):
        ms = (C.c_double * 5)()
        cnt = (_i64 * 5)()
        _check(lib().jacpcg_session_phase_times(self.handle, ms, cnt, int(bool(reset))))
        return {PHASES[i]: (ms[i], cnt[i]) for i in range(5)}


def jacpcg_gram(session, H, xi, precision=GRAM_FP32, A=None, diag=None, stream=None):
    """A = H^H H + xi I for H complex64 [batch, K, M]; returns A [batch, K, K]."""
    torch = _torch()
    _require(H, "H", torch.complex64)
    batch, K, M = H.shape
    if A is None:
        A = torch.empty((batch, K, K), dtype=torch.complex64, device=H.device)
    _require(A, "A", torch.complex64, (batch, K, K))
    if diag is not None:
        _require(diag, "diag", torch.float32, (batch, K))
    _check(lib().jacpcg_gram(session.handle, _stream(stream), batch, M, K, _ptr(H), M, K * M, float(xi),
                             int(precision), _ptr(A), K, K * K, _ptr(diag)))
    return A


def jacpcg_solve(session, A, B=None, tol=0.0, max_iter=16, flags=PRECOND_JACOBI, X=None, iters=None,
                 relres=None, status=None, stream=None):
    """X = A^{-1} B by Jacobi-PCG. A [batch, K, K]; B [batch, n, K] or None (identity).

    Returns X [batch, n, K]; iters/relres [batch, n] and status [batch] are
    filled when given."""
    torch = _torch()
    _require(A, "A", torch.complex64)
    batch, K, _ = A.shape
    n = K if B is None else B.shape[1]
    if B is not None:
        _require(B, "B", torch.complex64, (batch, n, K))
    if X is None:
        X = torch.empty((batch, n, K), dtype=torch.complex64, device=A.device)
    _require(X, "X", torch.complex64, (batch, n, K))
    if iters is not None:
        _require(iters, "iters", torch.int32, (batch, n))
    if relres is not None:
        _require(relres, "relres", torch.float32, (batch, n))
    if status is not None:
        _require(status, "status", torch.int32, (batch,))
    _check(lib().jacpcg_solve(session.handle, _stream(stream), batch, K, n, _ptr(A), K, K * K, _ptr(B), K,
                              n * K, _ptr(X), K, n * K, float(tol), int(max_iter), int(flags), _ptr(iters),
                              _ptr(relres), _ptr(status)))
    return X


def rzf_precoder(session, H, xi, power=1.0, tol=0.0, max_iter=16, precision=GRAM_FP32, flags=PRECOND_JACOBI,
                 refine_tol=1e-10, W=None, X_out=None, X64_out=None, stats=False, stream=None):
    """W = beta_pow H A^{-1} (Jacobi-PCG), H complex64 [batch, K, M] -> W [batch, K, M].

    Returns W, or (W, stats dict, return code) when stats=True (synchronises)."""
    torch = _torch()
    _require(H, "H", torch.complex64)
    batch, K, M = H.shape
    if W is None:
        W = torch.empty((batch, K, M), dtype=torch.complex64, device=H.device)
    _require(W, "W", torch.complex64, (batch, K, M))
    if X_out is not None:
        _require(X_out, "X_out", torch.complex64, (batch, K, K))
    if X64_out is not None:
        _require(X64_out, "X64_out", torch.complex128, (batch, K, K))
    st = JacpcgStats() if stats else None
    rc = _check(lib().rzf_precoder(session.handle, _stream(stream), batch, M, K, _ptr(H), M, K * M, float(xi),
                                   float(power), float(tol), int(max_iter), int(precision), int(flags),
                                   float(refine_tol), _ptr(W), M, K * M, _ptr(X_out), _ptr(X64_out),
                                   C.byref(st) if st is not None else None))
    if stats:
        return W, st.as_dict(), rc
    return W


def rzf_precoder_noalloc(session, H, xi, power=1.0, tol=0.0, max_iter=16, precision=GRAM_FP32,
                         flags=PRECOND_JACOBI, W=None, status=None, stream=None):
    """rzf_precoder on the library's fixed device workspace (allocates nothing
    in the call; calls overlapping on one GPU race). H complex64 [batch, K, M]
    -> W [batch, K, M]; status: optional int32 [batch] device tensor."""
    torch = _torch()
    _require(H, "H", torch.complex64)
    batch, K, M = H.shape
    if W is None:
        W = torch.empty((batch, K, M), dtype=torch.complex64, device=H.device)
    _require(W, "W", torch.complex64, (batch, K, M))
    if status is not None:
        _require(status, "status", torch.int32, (batch,))
    _check(lib().rzf_precoder_noalloc(session.handle, _stream(stream), batch, M, K, _ptr(H), M, K * M, float(xi),
                                      float(power), float(tol), int(max_iter), int(precision), int(flags), _ptr(W),
                                      M, K * M, _ptr(status)))
    return W


def rzf_precoder_plain(session, H, xi, power=1.0, tol=0.0, max_iter=16, flags=PRECOND_JACOBI, W=None, X_out=None,
                       stats=False, stream=None):
    """The same precoder, one instance at a time with one launch per iteration."""
    torch = _torch()
    _require(H, "H", torch.complex64)
    batch, K, M = H.shape
    if W is None:
        W = torch.empty((batch, K, M), dtype=torch.complex64, device=H.device)
    _require(W, "W", torch.complex64, (batch, K, M))
    if X_out is not None:
        _require(X_out, "X_out", torch.complex64, (batch, K, K))
    st = JacpcgStats() if stats else None
    rc = _check(lib().rzf_precoder_plain(session.handle, _stream(stream), batch, M, K, _ptr(H), M, K * M,
                                         float(xi), float(power), float(tol), int(max_iter), int(flags), _ptr(W),
                                         M, K * M, _ptr(X_out), C.byref(st) if st is not None else None))
    if stats:
        return W, st.as_dict(), rc
    return W


def rzf_transmit(session, H, S, xi, power=1.0, tol=0.0, max_iter=16, precision=GRAM_FP32, flags=PRECOND_JACOBI,
                 x=None, w_out=None, stats=False, stream=None):
    """Per-symbol transmission x = beta_pow H A^{-1} s (eqs. 15-16).

    H complex64 [batch, K, M]; S complex64 [batch, nsym, K] (symbol vectors as
    rows, i.e. column-major K x nsym). Returns x [batch, nsym, M], or
    (x, stats dict, return code) when stats=True (synchronises)."""
    torch = _torch()
    _require(H, "H", torch.complex64)
    _require(S, "S", torch.complex64)
    batch, K, M = H.shape
    if S.dim() != 3 or S.shape[0] != batch or S.shape[2] != K:
        raise ValueError(f"S must be [batch={batch}, nsym, K={K}], got {tuple(S.shape)}")
    nsym = S.shape[1]
    if x is None:
        x = torch.empty((batch, nsym, M), dtype=torch.complex64, device=H.device)
    _require(x, "x", torch.complex64, (batch, nsym, M))
    if w_out is not None:
        _require(w_out, "w_out", torch.complex64, (batch, nsym, K))
    st = JacpcgStats() if stats else None
    rc = _check(lib().rzf_transmit(session.handle, _stream(stream), batch, M, K, nsym, _ptr(H), M, K * M, _ptr(S),
                                   K, K * nsym, float(xi), float(power), float(tol), int(max_iter), int(precision),
                                   int(flags), _ptr(x), M, M * nsym, _ptr(w_out),
                                   C.byref(st) if st is not None else None))
    if stats:
        return x, st.as_dict(), rc
    return x


def rzf_precoder_vr(session, H, xi, user_span=None, power=1.0, tol=0.0, max_iter=16, precision=GRAM_FP32,
                    flags=PRECOND_JACOBI, refine_tol=1e-10, W=None, X_out=None, stats=False, stream=None):
    """rzf_precoder exploiting visibility-region sparsity. user_span: int32
    [batch, K, 2] device tensor of per-user antenna spans (first, end), or
    None to find them on the device."""
    torch = _torch()
    _require(H, "H", torch.complex64)
    batch, K, M = H.shape
    if user_span is not None:
        _require(user_span, "user_span", torch.int32, (batch, K, 2))
    if W is None:
        W = torch.empty((batch, K, M), dtype=torch.complex64, device=H.device)
    _require(W, "W", torch.complex64, (batch, K, M))
    if X_out is not None:
        _require(X_out, "X_out", torch.complex64, (batch, K, K))
    st = JacpcgStats() if stats else None
    rc = _check(lib().rzf_precoder_vr(session.handle, _stream(stream), batch, M, K, _ptr(H), M, K * M,
                                      _ptr(user_span), float(xi), float(power), float(tol), int(max_iter),
                                      int(precision), int(flags), float(refine_tol), _ptr(W), M, K * M, _ptr(X_out),
                                      C.byref(st) if st is not None else None))
    if stats:
        return W, st.as_dict(), rc
    return W


def rzf_block_precoder(session, H, xi, M1, Mc, M2, K1, K2, power=1.0, tol=0.0, max_iter=16, precision=GRAM_FP32,
                       flags=PRECOND_JACOBI, refine_tol=1e-10, G=None, stats=False, stream=None):
    """Subarray-block RZF G (eqs. 2, 6, 7) for H complex64 [batch, K1 + K2, M1 + Mc + M2].

    Returns G of the same shape, or (G, stats dict, return code) when stats=True."""
    torch = _torch()
    _require(H, "H", torch.complex64)
    batch, K, M = H.shape
    if M != M1 + Mc + M2 or K != K1 + K2:
        raise ValueError(f"H is [batch, {K}, {M}], blocks give K = {K1 + K2}, M = {M1 + Mc + M2}")
    if G is None:
        G = torch.empty_like(H)
    _require(G, "G", torch.complex64, (batch, K, M))
    st = JacpcgStats() if stats else None
    rc = _check(lib().rzf_block_precoder(session.handle, _stream(stream), batch, int(M1), int(Mc), int(M2), int(K1),
                                         int(K2), _ptr(H), M, K * M, float(xi), float(power), float(tol),
                                         int(max_iter), int(precision), int(flags), float(refine_tol), _ptr(G), M,
                                         K * M, C.byref(st) if st is not None else None))
    if stats:
        return G, st.as_dict(), rc
    return G


def rzf_sinr(session, H, W, sigma2, sinr=None, se=None, stream=None):
    """Per-user SINR and per-instance sum rate of precoder W on channel H
    (eqs. 8-10). H, W complex64 [batch, K, M]. Returns (sinr [batch, K],
    se [batch]) as float32 device tensors."""
    torch = _torch()
    _require(H, "H", torch.complex64)
    batch, K, M = H.shape
    _require(W, "W", torch.complex64, (batch, K, M))
    if sinr is None:
        sinr = torch.empty((batch, K), dtype=torch.float32, device=H.device)
    if se is None:
        se = torch.empty((batch,), dtype=torch.float32, device=H.device)
    _require(sinr, "sinr", torch.float32, (batch, K))
    _require(se, "se", torch.float32, (batch,))
    _check(lib().rzf_sinr(session.handle, _stream(stream), batch, M, K, _ptr(H), M, K * M, _ptr(W), M, K * M,
                          float(sigma2), _ptr(sinr), _ptr(se)))
    return sinr, se


def jacpcg_submit(session, H, W, xi, power=1.0, tol=0.0, max_iter=16, precision=GRAM_FP32, flags=PRECOND_JACOBI,
                  user_tag=0, stream=None):
    """Queue a request: H, W complex64 [n_sub, K, M] device tensors (kept alive
    by the caller until the result is collected). The request waits for the
    work queued so far on `stream` (default: the current stream), where H is
    produced. Returns the ticket."""
    torch = _torch()
    _require(H, "H", torch.complex64)
    n_sub, K, M = H.shape
    _require(W, "W", torch.complex64, (n_sub, K, M))
    r = JacpcgRequest(M, K, n_sub, H.data_ptr(), W.data_ptr(), float(xi), float(power), float(tol), int(max_iter),
                      int(precision), int(flags), int(user_tag), _stream(stream))
    t = C.c_uint64()
    _check(lib().jacpcg_submit(session.handle, C.byref(r), C.byref(t)))
    return t.value


def jacpcg_poll(session, ticket):
    """(rc, result dict): rc NOT_READY while in flight, OK when final."""
    res = JacpcgResult()
    rc = _check(lib().jacpcg_poll(session.handle, int(ticket), C.byref(res)))
    return rc, res.as_dict()


def jacpcg_wait(session, ticket, timeout_ms=-1):
    """Result dict of a final request; raises JacpcgError(E_TIMEOUT) on timeout."""
    res = JacpcgResult()
    _check(lib().jacpcg_wait(session.handle, int(ticket), int(timeout_ms), C.byref(res)))
    return res.as_dict()


def jacpcg_cancel(session, ticket):
    _check(lib().jacpcg_cancel(session.handle, int(ticket)))


def jacpcg_session_clock_us(session):
    return lib().jacpcg_session_clock_us(session.handle)


def exported_symbols():
    """Names declared in include/jacpcg.h (parsed from the header)."""
    import re
    hdr = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "jacpcg.h")
    text = open(hdr).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(\w+)\s*\(", text, flags=re.M)))


def to_numpy_instance(t):
    """Host copy of one [n, rows] column-major instance as a rows x n complex128 matrix."""
    return np.asarray(t.detach().cpu().numpy()).T.astype(np.complex128)


def mfma_peaks(session, stream=None):
    """Measured matrix-core peaks of the session's device:
    {"fp32": TFLOP/s, "bf16": TFLOP/s, "fp64": TFLOP/s, "int8": TOP/s}."""
    out = (C.c_double * 4)()
    _check(lib().jacpcg_mfma_peaks(session.handle, _stream(stream), out))
    return dict(zip(("fp32", "bf16", "fp64", "int8"), (round(v, 1) for v in out)))

