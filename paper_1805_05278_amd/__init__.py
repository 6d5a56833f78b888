"""Python binding of libmiqr (MI355X Householder QR / least squares, C ABI in
include/miqr.h).  Argument marshalling only: every step runs in the HIP
library; this module never computes a factorisation itself and raises if the
library is missing.

Matrices are float64 torch tensors on the GPU in column-major layout: a tensor
``A`` of shape (m, n) with ``A.stride(0) == 1`` and ``A.stride(1) >= m`` (for
example ``colmajor(m, n)`` or ``torch.empty(n, m).t()``).  Calls are enqueued on
torch's current stream.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmiqr.so")

OK, EINVAL, ENOMEM, EHIP, ESINGULAR, ENOCONV, EBUSY, ENOTSUP = range(8)
FP64, MIXED_FP32, MIXED_BF16 = 0, 1, 2
T_FULL, T_BLOCKED = 0, 1

_i64 = ctypes.c_int64
_vp = ctypes.c_void_p


class MiqrError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("miqr status %d: %s" % (status, message))
        self.status = status


class QrOpts(ctypes.Structure):
    _fields_ = [("b", _i64), ("leaf_rows", _i64), ("chain", _i64), ("arity", _i64),
                ("precision", ctypes.c_int32), ("normalize", ctypes.c_int32),
                ("sign_out", _vp), ("Q", _vp), ("ldq", _i64), ("bstar", _i64), ("nb", _i64),
                ("t_layout", ctypes.c_int32), ("no_lookahead", ctypes.c_int32)]


class QrInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("fallback", ctypes.c_int32),
                ("precision_used", ctypes.c_int32), ("singular_index", ctypes.c_int32),
                ("backward_error", ctypes.c_double)]


class QrBatchItem(ctypes.Structure):
    _fields_ = [("m", _i64), ("n", _i64), ("nrhs", _i64), ("A", _vp), ("lda", _i64),
                ("B", _vp), ("ldb", _i64)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", _i64), ("max_batch", _i64), ("max_pending", _i64),
                ("stage_bytes", _i64), ("keep_factors", ctypes.c_int32),
                ("precision", ctypes.c_int32)]


class ServerDone(ctypes.Structure):
    _fields_ = [("id", _i64), ("status", ctypes.c_int32), ("batch_size", ctypes.c_int32),
                ("submit_s", ctypes.c_double), ("start_s", ctypes.c_double),
                ("end_s", ctypes.c_double)]


_lib = None


def lib():
    """Load libmiqr.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmiqr.so is not built (run __graft_entry__.build() or "
                              "python -m paper_1805_05278_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        st = ctypes.c_int
        L.miqr_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int]
        L.miqr_create.restype = st
        L.miqr_destroy.argtypes = [_vp]
        L.miqr_destroy.restype = st
        L.miqr_status_string.argtypes = [st]
        L.miqr_status_string.restype = ctypes.c_char_p
        L.miqr_last_error.argtypes = [_vp]
        L.miqr_last_error.restype = ctypes.c_char_p
        L.qr_workspace_size.argtypes = [_i64, _i64, ctypes.POINTER(QrOpts)]
        L.qr_workspace_size.restype = _i64
        L.qr_t_rows.argtypes = [_i64, _i64, ctypes.POINTER(QrOpts)]
        L.qr_t_rows.restype = _i64
        L.qr_plan.argtypes = [_i64, _i64, ctypes.POINTER(QrOpts), ctypes.c_int, ctypes.c_char_p,
                              _i64]
        L.qr_plan.restype = _i64
        L.qr_apply_q_blocked.argtypes = [_vp, _vp, ctypes.c_char, _i64, _i64, _i64, _vp, _i64,
                                         _vp, _i64, _i64, _vp, _i64]
        L.qr_apply_q_blocked.restype = st
        L.qr_factor.argtypes = [_vp, _vp, _i64, _i64, _vp, _i64, _vp, _i64,
                                ctypes.POINTER(QrOpts)]
        L.qr_factor.restype = st
        L.qr_factor_noalloc.argtypes = L.qr_factor.argtypes
        L.qr_factor_noalloc.restype = st
        L.qr_apply_q.argtypes = [_vp, _vp, ctypes.c_char, _i64, _i64, _i64, _vp, _i64, _vp,
                                 _i64, _vp, _i64]
        L.qr_apply_q.restype = st
        L.qr_form_q.argtypes = [_vp, _vp, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _i64]
        L.qr_form_q.restype = st
        L.qr_lstsq.argtypes = [_vp, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64,
                               ctypes.POINTER(QrOpts), ctypes.POINTER(QrInfo)]
        L.qr_lstsq.restype = st
        L.qr_solve_r.argtypes = [_vp, _vp, _i64, _i64, _vp, _i64, _vp, _i64]
        L.qr_solve_r.restype = st
        L.qr_backward_error.argtypes = [_vp, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp,
                                        _i64, ctypes.POINTER(ctypes.c_double)]
        L.qr_backward_error.restype = st
        L.qr_lstsq_batched.argtypes = [_vp, _vp, _i64, ctypes.POINTER(QrBatchItem),
                                       ctypes.POINTER(QrOpts), ctypes.POINTER(ctypes.c_int32)]
        L.qr_lstsq_batched.restype = st
        L.qr_lstsq_batched_ex.argtypes = [_vp, _vp, _i64, ctypes.POINTER(QrBatchItem),
                                          ctypes.POINTER(QrOpts), ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_int32)]
        L.qr_lstsq_batched_ex.restype = st
        L.qr_server_create.argtypes = [_vp, ctypes.POINTER(ServerOpts), ctypes.POINTER(_vp)]
        L.qr_server_create.restype = st
        L.qr_server_destroy.argtypes = [_vp]
        L.qr_server_destroy.restype = st
        L.qr_server_clock.argtypes = [_vp]
        L.qr_server_clock.restype = ctypes.c_double
        L.qr_server_submit.argtypes = [_vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64,
                                       ctypes.POINTER(_i64)]
        L.qr_server_submit.restype = st
        L.qr_server_resolve.argtypes = [_vp, _i64, _i64, _vp, _i64, _vp, _i64,
                                        ctypes.POINTER(_i64)]
        L.qr_server_resolve.restype = st
        L.qr_server_release.argtypes = [_vp, _i64]
        L.qr_server_release.restype = st
        L.qr_server_poll.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(ServerDone), _i64,
                                     ctypes.POINTER(_i64)]
        L.qr_server_poll.restype = st
        L.qr_server_stats.argtypes = [_vp] + [ctypes.POINTER(_i64)] * 4
        L.qr_server_stats.restype = st
        L.miqr_last_gemm_flops.argtypes = [_vp]
        L.miqr_last_gemm_flops.restype = ctypes.c_double
        L.miqr_profile_enable.argtypes = [_vp, ctypes.c_int]
        L.miqr_profile_enable.restype = st
        L.miqr_graphs_enable.argtypes = [_vp, ctypes.c_int]
        L.miqr_graphs_enable.restype = st
        L.miqr_graph_count.argtypes = [_vp]
        L.miqr_graph_count.restype = _i64
        L.miqr_profile_kernels.argtypes = [_vp]
        L.miqr_profile_kernels.restype = ctypes.c_int
        L.miqr_profile_get.argtypes = [_vp, ctypes.c_int, ctypes.c_char_p, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64),
                                       ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double)]
        L.miqr_profile_get.restype = st
        _lib = L
    return _lib


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def colmajor(m: int, n: int, device="cuda", dtype=None):
    """Uninitialised column-major (m, n) float64 tensor."""
    import torch
    dtype = dtype or torch.float64
    return torch.empty((n, m), dtype=dtype, device=device).t()


def to_colmajor(x, device="cuda"):
    """Copy a 2-D array-like into a new column-major float64 GPU tensor."""
    import torch
    t = torch.as_tensor(x, dtype=torch.float64)
    if t.dim() == 1:
        t = t.reshape(-1, 1)
    return t.t().contiguous().to(device).t()


def _mat(x, name: str):
    import torch
    if not isinstance(x, torch.Tensor) or x.dtype != torch.float64 or not x.is_cuda:
        raise TypeError("%s must be a float64 CUDA tensor" % name)
    if x.dim() != 2:
        raise ValueError("%s must be 2-D" % name)
    if x.shape[0] > 1 and x.stride(0) != 1:
        raise ValueError("%s must be column-major (stride(0) == 1)" % name)
    ld = max(x.stride(1), x.shape[0], 1) if x.shape[1] > 1 else max(x.shape[0], 1)
    return ctypes.c_void_p(x.data_ptr()), ld


@dataclass
class Info:
    iterations: int
    fallback: int
    precision_used: int
    singular_index: int
    backward_error: float


class Handle:
    """Owns a miqr handle (device workspace) for one device."""

    def __init__(self, device: int = 0):
        self._h = _vp()
        st = lib().miqr_create(ctypes.byref(self._h), device)
        if st != OK:
            raise MiqrError(st, lib().miqr_status_string(st).decode())

    def close(self):
        if self._h:
            lib().miqr_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != OK:
            msg = lib().miqr_last_error(self._h).decode() or lib().miqr_status_string(st).decode()
            raise MiqrError(st, msg)

    @property
    def last_gemm_flops(self) -> float:
        return float(lib().miqr_last_gemm_flops(self._h))

    def profile(self, enable: bool = True):
        """Start (clearing earlier totals) or stop per-kernel event timing."""
        self._check(lib().miqr_profile_enable(self._h, 1 if enable else 0))

    def graphs(self, enable: bool = True):
        """Replay factor() calls as captured launch graphs (off: eager, and
        every kept graph dropped)."""
        self._check(lib().miqr_graphs_enable(self._h, 1 if enable else 0))

    def graph_count(self) -> int:
        """Number of factorisation graphs the handle keeps."""
        return lib().miqr_graph_count(self._h)

    def profile_totals(self) -> dict:
        """{kernel: dict(ms, launches, bytes, flops)} accumulated while enabled."""
        n = lib().miqr_profile_kernels(self._h)
        out = {}
        for i in range(n):
            name = ctypes.create_string_buffer(128)
            ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
            cnt = _i64()
            self._check(lib().miqr_profile_get(self._h, i, name, 128, ctypes.byref(ms),
                                               ctypes.byref(cnt), ctypes.byref(by),
                                               ctypes.byref(fl)))
            out[name.value.decode()] = dict(ms=ms.value, launches=cnt.value, bytes=by.value,
                                            flops=fl.value)
        return out

    @staticmethod
    def opts(b=0, leaf_rows=0, chain=0, arity=0, precision=FP64, normalize=False,
             sign_out=None, Q=None, bstar=0, nb=0, t_layout=T_FULL,
             lookahead=True) -> QrOpts:
        o = QrOpts()
        o.b, o.leaf_rows, o.chain, o.arity = b, leaf_rows, chain, arity
        o.bstar, o.nb, o.t_layout = bstar, nb, t_layout
        o.no_lookahead = 0 if lookahead else 1
        o.precision = precision
        o.normalize = 1 if normalize else 0
        o.sign_out = sign_out.data_ptr() if sign_out is not None else None
        if Q is not None:
            qp, ldq = _mat(Q, "Q")
            o.Q, o.ldq = qp.value, ldq
        return o

    def workspace_size(self, m: int, n: int, opts: Optional[QrOpts] = None) -> int:
        return int(lib().qr_workspace_size(m, n, ctypes.byref(opts) if opts else None))

    @staticmethod
    def t_rows(m: int, n: int, opts: Optional[QrOpts] = None) -> int:
        """Rows of T that factor() writes (n, or the BLOCKED panel width)."""
        return int(lib().qr_t_rows(m, n, ctypes.byref(opts) if opts else None))

    @staticmethod
    def plan(m: int, n: int, opts: Optional[QrOpts] = None, lstsq: bool = False) -> dict:
        """The library's plan for this shape (tuning, cost model, workspace
        regions, recursion nodes and TSQR panels) as a dict."""
        import json
        o = ctypes.byref(opts) if opts else None
        n_chars = lib().qr_plan(m, n, o, 1 if lstsq else 0, None, 0)
        if n_chars < 0:
            raise ValueError("invalid shape or options")
        buf = ctypes.create_string_buffer(n_chars + 1)
        lib().qr_plan(m, n, o, 1 if lstsq else 0, buf, n_chars + 1)
        return json.loads(buf.value.decode())

    def factor(self, A, T, opts: Optional[QrOpts] = None):
        """In-place QR of A (m x n); T (n x n) receives the kernel."""
        ap, lda = _mat(A, "A")
        tp, ldt = _mat(T, "T")
        m, n = A.shape
        self._check(lib().qr_factor(self._h, _stream(), m, n, ap, lda, tp, ldt,
                                    ctypes.byref(opts) if opts else None))

    def factor_noalloc(self, A, T, opts: Optional[QrOpts] = None):
        """factor() on the caller's stream in the library's static device
        workspace (no device allocation)."""
        ap, lda = _mat(A, "A")
        tp, ldt = _mat(T, "T")
        m, n = A.shape
        self._check(lib().qr_factor_noalloc(self._h, _stream(), m, n, ap, lda, tp, ldt,
                                            ctypes.byref(opts) if opts else None))

    def apply_q(self, trans: str, VR, T, C):
        vp, lda = _mat(VR, "VR")
        tp, ldt = _mat(T, "T")
        cp, ldc = _mat(C, "C")
        m, n = VR.shape
        self._check(lib().qr_apply_q(self._h, _stream(), trans.encode(), m, n, C.shape[1],
                                     vp, lda, tp, ldt, cp, ldc))

    def apply_q_blocked(self, trans: str, VR, T, nb: int, C):
        """apply_q for factors in the BLOCKED T layout with panel width nb."""
        vp, lda = _mat(VR, "VR")
        tp, ldt = _mat(T, "T")
        cp, ldc = _mat(C, "C")
        m, n = VR.shape
        self._check(lib().qr_apply_q_blocked(self._h, _stream(), trans.encode(), m, n,
                                             C.shape[1], vp, lda, tp, ldt, nb, cp, ldc))

    def form_q(self, VR, T, Q, sign=None):
        vp, lda = _mat(VR, "VR")
        tp, ldt = _mat(T, "T")
        qp, ldq = _mat(Q, "Q")
        m, n = VR.shape
        sp = ctypes.c_void_p(sign.data_ptr()) if sign is not None else None
        self._check(lib().qr_form_q(self._h, _stream(), m, n, vp, lda, tp, ldt, sp, qp, ldq))

    def solve_r(self, VR, X):
        vp, lda = _mat(VR, "VR")
        xp, ldx = _mat(X, "X")
        n = VR.shape[1]
        self._check(lib().qr_solve_r(self._h, _stream(), n, X.shape[1], vp, lda, xp, ldx))

    def backward_error(self, A, B, X):
        """beta_j = ||A^T r_j|| / (||A||_F (||A||_F ||x_j|| + ||r_j||)) per
        column of X (computed by the library, FP64); returns a list."""
        ap, lda = _mat(A, "A")
        bp, ldb = _mat(B, "B")
        xp, ldx = _mat(X, "X")
        m, n = A.shape
        k = B.shape[1]
        out = (ctypes.c_double * k)()
        self._check(lib().qr_backward_error(self._h, _stream(), m, n, k, ap, lda, bp, ldb, xp,
                                            ldx, out))
        return list(out)

    def lstsq(self, A, B, opts: Optional[QrOpts] = None, want_info: bool = True):
        """Least squares in place: A <- factors, B[:n] <- solutions.  Returns
        (status, Info or None); raises on errors other than ENOCONV/ESINGULAR."""
        ap, lda = _mat(A, "A")
        bp, ldb = _mat(B, "B")
        m, n = A.shape
        info = QrInfo()
        st = lib().qr_lstsq(self._h, _stream(), m, n, B.shape[1], ap, lda, bp, ldb,
                            ctypes.byref(opts) if opts else None,
                            ctypes.byref(info) if want_info else None)
        if st not in (OK, ENOCONV, ESINGULAR):
            self._check(st)
        out = Info(info.iterations, info.fallback, info.precision_used, info.singular_index,
                   info.backward_error) if want_info else None
        return st, out

    def lstsq_batched(self, As, Bs, opts: Optional[QrOpts] = None, want_status: bool = True,
                      want_iters: bool = False):
        """Batched least squares: for each i, A_i is overwritten (R in its
        upper triangle) and B_i[:n_i] receives the solution.  Returns (status,
        per-problem statuses or None) and, with want_iters, also the
        per-problem refinement iterations (-1: solved again in FP64); raises
        on errors other than ESINGULAR."""
        if len(As) != len(Bs):
            raise ValueError("As and Bs differ in length")
        items = (QrBatchItem * max(len(As), 1))()
        for i, (A, B) in enumerate(zip(As, Bs)):
            ap, lda = _mat(A, "A")
            bp, ldb = _mat(B, "B")
            items[i] = QrBatchItem(A.shape[0], A.shape[1], B.shape[1], ap.value, lda, bp.value, ldb)
        stat = (ctypes.c_int32 * max(len(As), 1))()
        its = (ctypes.c_int32 * max(len(As), 1))()
        st = lib().qr_lstsq_batched_ex(self._h, _stream(), len(As), items,
                                       ctypes.byref(opts) if opts else None,
                                       stat if want_status else None,
                                       its if want_iters else None)
        if st not in (OK, ESINGULAR):
            self._check(st)
        out = (st, (list(stat)[:len(As)] if want_status else None))
        return out + (list(its)[:len(As)],) if want_iters else out


def _host(x, name: str):
    """(pointer, leading dimension) of a host column-major float64 matrix: a
    Fortran-ordered numpy array (or a view with unit row stride), or a CPU torch
    tensor with stride(0) == 1 (pin it for overlapped uploads)."""
    import numpy as np
    try:
        import torch
    except ImportError:  # pragma: no cover
        torch = None
    if torch is not None and isinstance(x, torch.Tensor):
        if x.is_cuda or x.dtype != torch.float64 or x.dim() != 2:
            raise TypeError("%s must be a 2-D float64 CPU tensor" % name)
        if x.shape[0] > 1 and x.stride(0) != 1:
            raise ValueError("%s must be column-major" % name)
        return x.data_ptr(), max(x.stride(1), x.shape[0], 1)
    if not isinstance(x, np.ndarray) or x.dtype != np.float64 or x.ndim != 2:
        raise TypeError("%s must be a 2-D float64 numpy array" % name)
    if x.shape[0] > 1 and x.strides[0] != 8:
        raise ValueError("%s must be column-major (Fortran order)" % name)
    ld = x.strides[1] // 8 if x.shape[1] > 1 else x.shape[0]
    return x.ctypes.data, max(ld, x.shape[0], 1)


class Server:
    """Least-squares server on the handle's device (include/miqr.h: serving
    loop).  Host inputs are referenced until their request is reported done."""

    def __init__(self, handle: Handle, hbm_budget=0, max_batch=0, max_pending=0,
                 stage_bytes=0, keep_factors=False, precision=0):
        self._handle = handle
        o = ServerOpts(hbm_budget, max_batch, max_pending, stage_bytes,
                       1 if keep_factors else 0, precision)
        self._s = _vp()
        handle._check(lib().qr_server_create(handle._h, ctypes.byref(o), ctypes.byref(self._s)))
        self._hold = {}
        self._buf = (ServerDone * 4096)()

    def close(self):
        if self._s:
            lib().qr_server_destroy(self._s)
            self._s = _vp()
            self._hold.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def clock(self) -> float:
        return float(lib().qr_server_clock(self._s))

    def submit(self, A, B, X) -> int:
        """Queue min ||B - A X||; X (n x nrhs host) receives the solution."""
        ap, lda = _host(A, "A")
        bp, ldb = _host(B, "B")
        xp, ldx = _host(X, "X")
        rid = _i64()
        self._handle._check(lib().qr_server_submit(self._s, A.shape[0], A.shape[1], B.shape[1],
                                                   ap, lda, bp, ldb, xp, ldx, ctypes.byref(rid)))
        self._hold[rid.value] = (A, B, X)
        return rid.value

    def resolve(self, factored_id: int, B, X) -> int:
        bp, ldb = _host(B, "B")
        xp, ldx = _host(X, "X")
        rid = _i64()
        self._handle._check(lib().qr_server_resolve(self._s, factored_id, B.shape[1], bp, ldb,
                                                    xp, ldx, ctypes.byref(rid)))
        self._hold[rid.value] = (B, X)
        return rid.value

    def release(self, factored_id: int):
        self._handle._check(lib().qr_server_release(self._s, factored_id))

    def poll(self, wait: bool = False):
        """List of finished requests: dicts with id, status, batch_size and the
        submit/start/end times (server clock, seconds)."""
        n = _i64()
        self._handle._check(lib().qr_server_poll(self._s, 1 if wait else 0, self._buf,
                                                 len(self._buf), ctypes.byref(n)))
        out = []
        for i in range(n.value):
            d = self._buf[i]
            self._hold.pop(d.id, None)
            out.append(dict(id=d.id, status=d.status, batch_size=d.batch_size,
                            submit_s=d.submit_s, start_s=d.start_s, end_s=d.end_s))
        return out

    def stats(self) -> dict:
        v = [_i64() for _ in range(4)]
        self._handle._check(lib().qr_server_stats(self._s, *[ctypes.byref(x) for x in v]))
        return dict(pending=v[0].value, admitted=v[1].value, running=v[2].value,
                    hbm_used=v[3].value)
