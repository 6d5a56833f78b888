"""Plain FP64 CPU reference ("oracle") for the QR / least-squares hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the GPU library (``paper_1805_05278_amd``) and neither imports the other.

Contents (paper: "A 3D Parallel Algorithm for QR Decomposition"):

* ``qr``          -- unblocked Householder QR, the b = 1 right-looking algorithm
                     of Sec. 8.1 on one processor; output in the Householder
                     representation of Sec. 2.3 (V unit lower trapezoidal,
                     T upper triangular, R upper triangular).  The paper's
                     Elmroth-Gustavson recursion (Alg. 2) with its TSQR base case
                     (Sec. 5, App. C) reaches the same (V, T, R) in exact
                     arithmetic, so this is the plain definition of what the
                     GPU path computes.
* ``thin_q``      -- Q[:, :n] = (I - V T V^T)[I; 0].
* ``apply_q``     -- C <- Q C or Q^T C.
* ``lstsq``       -- min ||b - A x||_2 through the QR factors (the paper's
                     motivating use, Sec. 1); back substitution on R.
* ``normalize``   -- R~ = D R, Q~ = Q D with D = diag(sign(R_jj)), sign(0)=+1
                     (QR is unique only up to such D, App. C.2).
* ``backward_error`` -- beta(x) = ||A^T (b - A x)|| / (||A||_F (||A||_F ||x|| +
                     ||b - A x||)); the paper is silent on error measures.

The arithmetic lives in ``householder.c`` (plain C, FP64, compiled with
``-ffp-contract=off``); this module only marshals numpy arrays.  ``build()``
compiles it with gcc into ``oracle/_build``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "householder.c")
_BUILD_DIR = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD_DIR, "liboracle.so")
_lock = threading.Lock()
_lib = None

_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)


def compile_source(src: str, out: str) -> str:
    """Compile an oracle C source into a shared library (gcc, OpenMP,
    no floating-point contraction)."""
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-std=c99", "-o", tmp, src, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    """Compile householder.c into oracle/_build/liboracle.so."""
    os.makedirs(_BUILD_DIR, exist_ok=True)
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        compile_source(_SRC, _LIB_PATH)
    return _LIB_PATH


def open_library(path: str):
    """Load a compiled oracle library and declare its C signatures."""
    lib = ctypes.CDLL(path)
    lib.oracle_qr.argtypes = [_i64, _i64, _dp, _i64, _dp]
    lib.oracle_form_t.argtypes = [_i64, _i64, _dp, _i64, _dp, _dp, _i64]
    lib.oracle_apply_q.argtypes = [ctypes.c_char, _i64, _i64, _i64, _dp,
                                   _i64, _dp, _dp, _i64]
    lib.oracle_form_q.argtypes = [_i64, _i64, _dp, _i64, _dp, _dp, _i64]
    lib.oracle_trsv_upper.argtypes = [_i64, _i64, _dp, _i64, _dp, _i64]
    lib.oracle_lstsq.argtypes = [_i64, _i64, _i64, _dp, _i64, _dp, _i64, _dp]
    lib.oracle_num_threads.argtypes = []
    for f in ("oracle_qr", "oracle_form_t", "oracle_apply_q", "oracle_form_q",
              "oracle_trsv_upper", "oracle_lstsq", "oracle_num_threads"):
        getattr(lib, f).restype = ctypes.c_int
    return lib


def use_library(lib) -> None:
    """Route this module's functions through another compiled oracle library
    (``None`` restores the default).  Used by the tests that plant a mistake
    in a copy of the oracle source and check that the pins catch it."""
    global _lib
    with _lock:
        _lib = lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = open_library(_LIB_PATH)
            _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _fortran(a) -> np.ndarray:
    return np.array(a, dtype=np.float64, order="F", copy=True)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


class QRFactors:
    """Householder representation of a QR decomposition (Sec. 2.3).

    ``vr``  m x n, R in the upper triangle, V's strict lower trapezoid below it
    ``tau`` n reflector scalars, ``T`` n x n upper triangular kernel.
    """

    def __init__(self, vr: np.ndarray, tau: np.ndarray, T: np.ndarray):
        self.vr, self.tau, self.T = vr, tau, T

    @property
    def m(self) -> int:
        return self.vr.shape[0]

    @property
    def n(self) -> int:
        return self.vr.shape[1]

    @property
    def V(self) -> np.ndarray:
        n = self.n
        return np.tril(self.vr, -1) + np.eye(self.m, n)

    @property
    def R(self) -> np.ndarray:
        return np.triu(self.vr[: self.n, :])


def qr(A, with_t: bool = True) -> QRFactors:
    """Unblocked FP64 Householder QR of an m x n matrix, m >= n."""
    lib = _load()
    vr = _fortran(A)
    if vr.ndim != 2:
        raise ValueError("A must be 2-D")
    m, n = vr.shape
    if m < n:
        raise ValueError("oracle.qr requires m >= n")
    tau = np.zeros(n)
    rc = lib.oracle_qr(m, n, _ptr(vr), max(m, 1), _ptr(tau))
    if rc:
        raise RuntimeError("oracle_qr failed: %d" % rc)
    T = np.zeros((n, n), order="F")
    if with_t and n:
        rc = lib.oracle_form_t(m, n, _ptr(vr), max(m, 1), _ptr(tau), _ptr(T), max(n, 1))
        if rc:
            raise RuntimeError("oracle_form_t failed: %d" % rc)
    return QRFactors(vr, tau, T)


def thin_q(f: QRFactors) -> np.ndarray:
    lib = _load()
    m, n = f.m, f.n
    Q = np.zeros((m, n), order="F")
    rc = lib.oracle_form_q(m, n, _ptr(f.vr), max(m, 1), _ptr(f.tau), _ptr(Q), max(m, 1))
    if rc:
        raise RuntimeError("oracle_form_q failed: %d" % rc)
    return Q


def apply_q(f: QRFactors, C, trans: str = "T") -> np.ndarray:
    lib = _load()
    C = _fortran(C)
    if C.ndim == 1:
        C = C.reshape(-1, 1, order="F")
    m, n = f.m, f.n
    if C.shape[0] != m:
        raise ValueError("C must have m rows")
    rc = lib.oracle_apply_q(trans.encode(), m, n, C.shape[1], _ptr(f.vr), max(m, 1),
                            _ptr(f.tau), _ptr(C), max(m, 1))
    if rc:
        raise RuntimeError("oracle_apply_q failed: %d" % rc)
    return C


def solve_r(R, C) -> np.ndarray:
    """Back substitution with the upper triangle of R (n x n)."""
    lib = _load()
    R = _fortran(R)
    C = _fortran(C)
    vec = C.ndim == 1
    if vec:
        C = C.reshape(-1, 1, order="F")
    n = R.shape[1]
    rc = lib.oracle_trsv_upper(n, C.shape[1], _ptr(R), max(R.shape[0], 1), _ptr(C),
                               max(C.shape[0], 1))
    if rc:
        raise ZeroDivisionError("R[%d,%d] == 0" % (rc - 1, rc - 1))
    return C[:, 0] if vec else C


def lstsq(A, B):
    """x = argmin ||B - A x||_2 per column, via Householder QR."""
    lib = _load()
    vr = _fortran(A)
    m, n = vr.shape
    Bf = _fortran(B)
    vec = Bf.ndim == 1
    if vec:
        Bf = Bf.reshape(-1, 1, order="F")
    tau = np.zeros(n)
    rc = lib.oracle_lstsq(m, n, Bf.shape[1], _ptr(vr), max(m, 1), _ptr(Bf), max(m, 1),
                          _ptr(tau))
    if rc > 0:
        raise ZeroDivisionError("R[%d,%d] == 0" % (rc - 1, rc - 1))
    if rc < 0:
        raise RuntimeError("oracle_lstsq failed: %d" % rc)
    x = np.array(Bf[:n, :], order="F")
    return x[:, 0] if vec else x


def normalize(R, Q=None):
    """Return (R~, Q~, d) with d_j = sign(R_jj) (sign(0) = +1), R~ = diag(d) R,
    Q~ = Q diag(d); R~ has a non-negative diagonal."""
    R = np.asarray(R, dtype=np.float64)
    d = np.where(np.diag(R) < 0.0, -1.0, 1.0)
    Rn = d[:, None] * R
    Qn = None if Q is None else np.asarray(Q) * d[None, :]
    return Rn, Qn, d


def backward_error(A, x, b) -> float:
    """Normal-equations backward-error measure beta(x), FP64."""
    A = np.asarray(A, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    r = b - A @ x
    nA = np.linalg.norm(A)
    den = nA * (nA * np.linalg.norm(x) + np.linalg.norm(r))
    if den == 0.0:
        return 0.0
    return float(np.linalg.norm(A.T @ r) / den)
