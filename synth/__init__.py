"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module draws random numbers and assembles test matrices; it holds none of
the QR arithmetic (no reflector generation, no factorisation, no triangular
solve of the method).  Both the oracle side and the GPU side consume the same
bytes from here.

Workloads (the paper has no experiments or datasets; these are the shapes the
hot path is measured on):

* ``gaussian(m, n, seed)``  -- i.i.d. N(0, 1) entries, column-major float64.
* ``conditioned(m, n, cond, seed)`` -- A = U diag(sigma) W^T with U the first n
  columns of a product of random Householder-type reflections, W a random
  orthogonal n x n matrix (Cayley transform of a random skew-symmetric matrix)
  and sigma geometrically spaced from 1 down to 1/cond.
* ``ls_rhs(A, seed, noise)`` -- x_true ~ N(0, 1)^n, b = A x_true + noise N(0,1)^m.
* ``serving_trace(...)``    -- Poisson arrivals of least-squares requests with
  m ~ U{64..4096}, n ~ U{8..256} (m >= n), 1..4 right-hand sides.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def gaussian(m: int, n: int, seed: int) -> np.ndarray:
    """m x n float64 array in Fortran (column-major) order, N(0, 1) entries.

    Column j is the j-th row of an (n, m) C-ordered draw, so the bytes are laid
    out column by column exactly as drawn."""
    g = rng(seed).standard_normal((n, m), dtype=np.float64)
    return g.T  # Fortran-ordered view, no copy


def int_matrix(m: int, n: int, seed: int, lo: int = -4, hi: int = 4) -> np.ndarray:
    """Small-integer matrix (exact Gram matrix A^T A in FP64)."""
    return np.asfortranarray(rng(seed).integers(lo, hi + 1, size=(m, n)).astype(np.float64))


def _reflect_rows(X: np.ndarray, v: np.ndarray) -> None:
    """X <- (I - 2 v v^T / v^T v) X, in place (an orthogonal reflection)."""
    w = v @ X
    X -= np.outer(v, w * (2.0 / float(v @ v)))


def random_orthogonal(n: int, seed: int) -> np.ndarray:
    """Random n x n orthogonal matrix: Cayley transform (I - S)(I + S)^{-1} of a
    skew-symmetric S with N(0, 1/2) entries.  I + S is always invertible."""
    g = rng(seed).standard_normal((n, n))
    S = (g - g.T) * 0.5
    I = np.eye(n)
    W = np.linalg.solve((I + S).T, (I - S).T).T  # (I - S)(I + S)^{-1}
    return np.asfortranarray(W)


def conditioned(m: int, n: int, cond: float, seed: int, n_reflections: int = 8) -> np.ndarray:
    """A = U diag(sigma) W^T with 2-norm condition number ``cond``.

    U = first n columns of H_1 H_2 ... H_k (k random reflections with N(0, 1)
    vectors), W random orthogonal, sigma_i = cond^{-(i-1)/(n-1)}."""
    r = rng(seed)
    if n > 1:
        sigma = cond ** (-np.arange(n, dtype=np.float64) / (n - 1))
    else:
        sigma = np.ones(1)
    W = random_orthogonal(n, seed + 7919)
    top = sigma[:, None] * W.T  # diag(sigma) W^T
    A = np.zeros((m, n), order="F")
    A[:n, :] = top
    vs = [r.standard_normal(m) for _ in range(n_reflections)]
    for v in reversed(vs):  # A = H_1 (H_2 (... H_k [top; 0]))
        _reflect_rows(A, v)
    return np.asfortranarray(A)


def ls_rhs(A: np.ndarray, seed: int, noise: float = 1e-6, nrhs: int = 1):
    """x_true ~ N(0,1)^(n x nrhs), b = A x_true + noise * N(0,1)^(m x nrhs)."""
    r = rng(seed)
    m, n = A.shape
    x = np.asfortranarray(r.standard_normal((n, nrhs)))
    b = np.asfortranarray(A @ x + noise * r.standard_normal((m, nrhs)))
    return x, b


@dataclass
class Request:
    rid: int
    arrival_s: float
    m: int
    n: int
    nrhs: int
    seed: int


def serving_trace(n_requests: int, qps: float, seed: int,
                  m_range=(64, 4096), n_range=(8, 256), nrhs_range=(1, 4)):
    """Poisson request stream: Exp(1/qps) inter-arrival times; m, n, nrhs
    uniform integers (n resampled until m >= n)."""
    r = rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += float(r.exponential(1.0 / qps)) if qps > 0 else 0.0
        while True:
            m = int(r.integers(m_range[0], m_range[1] + 1))
            n = int(r.integers(n_range[0], n_range[1] + 1))
            if m >= n:
                break
        k = int(r.integers(nrhs_range[0], nrhs_range[1] + 1))
        out.append(Request(i, t, m, n, k, seed * 1_000_003 + i))
    return out


def gaussian_device(m: int, n: int, seed: int, device="cuda"):
    """m x n column-major float64 torch tensor of N(0, 1) entries drawn on the
    device from torch's seeded generator (for batches too large to draw on the
    host); copy it to the host to hand the same values to the oracle."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return torch.randn((n, m), generator=g, dtype=torch.float64, device=device).t()
