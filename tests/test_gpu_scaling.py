"""Inputs far from unit scale: every entry of A multiplied by 1e-152 (column
norms around 1e-150, squared norms near 1e-300) or by 1e150 (squared norms
near 1e304).  The reflectors take 1 / ||.|| and 1 / (alpha - beta) from the
hardware reciprocal square root and reciprocal with Newton steps, so these
check that the whole FP64 range is covered.

Gates, all scale-invariant: R~ (D-normalised, relative), V and T against the
oracle's as for unit-scale inputs; batched solutions by the oracle's
backward error beta(x) <= 1e-13 and the forward error bound of the batched
tests.  Mixed FP32 cannot hold these values, so every problem must fall back
to FP64 (iterations -1) and equal the FP64 call's result bitwise.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.test_gpu_parity import check_against_oracle, gpu_factor

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
U = 2.0 ** -53
SCALES = [1e-152, 1e150]


@pytest.fixture(scope="module")
def miqr():
    import paper_1805_05278_amd as m
    h = m.Handle(0)
    yield m, h
    h.close()


# 256-row leaf blocks and tree nodes on the blocked MFMA body; a chain of
# column-step leaves; the EG recursion over a TSQR base case.
@pytest.mark.parametrize("scale", SCALES)
@pytest.mark.parametrize("m,n", [(20000, 48), (3001, 64), (1000, 300)])
def test_factor_scaled(miqr, m, n, scale):
    m_, h = miqr
    A = synth.gaussian(m, n, 4100 + m + n) * scale
    g = gpu_factor(m_, h, A)
    check_against_oracle(A, g)


def batched_inputs(scale):
    shapes = [(2000, 100, 2), (600, 200, 1), (333, 31, 3)]
    As = [synth.gaussian(m, n, 4300 + 2 * i) * scale for i, (m, n, _) in enumerate(shapes)]
    Bs = [synth.gaussian(m, k, 4301 + 2 * i) for i, (m, _, k) in enumerate(shapes)]
    return As, Bs


def run_batched(m_, h, As, Bs, precision):
    Ad = [m_.to_colmajor(A) for A in As]
    Bd = [m_.to_colmajor(B) for B in Bs]
    st, stat, its = h.lstsq_batched(Ad, Bd, h.opts(precision=precision), want_iters=True)
    torch.cuda.synchronize()
    return st, stat, its, [A.cpu().numpy() for A in Ad], [B.cpu().numpy() for B in Bd]


@pytest.mark.parametrize("scale", SCALES)
def test_batched_scaled(miqr, scale):
    m_, h = miqr
    As, Bs = batched_inputs(scale)
    st, stat, _, _, Bo = run_batched(m_, h, As, Bs, m_.FP64)
    assert st == m_.OK and stat == [0] * len(As)
    for A, B, b in zip(As, Bs, Bo):
        n = A.shape[1]
        x = b[:n]
        xo = oracle.lstsq(A, B)
        kappa = np.linalg.cond(A)
        nA = np.linalg.norm(A, 2)
        for c in range(B.shape[1]):
            assert oracle.backward_error(A, x[:, c], B[:, c]) <= 1e-13
            r = B[:, c] - A @ xo[:, c]
            bound = 100 * U * (kappa + kappa ** 2 * np.linalg.norm(r) / (nA * np.linalg.norm(xo[:, c])))
            err = np.linalg.norm(x[:, c] - xo[:, c]) / np.linalg.norm(xo[:, c])
            assert err <= bound, (A.shape, c, err, bound)


@pytest.mark.parametrize("scale", SCALES)
def test_batched_mixed_scaled_falls_back(miqr, scale):
    m_, h = miqr
    As, Bs = batched_inputs(scale)
    st, stat, its, Ao, Bo = run_batched(m_, h, As, Bs, m_.MIXED_FP32)
    assert st == m_.OK and stat == [0] * len(As)
    assert its == [-1] * len(As), its
    st64, _, _, Ao64, Bo64 = run_batched(m_, h, As, Bs, m_.FP64)
    assert st64 == m_.OK
    for a, b, a64, b64 in zip(Ao, Bo, Ao64, Bo64):
        assert np.array_equal(a, a64) and np.array_equal(b, b64)
