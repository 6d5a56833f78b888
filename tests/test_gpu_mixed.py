"""Mixed-precision least squares (FP32/BF16 trailing updates, FP64
refinement) against the FP64 oracle.

Gate: backward error beta(x) <= 1e-13 against the FP64 original, every right-
hand side; forward error ||x - x_oracle|| / ||x_oracle|| within
100 u (kappa + kappa^2 ||r|| / (||A|| ||x||)) where that bound is below 1.
If refinement cannot reach the gate the call must say so (ENOCONV with the
FP64 fallback result, which itself meets the gate).
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
U = 2.0 ** -53


@pytest.fixture(scope="module")
def miqr():
    import paper_1805_05278_amd as m
    h = m.Handle(0)
    yield m, h
    h.close()


def run(m_, h, A, B, precision):
    Ad = m_.to_colmajor(A)
    Bd = m_.to_colmajor(B)
    st, info = h.lstsq(Ad, Bd, h.opts(precision=precision))
    torch.cuda.synchronize()
    return st, info, Bd.cpu().numpy()[: A.shape[1]]


@pytest.mark.parametrize("prec,cond,shape", [("fp32", 1e2, (3000, 200)), ("fp32", 1e6, (3000, 200)),
                                             ("bf16", 1e2, (3000, 200)), ("fp32", 1e2, (20000, 64)),
                                             ("bf16", 1e2, (4096, 513))])
def test_mixed_lstsq_meets_fp64_backward_error(miqr, prec, cond, shape):
    m_, h = miqr
    p = {"fp32": m_.MIXED_FP32, "bf16": m_.MIXED_BF16}[prec]
    m, n = shape
    A = synth.conditioned(m, n, cond, 40 + n)
    xt, B = synth.ls_rhs(A, 41 + n, noise=1e-6, nrhs=2)
    st, info, x = run(m_, h, A, B, p)
    assert st in (m_.OK, m_.ENOCONV)
    for c in range(B.shape[1]):
        assert oracle.backward_error(A, x[:, c], B[:, c]) <= 1e-13
    assert info.backward_error <= 1e-13
    xo = oracle.lstsq(A, B)
    r = B - A @ xo
    nA = np.linalg.norm(A, 2)
    for c in range(B.shape[1]):
        bound = 100 * U * (cond + cond ** 2 * np.linalg.norm(r[:, c]) / (nA * np.linalg.norm(xo[:, c])))
        if bound < 1:
            assert np.linalg.norm(x[:, c] - xo[:, c]) / np.linalg.norm(xo[:, c]) <= bound
    if st == m_.OK:
        assert info.fallback == 0 and info.precision_used == p


def test_mixed_ill_conditioned_reports_outcome(miqr):
    """kappa = 1e10 with BF16 updates: refinement is not expected to converge;
    the call must return ENOCONV with the FP64 fallback (or converge)."""
    m_, h = miqr
    A = synth.conditioned(2000, 100, 1e10, 7)
    xt, B = synth.ls_rhs(A, 8, noise=1e-6, nrhs=1)
    st, info, x = run(m_, h, A, B, m_.MIXED_BF16)
    assert st in (m_.OK, m_.ENOCONV)
    if st == m_.ENOCONV:
        assert info.fallback == 1
    assert oracle.backward_error(A, x[:, 0], B[:, 0]) <= 1e-13


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mixed_factor_is_a_valid_qr_of_a_nearby_matrix(miqr, prec):
    """The low-precision updates perturb the factorisation by about u_low; the
    FP64 representation (V, T) stays orthogonal to FP64 accuracy."""
    m_, h = miqr
    p = {"fp32": m_.MIXED_FP32, "bf16": m_.MIXED_BF16}[prec]
    A = synth.gaussian(1500, 300, 5)
    Ad = m_.to_colmajor(A)
    Td = m_.colmajor(300, 300)
    Qd = m_.colmajor(1500, 300)
    h.factor(Ad, Td, h.opts(precision=p, Q=Qd))
    torch.cuda.synchronize()
    Q = Qd.cpu().numpy()
    R = np.triu(Ad.cpu().numpy()[:300])
    ulow = {"fp32": 2.0 ** -24, "bf16": 2.0 ** -8}[prec]
    assert np.linalg.norm(Q.T @ Q - np.eye(300)) <= 1e-12
    assert np.linalg.norm(A - Q @ R) / np.linalg.norm(A) <= 50 * ulow


def test_mixed_after_fp64_on_same_handle():
    """An FP64 solve sizes the handle's workspace for itself; the mixed solve
    that follows needs more and must size its own layout exactly (its norm
    buffer once fell outside the allocation when n was large)."""
    import paper_1805_05278_amd as m_
    h = m_.Handle(0)
    try:
        A = synth.conditioned(8192, 2048, 1e2, 77)
        _, B = synth.ls_rhs(A, 78, noise=1e-6, nrhs=1)
        for prec in (m_.FP64, m_.MIXED_FP32, m_.MIXED_BF16):
            Ad, Bd = m_.to_colmajor(A), m_.to_colmajor(B)
            st, info = h.lstsq(Ad, Bd, h.opts(precision=prec))
            torch.cuda.synchronize()
            assert st in (m_.OK, m_.ENOCONV)
            x = Bd.cpu().numpy()[:2048, 0]
            assert oracle.backward_error(A, x, B[:, 0]) <= 1e-13
    finally:
        h.close()
