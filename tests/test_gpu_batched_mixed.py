"""Mixed-precision batched least squares (FP32 working copy with FP32 or BF16
MFMA products, FP64 refinement per problem) against the FP64 oracle.

Gates per right-hand side: backward error beta(x) <= 1e-13 by the oracle's
measure; forward error against the oracle's solution within what that
backward error implies, 1e-13 (||A||_F / sigma_min)^2 (1 + ||r|| / (||A||_F
||x||)) (A^T (b - A x) = A^T A (x* - x) bounds ||x - x*|| by
||A^T r|| / sigma_min^2), plus the oracle's own 100 u (kappa + kappa^2 ||r|| /
(||A|| ||x||)).  The R written into A comes from the
low-precision factorisation: ||R^T R - A^T A|| / ||A||^2 within 1e-5 (FP32
products) or 5e-2 (BF16 products).  Bitwise: a problem's result alone equals
its result inside a mixed batch, and a problem solved again in FP64 equals
the FP64 call's result.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def miqr():
    import paper_1805_05278_amd as m
    h = m.Handle(0)
    yield m, h
    h.close()


def precs(m_):
    return {"fp32": (m_.MIXED_FP32, 1e-5), "bf16": (m_.MIXED_BF16, 5e-2)}


SHAPES = [(64, 8, 1), (65, 7, 2), (300, 16, 1), (333, 31, 2), (1500, 124, 4), (1500, 125, 4),
          (900, 189, 4), (2000, 253, 4), (520, 312, 8), (4096, 256, 4), (17, 17, 3), (10, 5, 3)]


def make(shapes, seed, cond=None):
    As, Bs = [], []
    for i, (m, n, k) in enumerate(shapes):
        if cond is None:
            A = synth.gaussian(m, n, seed + 2 * i)
            B = synth.gaussian(m, k, seed + 2 * i + 1)
        else:
            A = synth.conditioned(m, n, cond, seed + 2 * i)
            _, B = synth.ls_rhs(A, seed + 2 * i + 1, noise=1e-6, nrhs=k)
        As.append(A)
        Bs.append(B)
    return As, Bs


def run(m_, h, As, Bs, precision):
    Ad = [m_.to_colmajor(A) for A in As]
    Bd = [m_.to_colmajor(B) for B in Bs]
    st, stat, its = h.lstsq_batched(Ad, Bd, h.opts(precision=precision), want_iters=True)
    torch.cuda.synchronize()
    return st, stat, its, [A.cpu().numpy() for A in Ad], [B.cpu().numpy() for B in Bd]


def check(A, B, Aout, Bout, g3_gate):
    m, n = A.shape
    x = Bout[:n]
    xo = oracle.lstsq(A, B)
    kappa = np.linalg.cond(A)
    nA = np.linalg.norm(A, 2)
    nF = np.linalg.norm(A)
    smin = np.linalg.svd(A, compute_uv=False)[-1]
    for c in range(B.shape[1]):
        assert oracle.backward_error(A, x[:, c], B[:, c]) <= 1e-13, (m, n, c)
        r = B[:, c] - A @ xo[:, c]
        xn = np.linalg.norm(xo[:, c])
        bound = (1e-13 * (nF / smin) ** 2 * (1 + np.linalg.norm(r) / (nF * xn)) +
                 100 * 2.0 ** -53 * (kappa + kappa ** 2 * np.linalg.norm(r) / (nA * xn)))
        err = np.linalg.norm(x[:, c] - xo[:, c]) / np.linalg.norm(xo[:, c])
        assert err <= max(bound, 1e-15), (m, n, c, err, bound)
    R = np.triu(Aout[:n, :n])
    g3 = np.linalg.norm(R.T @ R - A.T @ A) / np.linalg.norm(A) ** 2
    assert g3 <= g3_gate, (m, n, g3)
    assert np.array_equal(np.tril(Aout, -1), np.tril(A, -1))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mixed_batched_edge_shapes_meet_fp64_backward_error(miqr, prec):
    m_, h = miqr
    p, gate = precs(m_)[prec]
    As, Bs = make(SHAPES, 7100)
    st, stat, its, Ao, Bo = run(m_, h, As, Bs, p)
    assert st == m_.OK and stat == [0] * len(SHAPES)
    # Gaussian problems are well conditioned: refinement, not the fallback.
    assert all(i >= 0 for i in its), its
    for A, B, a, b in zip(As, Bs, Ao, Bo):
        check(A, B, a, b, gate)


@pytest.mark.parametrize("prec,cond", [("fp32", 1e2), ("fp32", 1e6), ("bf16", 1e2)])
def test_mixed_batched_conditioned(miqr, prec, cond):
    """Matrices of prescribed condition with near-consistent right-hand sides
    (the mixed least-squares workload's recipe at batched sizes)."""
    m_, h = miqr
    p, gate = precs(m_)[prec]
    shapes = [(2000, 100, 2), (800, 200, 1), (4096, 256, 4)]
    As, Bs = make(shapes, 7300, cond=cond)
    st, stat, its, Ao, Bo = run(m_, h, As, Bs, p)
    assert st == m_.OK and stat == [0] * len(shapes)
    for A, B, a, b, i in zip(As, Bs, Ao, Bo, its):
        # R's Gram residual is a backward error of the factorisation in the
        # working precision, whatever the conditioning.
        check(A, B, a, b, gate if i >= 0 else 1e-13)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mixed_batched_alone_equals_in_mix_bitwise(miqr, prec):
    m_, h = miqr
    p, _ = precs(m_)[prec]
    r = synth.rng(81)
    shapes = []
    while len(shapes) < 30:
        m, n = int(r.integers(64, 4097)), int(r.integers(8, 257))
        if m >= n:
            shapes.append((m, n, int(r.integers(1, 5))))
    As, Bs = make(shapes, 7500)
    st, stat, its, Ao, Bo = run(m_, h, As, Bs, p)
    assert st == m_.OK and stat == [0] * len(shapes)
    for i in (0, 9, 17, 29):
        st1, _, its1, a1, b1 = run(m_, h, [As[i]], [Bs[i]], p)
        assert st1 == m_.OK and its1[0] == its[i]
        assert np.array_equal(a1[0], Ao[i]) and np.array_equal(b1[0], Bo[i])


def test_mixed_batched_fallback_equals_fp64(miqr):
    """A problem far too ill-conditioned for BF16 products is solved again in
    FP64 (iterations -1), with exactly the FP64 call's result; its neighbour
    in the batch still refines."""
    m_, h = miqr
    A1 = synth.conditioned(1200, 100, 1e12, 7701)
    _, B1 = synth.ls_rhs(A1, 7702, noise=1e-6, nrhs=2)
    A0 = synth.gaussian(900, 60, 7703)
    B0 = synth.gaussian(900, 1, 7704)
    st, stat, its, Ao, Bo = run(m_, h, [A0, A1], [B0, B1], m_.MIXED_BF16)
    assert st == m_.OK and stat == [0, 0]
    assert its[0] >= 0 and its[1] == -1
    st64, _, _, Ao64, Bo64 = run(m_, h, [A1], [B1], m_.FP64)
    assert st64 == m_.OK
    assert np.array_equal(Ao[1], Ao64[0]) and np.array_equal(Bo[1], Bo64[0])
    check(A0, B0, Ao[0], Bo[0], 5e-2)


def test_mixed_batched_singular_goes_to_fp64(miqr):
    m_, h = miqr
    shapes = [(300, 40, 2), (500, 60, 1)]
    As, Bs = make(shapes, 7900)
    As[1][:, 17] = 0.0
    st, stat, its, Ao, Bo = run(m_, h, As, Bs, m_.MIXED_FP32)
    assert st == m_.ESINGULAR
    assert stat == [0, 18] and its[1] == -1
    check(As[0], Bs[0], Ao[0], Bo[0], 1e-5)
    assert np.array_equal(Ao[1], As[1])
