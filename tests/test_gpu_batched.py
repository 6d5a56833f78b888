"""Batched least squares (one persistent launch) against the oracle.

Gates per problem: forward error of X against the oracle's solution within
100 u (kappa + kappa^2 ||r|| / (||A|| ||x||)); ||R^T R - A^T A|| / ||A||^2 <=
1e-14 (G3); D-normalised R against the oracle's within 100 u kappa; backward
error beta(x) <= 1e-13.  Bitwise: a problem's result alone equals its result
inside a mixed batch (G9).
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


# Edge shapes: square, one block exactly, ragged tail, single column, fewer
# rows than a block, the widest n + nrhs, eight right-hand sides; panels of
# sixteen columns full, partial, and with right-hand sides in the panel's
# tile or in a tile of their own; n + nrhs at each queue boundary (128 / 129,
# 192 / 193, 256 / 257 columns) and at the limit of 320.
EDGE = [(256, 256, 1), (64, 64, 2), (65, 7, 1), (1000, 1, 1), (10, 5, 3), (129, 128, 4),
        (4096, 256, 4), (700, 312, 8), (64, 8, 1), (4095, 255, 2),
        (16, 16, 1), (17, 17, 3), (300, 15, 1), (300, 16, 1), (333, 31, 2), (1500, 124, 4),
        (1500, 125, 4), (900, 188, 4), (900, 189, 4), (2000, 253, 3), (2000, 253, 4),
        (520, 312, 8), (3000, 64, 8)]


def trace_shapes(k, seed):
    r = synth.rng(seed)
    out = []
    while len(out) < k:
        m = int(r.integers(64, 4097))
        n = int(r.integers(8, 257))
        if m >= n:
            out.append((m, n, int(r.integers(1, 5))))
    return out


def make(shapes, seed):
    As, Bs = [], []
    for i, (m, n, k) in enumerate(shapes):
        As.append(synth.gaussian(m, n, seed + 2 * i))
        Bs.append(synth.gaussian(m, k, seed + 2 * i + 1))
    return As, Bs


def run(m_, h, As, Bs):
    Ad = [m_.to_colmajor(A) for A in As]
    Bd = [m_.to_colmajor(B) for B in Bs]
    st, stat = h.lstsq_batched(Ad, Bd)
    torch.cuda.synchronize()
    return st, stat, [A.cpu().numpy() for A in Ad], [B.cpu().numpy() for B in Bd]


def check(A, B, Aout, Bout):
    m, n = A.shape
    x = Bout[:n]
    xo = oracle.lstsq(A, B)
    kappa = np.linalg.cond(A)
    nA = np.linalg.norm(A, 2)
    for c in range(B.shape[1]):
        r = B[:, c] - A @ xo[:, c]
        bound = 100 * U * (kappa + kappa ** 2 * np.linalg.norm(r) / (nA * np.linalg.norm(xo[:, c])))
        err = np.linalg.norm(x[:, c] - xo[:, c]) / np.linalg.norm(xo[:, c])
        assert err <= bound, (m, n, c, err, bound)
        assert oracle.backward_error(A, x[:, c], B[:, c]) <= 1e-13
    R = np.triu(Aout[:n, :n])
    AtA = A.T @ A
    g3 = np.linalg.norm(R.T @ R - AtA) / np.linalg.norm(A) ** 2
    Ro = oracle.qr(A, with_t=False).R
    g3o = np.linalg.norm(Ro.T @ Ro - AtA) / np.linalg.norm(A) ** 2
    # G3 (1e-14), or no worse than 4x the oracle's own figure where the
    # rounding of A^T A itself (about u sqrt(m)) approaches the gate.
    assert g3 <= max(1e-14, 4 * g3o), (m, n, g3, g3o)
    Rn, _, _ = oracle.normalize(R)
    Ro, _, _ = oracle.normalize(Ro)
    assert np.linalg.norm(Rn - Ro) / np.linalg.norm(Ro) <= 100 * U * kappa * np.sqrt(n)
    # rows below R are left as they were
    assert np.array_equal(np.tril(Aout, -1), np.tril(A, -1))


def test_batched_edge_shapes(miqr):
    m_, h = miqr
    As, Bs = make(EDGE, 500)
    st, stat, Ao, Bo = run(m_, h, As, Bs)
    assert st == m_.OK and stat == [0] * len(EDGE)
    for A, B, a, b in zip(As, Bs, Ao, Bo):
        check(A, B, a, b)


def test_batched_trace_mix_and_alone_bitwise(miqr):
    m_, h = miqr
    shapes = trace_shapes(40, 77)
    As, Bs = make(shapes, 900)
    st, stat, Ao, Bo = run(m_, h, As, Bs)
    assert st == m_.OK and stat == [0] * len(shapes)
    for A, B, a, b in zip(As, Bs, Ao, Bo):
        check(A, B, a, b)
    for i in (0, 7, 23, 39):
        st1, _, a1, b1 = run(m_, h, [As[i]], [Bs[i]])
        assert st1 == m_.OK
        assert np.array_equal(a1[0], Ao[i]) and np.array_equal(b1[0], Bo[i])


def test_batched_singular_problem_is_isolated(miqr):
    m_, h = miqr
    shapes = [(300, 40, 2), (500, 60, 1), (200, 30, 1)]
    As, Bs = make(shapes, 1300)
    As[1][:, 17] = 0.0
    st, stat, Ao, Bo = run(m_, h, As, Bs)
    assert st == m_.ESINGULAR
    assert stat[0] == 0 and stat[2] == 0 and stat[1] == 18
    check(As[0], Bs[0], Ao[0], Bo[0])
    check(As[2], Bs[2], Ao[2], Bo[2])
    assert np.array_equal(Ao[1], As[1])  # A of the singular problem is untouched


def test_batched_argument_errors(miqr):
    m_, h = miqr
    A = m_.colmajor(100, 300)
    B = m_.colmajor(100, 30)
    with pytest.raises(m_.MiqrError) as e:
        h.lstsq_batched([A], [B])
    assert e.value.status == m_.EINVAL
    A = m_.colmajor(400, 313)
    B = m_.colmajor(400, 8)
    with pytest.raises(m_.MiqrError) as e:
        h.lstsq_batched([A], [B])
    assert e.value.status == m_.EINVAL
    A = m_.colmajor(100, 10)
    B = m_.colmajor(100, 1)
    with pytest.raises(m_.MiqrError) as e:
        h.lstsq_batched([A], [B], h.opts(precision=7))
    assert e.value.status == m_.EINVAL
    with pytest.raises(m_.MiqrError) as e:
        h.lstsq_batched([A], [B], h.opts(normalize=1))
    assert e.value.status == m_.ENOTSUP
    assert h.lstsq_batched([], []) == (m_.OK, [])


def test_batched_full_trace_sampled(miqr):
    """The serving workload's full size: 10,000 problems (m in [64, 4096],
    n in [8, 256], 1-4 right-hand sides) in one call, inputs drawn on the
    device; 12 sampled problems checked against the oracle."""
    m_, h = miqr
    shapes = trace_shapes(10000, 4242)
    As = [synth.gaussian_device(m, n, 10 ** 6 + i) for i, (m, n, k) in enumerate(shapes)]
    Bs = [synth.gaussian_device(m, k, 2 * 10 ** 6 + i) for i, (m, n, k) in enumerate(shapes)]
    pick = [int(i) for i in synth.rng(5).choice(len(shapes), 12, replace=False)]
    host = {i: (As[i].cpu().numpy().copy(), Bs[i].cpu().numpy().copy()) for i in pick}
    st, stat = h.lstsq_batched(As, Bs)
    torch.cuda.synchronize()
    assert st == m_.OK and not any(stat)
    for i in pick:
        A, B = host[i]
        check(A, B, As[i].cpu().numpy(), Bs[i].cpu().numpy())
