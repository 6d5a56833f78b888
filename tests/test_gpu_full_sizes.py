"""Full-size parity at the measured shapes, where the oracle cannot factor the
whole matrix in seconds.

Checks that hold at any size, computed on the host in FP64 from the inputs:
 * the leading 1024 columns of R, V and T equal the oracle's factors of
   A[:, :1024] (the QR of a leading column block is the leading block of the
   QR: reflectors 0..1023 and the leading 1024 x 1024 block of T depend on
   those columns only), with the G5 gates and the elementwise gates of the
   parity tests;
 * sampled entries of R^T R equal the matching inner products a_i^T a_j;
 * G1 probe ||A z - Q (R z)|| / (||A||_F ||z||) <= 1e-13 and G2 probe
   ||Q^T (Q Z) - Z|| / ||Z|| <= 1e-13 on random Z (8 columns);
 * mixed-precision least squares at 65536 x 2048: backward error <= 1e-13
   against the FP64 original, without fallback where refinement converges.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.test_gpu_parity import check_against_oracle, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def miqr():
    import paper_1805_05278_amd as m
    h = m.Handle(0)
    yield m, h
    h.close()


def factor_and_check(m_, h, m, n, seed, b=0):
    A = synth.gaussian(m, n, seed)
    Ad = m_.to_colmajor(A)
    Td = m_.colmajor(n, n)
    h.factor(Ad, Td, h.opts(b=b))
    torch.cuda.synchronize()
    VR = Ad.cpu().numpy()
    R = np.triu(VR[:n, :n])
    # Leading 1024-column block against the oracle.
    k = 1024
    print("oracle of the %dx%d prefix" % (m, k), flush=True)
    fo = oracle.qr(np.asfortranarray(A[:, :k]))
    g = {"R": R[:k, :k], "V": np.tril(VR[:, :k], -1) + np.eye(m, k),
         "T": Td[:k, :k].cpu().numpy()}
    check_against_oracle(np.asfortranarray(A[:, :k]), g, tol_r=1e-13, tol_vt=1e-12, f=fo)
    lead = rel(oracle.normalize(g["R"])[0], oracle.normalize(fo.R)[0])
    del fo, g
    # Sampled Gram identities (RᵀR)_ij = a_i^T a_j.
    r = synth.rng(seed + 1)
    cols = np.linalg.norm(A, axis=0)
    worst = 0.0
    for _ in range(64):
        i, j = sorted(int(v) for v in r.integers(0, n, 2))
        g = R[: i + 1, i] @ R[: i + 1, j]
        worst = max(worst, abs(g - A[:, i] @ A[:, j]) / (cols[i] * cols[j]))
    assert worst <= 1e-13, worst
    # G1 / G2 probes through the factors.
    Z = synth.gaussian(n, 8, seed + 2)
    Y = m_.to_colmajor(R @ Z if m == n else np.vstack([R @ Z, np.zeros((m - n, 8))]))
    h.apply_q("N", Ad, Td, Y)
    torch.cuda.synchronize()
    g1 = np.linalg.norm(A @ Z - Y.cpu().numpy()) / (np.linalg.norm(A) * np.linalg.norm(Z))
    assert g1 <= 1e-13, g1
    W = synth.gaussian(m, 8, seed + 3)
    Wd = m_.to_colmajor(W)
    h.apply_q("N", Ad, Td, Wd)
    h.apply_q("T", Ad, Td, Wd)
    torch.cuda.synchronize()
    g2 = np.linalg.norm(Wd.cpu().numpy() - W) / np.linalg.norm(W)
    assert g2 <= 1e-13, g2
    return lead, worst, g1, g2


@pytest.mark.parametrize("b", [32, 64])
def test_square_16384(miqr, b):
    m_, h = miqr
    factor_and_check(m_, h, 16384, 16384, 31000 + b, b=b)


def test_tall_65536x8192(miqr):
    m_, h = miqr
    factor_and_check(m_, h, 65536, 8192, 32000)


def test_config1_1024x64_binary_tree(miqr):
    """1024 x 64, 8 row blocks of 128, binary tree: full oracle parity."""
    m_, h = miqr
    A = synth.gaussian(1024, 64, 33000)
    Ad = m_.to_colmajor(A)
    Td = m_.colmajor(64, 64)
    Q = m_.colmajor(1024, 64)
    sign = torch.empty(64, dtype=torch.float64, device="cuda")
    h.factor(Ad, Td, h.opts(leaf_rows=128, chain=1, arity=2, normalize=True, sign_out=sign, Q=Q))
    torch.cuda.synchronize()
    f = oracle.qr(A)
    Ro, Qo, _ = oracle.normalize(f.R, oracle.thin_q(f))
    R = np.triu(Ad.cpu().numpy()[:64])
    assert np.all(np.diag(R) >= 0)
    assert np.linalg.norm(R - Ro) / np.linalg.norm(Ro) <= 1e-14
    assert np.linalg.norm(Q.cpu().numpy() - Qo) / np.linalg.norm(Qo) <= 1e-13


# FP32 at kappa = 1e6 is the marginal cell: refinement may converge or fall back.
@pytest.mark.parametrize("prec,cond,expect_ok", [("fp32", 1e2, True), ("fp32", 1e6, None),
                                                 ("bf16", 1e2, True), ("fp32", 1e10, False),
                                                 ("bf16", 1e10, False)])
def test_mixed_65536x2048(miqr, prec, cond, expect_ok):
    m_, h = miqr
    p = {"fp32": m_.MIXED_FP32, "bf16": m_.MIXED_BF16}[prec]
    A = synth.conditioned(65536, 2048, cond, 34000 + int(np.log10(cond)))
    _, B = synth.ls_rhs(A, 34100, noise=1e-6, nrhs=1)
    Ad, Bd = m_.to_colmajor(A), m_.to_colmajor(B)
    st, info = h.lstsq(Ad, Bd, h.opts(precision=p))
    torch.cuda.synchronize()
    x = Bd.cpu().numpy()[:2048, 0]
    beta = oracle.backward_error(A, x, B[:, 0])
    assert beta <= 1e-13, beta
    assert info.backward_error <= 1e-13
    print("%s kappa=%g: status %d, %d iterations, fallback %d, beta %.2e"
          % (prec, cond, st, info.iterations, info.fallback, beta))
    if expect_ok:
        assert st == m_.OK and info.fallback == 0, (st, info)
    else:
        assert st in (m_.OK, m_.ENOCONV)
        assert (st == m_.ENOCONV) == (info.fallback == 1)
