"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances (u = 2^-53), per quantity, from the project's gates:
  R (after normalising diag >= 0): ||dR|| / ||R|| <= 1e-13             (G5)
  V, T (same reflector sign rule on both sides): <= 1e-12             (G5)
  thin Q: ||dQ|| / ||Q|| <= 1e-12; ||A - QR|| / ||A|| <= 1e-14 (n <= 256)
  least squares: backward error beta(x) <= 1e-13                      (G8)
  tuning invariance: any (b, leaf_rows, chain, arity) within 1e-13   (G10)
Exact zeros (R and T strictly lower) are checked bitwise (G4).
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rel(a, b):
    d = np.linalg.norm(np.asarray(a) - np.asarray(b))
    nb = np.linalg.norm(b)
    return d if nb == 0 else d / nb


@pytest.fixture(scope="module")
def miqr():
    import paper_1805_05278_amd as m
    h = m.Handle(0)
    yield m, h
    h.close()


def gpu_factor(m_, h, A, with_q=False, normalize=False, **tune):
    mm, nn = A.shape
    Ad = m_.to_colmajor(A)
    Td = m_.colmajor(nn, nn)
    Qd = m_.colmajor(mm, nn) if with_q else None
    sd = torch.empty(nn, dtype=torch.float64, device="cuda") if normalize else None
    opts = h.opts(Q=Qd, normalize=normalize, sign_out=sd, **tune)
    h.factor(Ad, Td, opts)
    torch.cuda.synchronize()
    vr = Ad.cpu().numpy()
    out = {"vr": vr, "V": np.tril(vr, -1) + np.eye(mm, nn), "R": np.triu(vr[:nn]),
           "T": Td.cpu().numpy()}
    if with_q:
        out["Q"] = Qd.cpu().numpy()
    if normalize:
        out["d"] = sd.cpu().numpy()
    return out


def check_against_oracle(A, g, tol_r=1e-13, tol_vt=1e-12):
    f = oracle.qr(A)
    assert rel(oracle.normalize(g["R"])[0], oracle.normalize(f.R)[0]) <= tol_r
    assert rel(g["V"], f.V) <= tol_vt
    assert rel(g["T"], f.T) <= tol_vt
    assert np.all(np.tril(g["T"], -1) == 0.0)
    return f


# 20000 x 48, 40000 x 40 and 70000 x 64 take 256-row leaf blocks and the
# blocked MFMA block QR for first blocks and tree nodes (40 columns: a
# partial 16-column sub-panel; five children stack 160 rows).
SHAPES_TSQR = [(1, 1), (5, 3), (64, 64), (100, 7), (130, 64), (1000, 33), (1024, 64),
               (3001, 64), (20000, 48), (40000, 40), (70000, 64)]


@pytest.mark.parametrize("m,n", SHAPES_TSQR)
def test_tsqr_panel_matches_oracle(miqr, m, n):
    m_, h = miqr
    A = synth.gaussian(m, n, 100 + m + n)
    g = gpu_factor(m_, h, A)
    check_against_oracle(A, g)


def test_config1_binary_tree_normalised(miqr):
    """1024 x 64, 8 leaf blocks of 128 rows, binary tree; R with diag >= 0."""
    m_, h = miqr
    A = synth.gaussian(1024, 64, 1000)
    g = gpu_factor(m_, h, A, with_q=True, normalize=True, leaf_rows=128, chain=1, arity=2)
    f = oracle.qr(A)
    Rn, Qn, d = oracle.normalize(f.R, oracle.thin_q(f))
    assert np.all(np.diag(g["R"]) >= 0)
    assert rel(g["R"], Rn) <= 1e-13
    assert np.array_equal(g["d"], d)
    assert rel(g["V"], f.V) <= 1e-12 and rel(g["T"], f.T) <= 1e-12
    assert rel(g["Q"], Qn) <= 1e-12
    assert np.linalg.norm(A - g["Q"] @ g["R"]) / np.linalg.norm(A) <= 1e-14
    assert np.linalg.norm(g["Q"].T @ g["Q"] - np.eye(64)) <= 1e-13


@pytest.mark.parametrize("m,n", [(200, 65), (300, 100), (1000, 256), (1500, 300), (4096, 513),
                                 (33000, 100)])
def test_eg_recursion_matches_oracle(miqr, m, n):
    m_, h = miqr
    A = synth.gaussian(m, n, 200 + n)
    g = gpu_factor(m_, h, A)
    check_against_oracle(A, g)


@pytest.mark.parametrize("m,n", [(777, 64), (2000, 200)])
def test_thin_q(miqr, m, n):
    m_, h = miqr
    A = synth.gaussian(m, n, 300 + n)
    g = gpu_factor(m_, h, A, with_q=True)
    f = oracle.qr(A)
    Q = oracle.thin_q(f)
    assert rel(g["Q"], Q) <= 1e-12
    assert np.linalg.norm(A - g["Q"] @ g["R"]) / np.linalg.norm(A) <= 1e-14


@pytest.mark.parametrize("tune", [dict(b=16), dict(b=32), dict(leaf_rows=128), dict(leaf_rows=256),
                                  dict(chain=3, arity=3), dict(chain=1, arity=2),
                                  dict(b=48, chain=2, arity=5)])
def test_tuning_invariance(miqr, tune):
    m_, h = miqr
    A = synth.gaussian(5000, 150, 77)
    base = gpu_factor(m_, h, A)
    g = gpu_factor(m_, h, A, **tune)
    assert rel(oracle.normalize(g["R"])[0], oracle.normalize(base["R"])[0]) <= 1e-13
    assert rel(g["V"], base["V"]) <= 1e-13 * 10
    assert rel(g["T"], base["T"]) <= 1e-13 * 10


@pytest.mark.parametrize("trans", ["T", "N"])
def test_apply_q(miqr, trans):
    m_, h = miqr
    A = synth.gaussian(900, 130, 5)
    C = synth.gaussian(900, 3, 6)
    f = oracle.qr(A)
    Ad = m_.to_colmajor(A)
    Td = m_.colmajor(130, 130)
    h.factor(Ad, Td)
    Cd = m_.to_colmajor(C)
    h.apply_q(trans, Ad, Td, Cd)
    ref = oracle.apply_q(f, C, trans)
    assert rel(Cd.cpu().numpy(), ref) <= 1e-13


@pytest.mark.parametrize("m,n,nrhs", [(500, 40, 1), (3000, 200, 3), (20000, 64, 2)])
def test_lstsq(miqr, m, n, nrhs):
    m_, h = miqr
    A = synth.conditioned(m, n, 1e4, 9 + n)
    xt, B = synth.ls_rhs(A, 10 + n, noise=1e-6, nrhs=nrhs)
    Ad = m_.to_colmajor(A)
    Bd = m_.to_colmajor(B)
    st, info = h.lstsq(Ad, Bd)
    assert st == m_.OK
    x = Bd.cpu().numpy()[:n]
    xo = oracle.lstsq(A, B)
    for c in range(nrhs):
        assert oracle.backward_error(A, x[:, c], B[:, c]) <= 1e-13
    assert rel(x, xo) <= 1e-10
    assert info.backward_error <= 1e-13


def test_lstsq_singular(miqr):
    m_, h = miqr
    A = synth.gaussian(300, 20, 3).copy()
    A[:, 5] = 0.0
    Ad = m_.to_colmajor(A)
    Bd = m_.to_colmajor(np.ones((300, 1)))
    st, info = h.lstsq(Ad, Bd)
    assert st == m_.ESINGULAR and info.singular_index == 6


def test_solve_r(miqr):
    m_, h = miqr
    A = synth.gaussian(400, 150, 8)
    f = oracle.qr(A)
    X = synth.gaussian(150, 2, 9)
    Rd = m_.to_colmajor(f.vr)
    Xd = m_.to_colmajor(X)
    h.solve_r(Rd, Xd)
    ref = oracle.solve_r(f.R, X)
    assert rel(Xd.cpu().numpy(), ref) <= 1e-12


def test_degenerate_inputs_invariants(miqr):
    """Exactly degenerate inputs: only the invariants are compared (the
    reconstruction reflects where the unblocked rule would not)."""
    m_, h = miqr
    A = np.vstack([np.eye(8), np.zeros((40, 8))])
    g = gpu_factor(m_, h, A, with_q=True)
    assert np.abs(A - g["Q"] @ g["R"]).max() <= 1e-15
    assert np.linalg.norm(g["Q"].T @ g["Q"] - np.eye(8)) <= 1e-14
    B = synth.gaussian(100, 10, 4).copy()
    B[:, 3] = 0.0
    g = gpu_factor(m_, h, B, with_q=True)
    assert np.linalg.norm(B - g["Q"] @ g["R"]) <= 1e-13 * np.linalg.norm(B)
    assert np.linalg.norm(g["Q"].T @ g["Q"] - np.eye(10)) <= 1e-13
