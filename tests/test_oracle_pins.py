"""Pins of the FP64 CPU oracle against facts that do not come from the oracle.

Each check rests on something independent of the oracle's own code:

* a hand-derived worked example (tests/golden/householder_3x2.txt);
* brute force in extended precision (mpmath modified Gram-Schmidt, 50 digits);
* LAPACK routines called through scipy (dgeqrt returns the same Householder
  representation with the same reflector sign rule; dorgqr the thin Q);
* closed forms: one column, orthonormal columns times a diagonal, [I; 0];
* exact identities: R^T R = A^T A for small integer A (exact Gram matrix),
  T^{-1} + T^{-T} = V^T V (the closed form for T in Sec. 2.3, read with a
  strictly upper triangular part), A = QR, Q^T Q = I, exact zeros.

The numbered gates (G1 ...) are the tolerances stated for the whole project.
"""
import os

import mpmath
import numpy as np
import pytest
import scipy.linalg as sla
from scipy.linalg import lapack

import oracle
import synth

U = 2.0 ** -53
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "householder_3x2.txt")
GOLDEN_BETA = os.path.join(os.path.dirname(__file__), "golden", "backward_error_3x2.txt")


def rel(a, b):
    """||a - b||_F / ||b||_F, with 0 when both are zero."""
    d = np.linalg.norm(np.asarray(a) - np.asarray(b))
    nb = np.linalg.norm(b)
    return d if nb == 0.0 else d / nb


def read_golden(path):
    out = {}
    with open(path) as f:
        lines = [ln.strip() for ln in f if ln.strip() and not ln.startswith("#")]
    i = 0
    while i < len(lines):
        name, r, c = lines[i].split()
        r, c = int(r), int(c)
        vals = [list(map(float, lines[i + 1 + k].split())) for k in range(r)]
        out[name] = np.array(vals).reshape(r, c)
        i += 1 + r
    return out


# ----------------------------------------------------------------- golden
def test_golden_3x2_worked_example():
    g = read_golden(GOLDEN)
    f = oracle.qr(g["A"])
    np.testing.assert_allclose(f.R, g["R"], rtol=0, atol=4 * U * 8)
    np.testing.assert_allclose(f.V, g["V"], rtol=0, atol=4 * U)
    np.testing.assert_allclose(f.tau, g["tau"].ravel(), rtol=0, atol=4 * U * 2)
    np.testing.assert_allclose(f.T, g["T"], rtol=0, atol=8 * U * 2)
    np.testing.assert_allclose(oracle.thin_q(f), g["Q"], rtol=0, atol=8 * U)
    x = oracle.lstsq(g["A"], g["b"])
    np.testing.assert_allclose(x, g["x"], rtol=0, atol=64 * U)


# ------------------------------------------------------------- brute force
def mgs_mp(A, dps=50):
    """Modified Gram-Schmidt in mpmath; returns Q (m x n) and R (n x n, diag > 0)."""
    with mpmath.workdps(dps):
        m, n = A.shape
        Q = [[mpmath.mpf(float(A[i, j])) for j in range(n)] for i in range(m)]
        R = [[mpmath.mpf(0)] * n for _ in range(n)]
        for j in range(n):
            for k in range(j):
                s = mpmath.fsum(Q[i][k] * Q[i][j] for i in range(m))
                R[k][j] += s
                for i in range(m):
                    Q[i][j] -= s * Q[i][k]
            # one re-orthogonalisation pass for safety
            for k in range(j):
                s = mpmath.fsum(Q[i][k] * Q[i][j] for i in range(m))
                R[k][j] += s
                for i in range(m):
                    Q[i][j] -= s * Q[i][k]
            nrm = mpmath.sqrt(mpmath.fsum(Q[i][j] ** 2 for i in range(m)))
            R[j][j] = nrm
            for i in range(m):
                Q[i][j] /= nrm
        return (np.array([[float(Q[i][j]) for j in range(n)] for i in range(m)]),
                np.array([[float(R[i][j]) for j in range(n)] for i in range(n)]))


@pytest.mark.parametrize("m,n,seed,cond", [(4, 1, 1, None), (5, 3, 2, None), (8, 4, 3, None),
                                           (12, 6, 4, None), (10, 5, 5, 1e3), (6, 6, 6, 1e2)])
def test_g6_against_mpmath_gram_schmidt(m, n, seed, cond):
    A = synth.gaussian(m, n, seed) if cond is None else synth.conditioned(m, n, cond, seed, 3)
    f = oracle.qr(A)
    Rn, Qn, _ = oracle.normalize(f.R, oracle.thin_q(f))
    Qgs, Rgs = mgs_mp(np.asarray(A))
    nA = np.linalg.norm(A)
    assert np.abs(Rn - Rgs).max() / nA <= 1e-14
    assert np.abs(Qn - Qgs).max() <= 1e-12


# ----------------------------------------------------------------- LAPACK
@pytest.mark.parametrize("m,n,seed", [(1, 1, 0), (7, 7, 1), (64, 17, 2), (300, 40, 3), (129, 64, 4)])
def test_matches_lapack_dgeqrt(m, n, seed):
    A = np.asfortranarray(synth.gaussian(m, n, seed))
    f = oracle.qr(A)
    vr, t, info = lapack.dgeqrt(n, A.copy(order="F"))
    assert info == 0
    V = np.tril(vr, -1) + np.eye(m, n)
    R = np.triu(vr[:n])
    assert rel(f.R, R) <= 1e-13
    assert rel(f.V, V) <= 1e-12
    assert rel(f.T, np.triu(t)) <= 1e-12


@pytest.mark.parametrize("m,n,seed", [(50, 9, 5), (200, 31, 6)])
def test_thin_q_matches_lapack_dorgqr(m, n, seed):
    A = np.asfortranarray(synth.gaussian(m, n, seed))
    qr_, tau, work, info = lapack.dgeqrf(A.copy(order="F"))
    Q, work, info2 = lapack.dorgqr(qr_[:, :n].copy(order="F"), tau)
    f = oracle.qr(A)
    np.testing.assert_allclose(f.tau, tau, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(oracle.thin_q(f), Q[:, :n], rtol=0, atol=1e-13)


# ------------------------------------------------------------ closed forms
def test_single_column_closed_form():
    x = np.array([2.0, -1.0, 2.0, 4.0])  # ||x|| = 5
    f = oracle.qr(x.reshape(-1, 1))
    alpha, nrm = 2.0, 5.0
    beta = -nrm
    assert f.R[0, 0] == beta
    assert abs(f.tau[0] - (beta - alpha) / beta) <= U
    np.testing.assert_allclose(f.V[1:, 0], x[1:] / (alpha - beta), rtol=0, atol=2 * U)
    # negative leading entry reflects to +||x||
    f2 = oracle.qr(-x.reshape(-1, 1))
    assert f2.R[0, 0] == nrm
    # signed zero counts as positive
    z = np.array([-0.0, 3.0, 4.0])
    assert oracle.qr(z.reshape(-1, 1)).R[0, 0] == -5.0


def hadamard(k):
    H = np.array([[1.0]])
    for _ in range(k):
        H = np.block([[H, H], [H, -H]])
    return H


def test_orthonormal_times_diagonal():
    Q0 = hadamard(4)[:, :6] / 4.0  # 16 x 6, exactly orthonormal columns
    d = np.array([3.0, -0.5, 2.0, -7.0, 1e-3, 4.0])
    A = Q0 * d[None, :]
    f = oracle.qr(A)
    Rn, Qn, _ = oracle.normalize(f.R, oracle.thin_q(f))
    np.testing.assert_allclose(Rn, np.diag(np.abs(d)), rtol=0, atol=8 * U * 7)
    np.testing.assert_allclose(np.abs(Qn), np.abs(Q0), rtol=0, atol=8 * U)
    Qo = hadamard(3)[:, :5] / np.sqrt(8.0)
    Rn2, _, _ = oracle.normalize(oracle.qr(Qo).R)
    np.testing.assert_allclose(Rn2, np.eye(5), rtol=0, atol=16 * U)


def test_identity_block_has_no_reflections():
    A = np.vstack([np.eye(4), np.zeros((3, 4))])
    f = oracle.qr(A)
    assert np.all(f.tau == 0.0)
    assert np.array_equal(f.R, np.eye(4))
    assert np.array_equal(f.V, A)
    assert np.array_equal(f.T, np.zeros((4, 4)))


def test_zero_column_gives_zero_pivot_and_singular_solve():
    A = synth.gaussian(10, 4, 9).copy(order="F")
    A[:, 2] = 0.0
    A[:, 3] = A[:, 0]  # rank deficient, column 3 ends with an exact zero subcolumn? not in general
    f = oracle.qr(A)
    assert f.tau[2] == 0.0 and f.R[2, 2] == 0.0
    with pytest.raises(ZeroDivisionError):
        oracle.lstsq(A, np.ones(10))


# ------------------------------------------------------- exact identities
@pytest.mark.parametrize("m,n,seed", [(6, 3, 1), (9, 8, 2), (20, 8, 3)])
def test_g7_exact_gram_identity(m, n, seed):
    A = synth.int_matrix(m, n, seed)
    f = oracle.qr(A)
    G = A.T @ A  # exact: small integers
    err = np.abs(f.R.T @ f.R - G).max() / np.abs(G).max()
    assert err <= 1e-14


@pytest.mark.parametrize("m,n,seed", [(30, 12, 1), (200, 64, 2)])
def test_t_closed_form(m, n, seed):
    f = oracle.qr(synth.gaussian(m, n, seed))
    V, T = f.V, f.T
    G = V.T @ V
    # T^{-1} + T^{-T} = V^T V
    Ti = np.linalg.inv(T)
    assert np.abs(Ti + Ti.T - G).max() / np.abs(G).max() <= 1e-13
    # T = (striu(V^T V) + diag(V^T V)/2)^{-1}
    Tc = np.linalg.inv(np.triu(G, 1) + np.diag(np.diag(G)) / 2.0)
    assert np.linalg.norm(T - Tc) / np.linalg.norm(T) <= 1e-12
    # Q = I - V T V^T reproduces the reflector product
    Q = np.eye(m) - V @ T @ V.T
    np.testing.assert_allclose(Q[:, :n], oracle.thin_q(f), rtol=0, atol=1e-13)


@pytest.mark.parametrize("m,n,seed", [(1000, 64, 11), (257, 100, 12), (64, 64, 13)])
def test_g1_to_g4_invariants(m, n, seed):
    A = synth.gaussian(m, n, seed)
    f = oracle.qr(A)
    Q = oracle.thin_q(f)
    R = f.R
    nA = np.linalg.norm(A)
    assert np.linalg.norm(A - Q @ R) / nA <= 1e-14                      # G1
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 1e-13                  # G2
    assert np.linalg.norm(R.T @ R - A.T @ A) / nA ** 2 <= 1e-14          # G3
    assert np.all(np.tril(R, -1) == 0.0) and np.all(np.tril(f.T, -1) == 0.0)  # G4
    # apply_q agrees with the explicit product
    C = synth.gaussian(m, 3, seed + 1)
    QtC = oracle.apply_q(f, C, "T")
    QC = oracle.apply_q(f, QtC, "N")
    np.testing.assert_allclose(QC, C, rtol=0, atol=1e-13)
    np.testing.assert_allclose(QtC[:n], Q.T @ C, rtol=0, atol=1e-13)


# ----------------------------------------------------------- least squares
@pytest.mark.parametrize("m,n,cond,seed", [(200, 20, 1e2, 1), (500, 40, 1e6, 2)])
def test_lstsq_consistent_system(m, n, cond, seed):
    A = synth.conditioned(m, n, cond, seed)
    x_true = synth.rng(seed).standard_normal(n)
    b = A @ x_true
    x = oracle.lstsq(A, b)
    assert np.linalg.norm(x - x_true) / np.linalg.norm(x_true) <= 100 * U * cond
    assert oracle.backward_error(A, x, b) <= 1e-14


@pytest.mark.parametrize("m,n,nrhs,seed", [(300, 30, 1, 3), (120, 50, 4, 4)])
def test_lstsq_matches_scipy(m, n, nrhs, seed):
    A = synth.gaussian(m, n, seed)
    x_true, B = synth.ls_rhs(np.asarray(A), seed, noise=1e-2, nrhs=nrhs)
    x = oracle.lstsq(A, B)
    xs = sla.lstsq(A, B)[0]
    np.testing.assert_allclose(x, xs, rtol=0, atol=1e-12)
    for c in range(nrhs):
        assert oracle.backward_error(A, x[:, c], B[:, c]) <= 1e-15


# ------------------------------------------------------ backward error beta
def read_beta_cases(path):
    cases = []
    with open(path) as f:
        for ln in f:
            if ln.startswith("case"):
                _, x0, x1, num2, r2, x2 = ln.split()
                cases.append((np.array([float(x0), float(x1)]), int(num2), int(r2), int(x2)))
    return cases


def test_backward_error_golden_3x2():
    """beta(x) = ||A^T r|| / (||A||_F (||A||_F ||x|| + ||r||)) at hand-derived
    points of the 3 x 2 example (exact integers in the fixture), and zero at
    the least-squares solution although r != 0."""
    g = read_golden(GOLDEN)
    A, b = g["A"], g["b"][:, 0]
    nA = np.sqrt(66.0)
    for x, num2, r2, x2 in read_beta_cases(GOLDEN_BETA):
        want = np.sqrt(num2) / (nA * (nA * np.sqrt(x2) + np.sqrt(r2)))
        got = oracle.backward_error(A, x, b)
        assert abs(got - want) <= 8 * U * want, (x, got, want)
    xls = g["x"][:, 0]
    assert np.linalg.norm(b - A @ xls) > 1.0
    assert oracle.backward_error(A, xls, b) <= 1e-16


def test_backward_error_properties():
    """Invariances of the measure (to 1e-8: A^T r cancels to about 1e-6 of
    ||A|| ||r|| here, so rounding in r shows near 1e-10): unchanged when (A, b)
    are scaled together,
    when A's rows and b are permuted alike, and when A's columns are permuted
    with x; a perturbation dx of the least-squares solution gives beta within
    [||A^T A dx|| / den, same] computed from its own pieces."""
    A = synth.gaussian(40, 6, 21)
    x_true, B = synth.ls_rhs(np.asarray(A), 22, noise=1e-1)
    b = B[:, 0]
    x = sla.lstsq(A, b)[0]
    dx = 1e-6 * synth.rng(23).standard_normal(6)
    beta = oracle.backward_error(A, x + dx, b)
    assert beta > 1e-9
    assert abs(oracle.backward_error(3.0 * A, x + dx, 3.0 * b) - beta) <= 1e-8 * beta
    p = synth.rng(24).permutation(40)
    assert abs(oracle.backward_error(A[p], x + dx, b[p]) - beta) <= 1e-8 * beta
    q = synth.rng(25).permutation(6)
    assert abs(oracle.backward_error(A[:, q], (x + dx)[q], b) - beta) <= 1e-8 * beta
    # At x + dx, A^T r = A^T (r_LS - A dx) = -A^T A dx (A^T r_LS = 0).
    r = b - A @ (x + dx)
    nA = np.sqrt(np.sum(A * A))
    want = np.linalg.norm(A.T @ A @ dx) / (nA * (nA * np.linalg.norm(x + dx) + np.linalg.norm(r)))
    assert abs(beta - want) <= 1e-6 * want
