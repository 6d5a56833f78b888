"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances (u = 2^-53), per quantity, from the project's gates:
  R (after normalising diag >= 0): ||dR|| / ||R|| <= 1e-13             (G5)
  V, T (same reflector sign rule on both sides): <= 1e-12             (G5)
  thin Q: ||dQ|| / ||Q|| <= 1e-12; ||A - QR|| / ||A|| <= 1e-14 (n <= 256)
  least squares: backward error beta(x) <= 1e-13                      (G8)
  tuning invariance: any (b, leaf_rows, chain, arity) within 1e-13   (G10)
Exact zeros (R and T strictly lower) are checked bitwise (G4).

Beside the Frobenius gates every parity check also gates elementwise, scaled
by column norms, so that an error confined to a few rows or one block cannot
hide in a norm over the whole matrix: the G5 tolerances applied per column,
  |dR~_ij| <= 1e-13 ||a_j||,  |dV_ij| <= 1e-12 ||v_j||,  |dT_ij| <= 1e-12 ||t_j||
(LAPACK's recursive dgeqrt, a different summation order, sits within 60 u,
2 u and 7 u of the oracle on these shapes; the GPU's largest measured T
deviation, 2.7e-13, is in the square tail of a 700 x 700 matrix, where the
last panels are nearly square).
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


EL_R, EL_VT = 1e-13, 1e-12


def colwise(a, b, scale):
    """max_ij |a_ij - b_ij| / scale_j (scale_j = 1 where it is zero)."""
    sc = np.where(scale > 0, scale, 1.0)
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)) / sc[None, :]))


def check_elementwise(A, f, R, V=None, T=None, el_r=EL_R, el_vt=EL_VT):
    """Column-scaled elementwise gates of R~ (against the columns of A), V and
    T (against their own columns); returns the measured values."""
    out = {"R": colwise(oracle.normalize(R)[0], oracle.normalize(f.R)[0],
                        np.linalg.norm(A, axis=0))}
    if V is not None:
        out["V"] = colwise(V, f.V, np.linalg.norm(f.V, axis=0))
    if T is not None:
        out["T"] = colwise(T, f.T, np.linalg.norm(f.T, axis=0))
    assert out["R"] <= el_r, out
    assert out.get("V", 0.0) <= el_vt and out.get("T", 0.0) <= el_vt, out
    return out


def check_against_oracle(A, g, tol_r=1e-13, tol_vt=1e-12, f=None):
    f = f if f is not None else oracle.qr(A)
    assert rel(oracle.normalize(g["R"])[0], oracle.normalize(f.R)[0]) <= tol_r
    assert rel(g["V"], f.V) <= tol_vt
    assert rel(g["T"], f.T) <= tol_vt
    assert np.all(np.tril(g["T"], -1) == 0.0)
    assert np.all(np.tril(g["R"], -1) == 0.0)
    check_elementwise(A, f, g["R"], g["V"], g["T"])
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


# Widths whose left recursion child is wider than the root's split product:
# n in [2b + 2, 2.5b) makes the left child 2b wide, which splits into b x b
# (more than the root's n1 x n2), so the EG temporaries must be sized from
# every node, not the root.
@pytest.mark.parametrize("m,n,b", [(900, 130, 64), (1200, 135, 64), (700, 159, 64),
                                   (500, 66, 32), (800, 70, 32)])
def test_eg_widths_with_wide_left_child(miqr, m, n, b):
    m_, h = miqr
    A = synth.gaussian(m, n, 250 + n + b)
    g = gpu_factor(m_, h, A, b=b)
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
    """G10: every tuning gives the oracle's R~, V and T within 1e-13."""
    m_, h = miqr
    A = synth.gaussian(5000, 150, 77)
    g = gpu_factor(m_, h, A, **tune)
    check_against_oracle(A, g, tol_r=1e-13, tol_vt=1e-13)


# Leaf chains longer than one block at 256-row blocks (the stacked-block leaf
# launch and its Q-emitting downsweep), with binary and five-way trees.
@pytest.mark.parametrize("m,n", [(20000, 64), (70000, 40)])
@pytest.mark.parametrize("chain,arity", [(2, 2), (3, 5), (8, 5), (8, 2)])
@pytest.mark.parametrize("with_q", [False, True])
def test_chained_256_row_leaves(miqr, m, n, chain, arity, with_q):
    m_, h = miqr
    A = synth.gaussian(m, n, 400 + n + chain + arity)
    g = gpu_factor(m_, h, A, with_q=with_q, leaf_rows=256, chain=chain, arity=arity)
    f = check_against_oracle(A, g, tol_r=1e-13, tol_vt=1e-13)
    if with_q:
        Q = oracle.thin_q(f)
        assert rel(g["Q"], Q) <= 1e-12
        assert colwise(g["Q"], Q, np.ones(n)) <= 1e-13


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
    betas = [oracle.backward_error(A, x[:, c], B[:, c]) for c in range(nrhs)]
    assert max(betas) <= 1e-13
    assert rel(x, xo) <= 1e-10
    # The library's reported beta is the worst right-hand side's.  Here beta
    # sits at rounding level, where the residual's own rounding decides its
    # value, so the two agree to an absolute 1e-15 rather than relatively.
    assert info.backward_error <= 1e-13
    assert abs(info.backward_error - max(betas)) <= 1e-6 * max(betas) + 1e-15


def test_backward_error_matches_oracle(miqr):
    """The library's beta against the oracle's at points away from the
    solution (beta 1e-11 .. 1e-2): 1e-9 relative, plus 1e-15 absolute for the
    rounding of r = b - A x, which both sides compute in their own order (the
    perturbation of A^T r it causes is about u ||A|| (||b|| + ||A|| ||x||),
    i.e. a few u after beta's normalisation)."""
    m_, h = miqr
    A = synth.gaussian(3000, 40, 61)
    _, B = synth.ls_rhs(A, 62, noise=1e-3, nrhs=1)
    xo = oracle.lstsq(A, B)[:, 0]
    d = synth.rng(63).standard_normal(40)
    X = np.stack([xo + s * d for s in (1e-9, 1e-6, 1e-3, 1.0)], axis=1)
    Bk = np.repeat(B, 4, axis=1)
    got = h.backward_error(m_.to_colmajor(A), m_.to_colmajor(Bk), m_.to_colmajor(X))
    for c in range(4):
        want = oracle.backward_error(A, X[:, c], Bk[:, c])
        assert want > 1e-12
        assert abs(got[c] - want) <= 1e-9 * want + 1e-15, (c, got[c], want)


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


# ---------------------------------------------------------------- BLOCKED T
def gpu_factor_blocked(m_, h, A, nb, with_q=False, normalize=False, lookahead=True, **tune):
    mm, nn = A.shape
    o = h.opts(t_layout=m_.T_BLOCKED, nb=nb, lookahead=lookahead, **tune)
    tr = h.t_rows(mm, nn, o)
    assert tr == min(nb, nn)
    Ad = m_.to_colmajor(A)
    Td = m_.colmajor(tr, nn)
    Td.fill_(7.0)  # every entry must be written
    Qd = m_.colmajor(mm, nn) if with_q else None
    sd = torch.empty(nn, dtype=torch.float64, device="cuda") if normalize else None
    o = h.opts(t_layout=m_.T_BLOCKED, nb=nb, lookahead=lookahead, Q=Qd, normalize=normalize,
               sign_out=sd, **tune)
    h.factor(Ad, Td, o)
    torch.cuda.synchronize()
    vr = Ad.cpu().numpy()
    out = {"vr": vr, "V": np.tril(vr, -1) + np.eye(mm, nn), "R": np.triu(vr[:nn]),
           "Tb": Td.cpu().numpy(), "Ad": Ad, "Td": Td}
    if with_q:
        out["Q"] = Qd.cpu().numpy()
    if normalize:
        out["d"] = sd.cpu().numpy()
    return out


def check_blocked(A, g, nb, f=None):
    """V and R~ as the oracle's; panel k's T equals the diagonal block of the
    oracle's full T (the kernel of reflectors k nb .. k nb + w - 1 alone),
    zeros below it and below the panel's width."""
    f = f if f is not None else oracle.qr(A)
    n = A.shape[1]
    assert rel(oracle.normalize(g["R"])[0], oracle.normalize(f.R)[0]) <= 1e-13
    assert rel(g["V"], f.V) <= 1e-12
    Tb = g["Tb"]
    for j in range(0, n, nb):
        w = min(nb, n - j)
        blk = Tb[:w, j:j + w]
        want = f.T[j:j + w, j:j + w]
        assert rel(blk, want) <= 1e-12, j
        assert colwise(blk, want, np.linalg.norm(want, axis=0)) <= EL_VT, j
        assert np.all(np.tril(blk, -1) == 0.0)
        assert np.all(Tb[w:, j:j + w] == 0.0)
    check_elementwise(A, f, g["R"], g["V"])
    return f


@pytest.mark.parametrize("m,n,nb", [(3000, 700, 256), (5000, 1000, 256), (4096, 513, 200),
                                    (1500, 300, 128), (2000, 2000, 512), (700, 700, 256),
                                    (20000, 320, 64), (1000, 65, 64)])
@pytest.mark.parametrize("lookahead", [True, False])
def test_blocked_matches_oracle(miqr, m, n, nb, lookahead):
    m_, h = miqr
    A = synth.gaussian(m, n, 500 + n + nb)
    g = gpu_factor_blocked(m_, h, A, nb, lookahead=lookahead)
    check_blocked(A, g, nb)


def test_blocked_lookahead_column_chunks(miqr):
    """More than 3072 trailing columns: the look-ahead stream updates them in
    column chunks (early panels here take two)."""
    m_, h = miqr
    A = synth.gaussian(3400, 3300, 611)
    g = gpu_factor_blocked(m_, h, A, 64, lookahead=True)
    check_blocked(A, g, 64)


def test_blocked_lookahead_equals_one_stream_8192(miqr):
    """8192^2 with nb = 128 (up to three update chunks per panel): the
    look-ahead factors equal the one-stream ones to rounding (the one-stream
    path is checked against the oracle above).  A skipped or doubled chunk
    would change whole columns by O(1)."""
    m_, h = miqr
    A = synth.gaussian(8192, 8192, 612)
    ga = gpu_factor_blocked(m_, h, A, 128, lookahead=True)
    g1 = gpu_factor_blocked(m_, h, A, 128, lookahead=False)
    # normwise, at the size where kappa(A) ~ 1e4 amplifies rounding in V and T
    assert rel(ga["R"], g1["R"]) <= 1e-11
    assert rel(ga["V"], g1["V"]) <= 1e-10
    assert rel(ga["Tb"], g1["Tb"]) <= 1e-10


@pytest.mark.parametrize("b,bstar", [(128, 64), (128, 32), (32, 32)])
def test_blocked_with_thresholds(miqr, b, bstar):
    m_, h = miqr
    A = synth.gaussian(6000, 900, 601 + b + bstar)
    g = gpu_factor_blocked(m_, h, A, 384, b=b, bstar=bstar)
    check_blocked(A, g, 384)


def test_blocked_thin_q_normalised(miqr):
    m_, h = miqr
    A = synth.gaussian(4000, 600, 611)
    g = gpu_factor_blocked(m_, h, A, 256, with_q=True, normalize=True)
    f = oracle.qr(A)
    Rn, Qn, d = oracle.normalize(f.R, oracle.thin_q(f))
    assert np.all(np.diag(g["R"]) >= 0)
    assert np.array_equal(g["d"], d)
    assert rel(g["R"], Rn) <= 1e-13
    assert rel(g["Q"], Qn) <= 1e-12
    assert colwise(g["Q"], Qn, np.ones(600)) <= 1e-13
    assert np.linalg.norm(A - g["Q"] @ g["R"]) / np.linalg.norm(A) <= 1e-14


@pytest.mark.parametrize("trans", ["T", "N"])
def test_blocked_apply_q(miqr, trans):
    m_, h = miqr
    A = synth.gaussian(2500, 500, 621)
    C = synth.gaussian(2500, 5, 622)
    g = gpu_factor_blocked(m_, h, A, 192)
    Cd = m_.to_colmajor(C)
    h.apply_q_blocked(trans, g["Ad"], g["Td"], 192, Cd)
    ref = oracle.apply_q(oracle.qr(A), C, trans)
    assert rel(Cd.cpu().numpy(), ref) <= 1e-13


@pytest.mark.parametrize("layout", ["full", "blocked", "auto"])
@pytest.mark.parametrize("m,n,nrhs", [(6000, 700, 2), (3000, 200, 1)])
def test_lstsq_layouts(miqr, layout, m, n, nrhs):
    m_, h = miqr
    A = synth.conditioned(m, n, 1e3, 631 + n)
    _, B = synth.ls_rhs(A, 632 + n, noise=1e-6, nrhs=nrhs)
    o = {"full": h.opts(t_layout=m_.T_FULL, b=64), "blocked": h.opts(t_layout=m_.T_BLOCKED, nb=256),
         "auto": None}[layout]
    Ad, Bd = m_.to_colmajor(A), m_.to_colmajor(B)
    st, info = h.lstsq(Ad, Bd, o)
    assert st == m_.OK
    x = Bd.cpu().numpy()[:n]
    xo = oracle.lstsq(A, B)
    betas = [oracle.backward_error(A, x[:, c], B[:, c]) for c in range(nrhs)]
    assert max(betas) <= 1e-13
    assert rel(x, xo) <= 1e-10
    assert abs(info.backward_error - max(betas)) <= 1e-6 * max(betas) + 1e-15


@pytest.mark.parametrize("m,n", [(5000, 150), (20000, 640), (3000, 3000)])
def test_autotuned_factor_matches_oracle(miqr, m, n):
    """qr_factor with no options runs the cost model's tuning; the same
    tuning, given explicitly, gives the same bits, and both match the oracle."""
    m_, h = miqr
    A = synth.gaussian(m, n, 641 + n)
    p = h.plan(m, n)
    t = p["tuning"]
    g = gpu_factor(m_, h, A)
    check_against_oracle(A, g)
    g2 = gpu_factor(m_, h, A, b=t["b"], bstar=t["bstar"])
    assert np.array_equal(g2["vr"], g["vr"]) and np.array_equal(g2["T"], g["T"])
