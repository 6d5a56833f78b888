"""Serving loop: admission by HBM budget, continuous batching over captured
graph replays, kept factorisations for further right-hand sides.

Every served result is compared bitwise with the same problem solved alone by
an eager qr_lstsq_batched call (a request's arithmetic does not depend on its
batch), and sampled results against the oracle.
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


def shapes(k, seed, m_hi=4096, n_hi=256):
    r = synth.rng(seed)
    out = []
    while len(out) < k:
        m = int(r.integers(64, m_hi + 1))
        n = int(r.integers(8, n_hi + 1))
        if m >= n:
            out.append((m, n, int(r.integers(1, 5))))
    return out


def problems(sh, seed):
    return [(np.asfortranarray(synth.gaussian(m, n, seed + 2 * i)),
             np.asfortranarray(synth.gaussian(m, k, seed + 2 * i + 1))) for i, (m, n, k) in enumerate(sh)]


def eager(m_, h, A, B):
    """The same problem alone, through qr_lstsq_batched."""
    Ad, Bd = m_.to_colmajor(A), m_.to_colmajor(B)
    st, stat = h.lstsq_batched([Ad], [Bd])
    torch.cuda.synchronize()
    return stat[0], Bd.cpu().numpy()[: A.shape[1]]


def drain(srv, ids, done=None, limit_s=120.0):
    """Poll until every id in `ids` is reported (earlier reports in `done`)."""
    import time
    done = {} if done is None else done
    t0 = time.monotonic()
    while not all(i in done for i in ids):
        for d in srv.poll(wait=True):
            done[d["id"]] = d
        assert time.monotonic() - t0 < limit_s, "server did not finish in time"
    return done


def test_server_continuous_batching_matches_eager(miqr):
    m_, h = miqr
    sh = shapes(60, 31)
    probs = problems(sh, 7000)
    X = [np.zeros((n, k), order="F") for (m, n, k) in sh]
    # Small batches so that the captured graph is replayed many times, with
    # eager work (the reference solves) between the replays.
    srv = m_.Server(h, hbm_budget=256 << 20, max_batch=8)
    ids = []
    refs = {}
    done = {}
    for i, ((A, B), x) in enumerate(zip(probs, X)):
        ids.append(srv.submit(A, B, x))
        if i % 5 == 4:
            for d in srv.poll():
                done[d["id"]] = d
            j = i - 2
            refs[j] = eager(m_, h, *probs[j])
    done = drain(srv, ids, done)
    srv.close()
    sizes = [d["batch_size"] for d in done.values()]
    assert max(sizes) <= 8 and len(set(d["start_s"] for d in done.values())) >= 8
    for i, rid in enumerate(ids):
        d = done[rid]
        assert d["status"] == 0
        assert d["submit_s"] <= d["start_s"] <= d["end_s"]
        st, xe = refs[i] if i in refs else eager(m_, h, *probs[i])
        assert st == 0
        assert np.array_equal(X[i], xe), i
    for i in (0, 17, 59):
        A, B = probs[i]
        xo = oracle.lstsq(A, B)
        kappa = np.linalg.cond(A)
        for c in range(B.shape[1]):
            r = B[:, c] - A @ xo[:, c]
            bound = 100 * U * (kappa + kappa ** 2 * np.linalg.norm(r) /
                               (np.linalg.norm(A, 2) * np.linalg.norm(xo[:, c])))
            assert np.linalg.norm(X[i][:, c] - xo[:, c]) / np.linalg.norm(xo[:, c]) <= bound


def test_server_admission_respects_hbm_budget(miqr):
    m_, h = miqr
    budget = 6 << 20
    sh = [(2048, 128, 2)] * 12  # about 2.1 MB of device memory each
    probs = problems(sh, 8100)
    X = [np.zeros((n, k), order="F") for (m, n, k) in sh]
    srv = m_.Server(h, hbm_budget=budget, max_batch=64)
    ids = [srv.submit(A, B, x) for (A, B), x in zip(probs, X)]
    seen_pending = False
    done = {}
    import time
    t0 = time.monotonic()
    while len(done) < len(ids):
        assert time.monotonic() - t0 < 120.0, "server did not finish in time"
        st = srv.stats()
        assert st["hbm_used"] <= budget
        seen_pending |= st["pending"] > 0 and st["running"] + st["admitted"] > 0
        for d in srv.poll(wait=False):
            done[d["id"]] = d
    srv.close()
    assert seen_pending
    for i in range(len(sh)):
        st, xe = eager(m_, h, *probs[i])
        assert np.array_equal(X[i], xe)


def test_server_kept_factors_serve_new_rhs(miqr):
    m_, h = miqr
    sh = [(1500, 100, 1), (700, 200, 2), (4096, 256, 1)]
    probs = problems(sh, 9100)
    X = [np.zeros((n, k), order="F") for (m, n, k) in sh]
    srv = m_.Server(h, keep_factors=True, max_batch=16)
    ids = [srv.submit(A, B, x) for (A, B), x in zip(probs, X)]
    drain(srv, ids)
    for i in range(3):
        st, xe = eager(m_, h, *probs[i])
        assert np.array_equal(X[i], xe)
    # New right-hand sides against the kept factorisations.
    B2 = [np.asfortranarray(synth.gaussian(m, 3, 9900 + i)) for i, (m, n, k) in enumerate(sh)]
    X2 = [np.zeros((n, 3), order="F") for (m, n, k) in sh]
    ids2 = [srv.resolve(ids[i], B2[i], X2[i]) for i in range(3)]
    with pytest.raises(m_.MiqrError) as e:
        srv.release(ids[0])  # solves against it still queued
    assert e.value.status == m_.EBUSY
    done = drain(srv, ids2)
    assert all(d["status"] == 0 for d in done.values())
    for i in range(3):
        A = probs[i][0]
        xo = oracle.lstsq(A, B2[i])
        for c in range(3):
            assert oracle.backward_error(A, X2[i][:, c], B2[i][:, c]) <= 1e-13
            kappa = np.linalg.cond(A)
            r = B2[i][:, c] - A @ xo[:, c]
            bound = 100 * U * (kappa + kappa ** 2 * np.linalg.norm(r) /
                               (np.linalg.norm(A, 2) * np.linalg.norm(xo[:, c])))
            assert np.linalg.norm(X2[i][:, c] - xo[:, c]) / np.linalg.norm(xo[:, c]) <= bound
    for rid in ids:
        srv.release(rid)
    assert srv.stats()["hbm_used"] == 0
    srv.close()


def test_server_errors_and_singular(miqr):
    m_, h = miqr
    srv = m_.Server(h, hbm_budget=1 << 20, max_pending=2, max_batch=4)
    big = np.zeros((4096, 64), order="F")
    bb = np.zeros((4096, 1), order="F")
    xb = np.zeros((64, 1), order="F")
    with pytest.raises(m_.MiqrError) as e:
        srv.submit(big, bb, xb)  # 2 MB > 1 MB budget
    assert e.value.status == m_.EINVAL
    A, B = problems([(300, 20, 1)], 9500)[0]
    A = A.copy(order="F")
    A[:, 5] = 0.0
    x = np.zeros((20, 1), order="F")
    r1 = srv.submit(A, B, x)
    A2, B2 = problems([(200, 10, 1)], 9600)[0]
    x2 = np.zeros((10, 1), order="F")
    r2 = srv.submit(A2, B2, x2)
    x3 = np.zeros((10, 1), order="F")
    with pytest.raises(m_.MiqrError) as e:
        srv.submit(A2, B2, x3)  # third waiting request: back-pressure
    assert e.value.status == m_.EBUSY
    done = drain(srv, [r1, r2])
    assert done[r1]["status"] == 6 and done[r2]["status"] == 0
    with pytest.raises(m_.MiqrError):
        srv.resolve(r2, B2, x3)  # not kept
    srv.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_server_mixed_precision_matches_batched(miqr, prec):
    """A mixed-precision server: every result bitwise equal to the same problem
    solved alone by the mixed batched call, and within the FP64 backward-error
    gate; a request too ill-conditioned for the products is solved again in
    FP64 in a later batch, bitwise equal to the FP64 call."""
    m_, h = miqr
    p = {"fp32": m_.MIXED_FP32, "bf16": m_.MIXED_BF16}[prec]
    sh = shapes(24, 57)
    probs = problems(sh, 7600)
    A1 = np.asfortranarray(synth.conditioned(1200, 100, 1e12, 7701))
    _, B1 = synth.ls_rhs(A1, 7702, noise=1e-6, nrhs=2)
    probs.append((A1, np.asfortranarray(B1)))
    X = [np.zeros((A.shape[1], B.shape[1]), order="F") for A, B in probs]
    srv = m_.Server(h, hbm_budget=256 << 20, max_batch=8, precision=p)
    ids = [srv.submit(A, B, x) for (A, B), x in zip(probs, X)]
    done = drain(srv, ids)
    srv.close()
    for i, rid in enumerate(ids):
        assert done[rid]["status"] == 0
        A, B = probs[i]
        Ad, Bd = m_.to_colmajor(A), m_.to_colmajor(B)
        last = i == len(probs) - 1
        st, stat, its = h.lstsq_batched([Ad], [Bd], h.opts(precision=p), want_iters=True)
        torch.cuda.synchronize()
        assert stat == [0] and (its[0] == -1) == last
        assert np.array_equal(X[i], Bd.cpu().numpy()[: A.shape[1]]), i
        for c in range(B.shape[1]):
            assert oracle.backward_error(A, X[i][:, c], B[:, c]) <= 1e-13
    with pytest.raises(m_.MiqrError) as e:
        m_.Server(h, keep_factors=True, precision=p)
    assert e.value.status == m_.ENOTSUP
