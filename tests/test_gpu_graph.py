"""qr_factor through captured launch graphs (miqr_graphs_enable).

A replay runs the captured kernels in the captured order, so every replay must
equal the eager call bitwise.  Replays are interleaved with eager work and
synchronisations and each one is checked, because graph replays after the
first have misbehaved on this hardware where a graph held memset nodes (the
factorisation records none; the test covers the whole sequence).  One case is
also checked against the oracle directly.
"""
import numpy as np
import pytest

import synth
from tests.test_gpu_parity import check_against_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def miqr():
    import paper_1805_05278_amd as m
    h = m.Handle(0)
    yield m, h
    h.close()


CASES = [
    # one TSQR panel and the thin Q
    dict(m=1024, n=64, with_q=True),
    # Alg. 2 recursion over TSQR base cases, full T
    dict(m=5000, n=150),
    # 256-row leaf chains of three blocks, five-way tree
    dict(m=20000, n=64, leaf_rows=256, chain=3, arity=5),
    # right-looking top level with look-ahead on the second stream
    dict(m=3000, n=600, blocked=True, nb=128),
]


def _opts(m_, h, c, Q=None):
    kw = {}
    for k in ("leaf_rows", "chain", "arity"):
        if k in c:
            kw[k] = c[k]
    if c.get("blocked"):
        kw.update(t_layout=m_.T_BLOCKED, nb=c["nb"])
    if Q is not None:
        kw["Q"] = Q
    return h.opts(**kw)


def _run(m_, h, c, A0, Ad, Td, Qd):
    Ad.copy_(A0)
    Td.fill_(7.0)  # every entry the call writes must be rewritten
    if Qd is not None:
        Qd.fill_(7.0)
    h.factor(Ad, Td, _opts(m_, h, c, Qd))


def _alloc(m_, h, c):
    mm, nn = c["m"], c["n"]
    tr = h.t_rows(mm, nn, _opts(m_, h, c))
    return (m_.colmajor(mm, nn), m_.colmajor(tr, nn),
            m_.colmajor(mm, nn) if c.get("with_q") else None)


@pytest.mark.parametrize("side_stream", [False, True])
@pytest.mark.parametrize("c", CASES, ids=lambda c: "%dx%d" % (c["m"], c["n"]))
def test_graph_replays_equal_eager(miqr, c, side_stream):
    m_, h = miqr
    A0 = synth.gaussian_device(c["m"], c["n"], 7100 + c["n"])
    h.graphs(False)
    Ae, Te, Qe = _alloc(m_, h, c)
    _run(m_, h, c, A0, Ae, Te, Qe)
    torch.cuda.synchronize()
    ref = [x.cpu().numpy() for x in (Ae, Te, Qe) if x is not None]

    h.graphs(True)
    assert h.graph_count() == 0
    Ag, Tg, Qg = _alloc(m_, h, c)
    stream = torch.cuda.Stream() if side_stream else torch.cuda.current_stream()
    noise = torch.randn(512, 512, dtype=torch.float64, device="cuda")
    for rep in range(4):
        with torch.cuda.stream(stream):
            _run(m_, h, c, A0, Ag, Tg, Qg)
        stream.synchronize()
        got = [x.cpu().numpy() for x in (Ag, Tg, Qg) if x is not None]
        for g, r in zip(got, ref):
            assert np.array_equal(g, r), ("replay", rep)
        assert h.graph_count() == 1
        # eager work and a synchronisation between replays
        noise = noise @ noise.t() / 512.0
        torch.cuda.synchronize()
    h.graphs(False)
    assert h.graph_count() == 0


def test_graph_keys(miqr):
    """A new buffer or shape is captured anew; the same ones replay."""
    m_, h = miqr
    c = CASES[1]
    A0 = synth.gaussian_device(c["m"], c["n"], 7200)
    h.graphs(True)
    Ad, Td, _ = _alloc(m_, h, c)
    _run(m_, h, c, A0, Ad, Td, None)
    _run(m_, h, c, A0, Ad, Td, None)
    assert h.graph_count() == 1
    A2, T2, _ = _alloc(m_, h, c)
    _run(m_, h, c, A0, A2, T2, None)
    assert h.graph_count() == 2
    torch.cuda.synchronize()
    assert np.array_equal(Ad.cpu().numpy(), A2.cpu().numpy())
    assert np.array_equal(Td.cpu().numpy(), T2.cpu().numpy())
    B0 = synth.gaussian(1500, 70, 7201)
    g = {}
    Bd = m_.to_colmajor(B0)
    Tb = m_.colmajor(70, 70)
    h.factor(Bd, Tb)
    assert h.graph_count() == 3
    torch.cuda.synchronize()
    vr = Bd.cpu().numpy()
    g = {"vr": vr, "V": np.tril(vr, -1) + np.eye(1500, 70), "R": np.triu(vr[:70]),
         "T": Tb.cpu().numpy()}
    check_against_oracle(B0, g)
    h.graphs(False)
    assert h.graph_count() == 0
