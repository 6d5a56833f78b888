"""qr_factor_noalloc (static device workspace, no allocation) against
qr_factor on the same inputs, through the C ABI: two calls in a row, the
second on a smaller matrix, in both T layouts.

The two entry points run the same factorisation; the allocation-free one has
no look-ahead stream and fewer split-K partials, so the summation order of some
products differs.  Gates: the G5 tolerances between the two results (R~
1e-13, V and T 1e-12 in Frobenius norm), and both against the oracle with the
elementwise gates of the parity tests; exact zeros below the diagonals.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.test_gpu_parity import check_against_oracle, check_elementwise, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def miqr():
    import paper_1805_05278_amd as m
    h = m.Handle(0)
    yield m, h
    h.close()


def both(m_, h, A, opts_kw):
    mm, nn = A.shape
    o = h.opts(**opts_kw)
    tr = h.t_rows(mm, nn, o)
    outs = []
    for fn in (h.factor, h.factor_noalloc):
        Ad = m_.to_colmajor(A)
        Td = m_.colmajor(tr, nn)
        Td.fill_(3.0)
        print("%s %dx%d %s" % (fn.__name__, mm, nn, opts_kw), flush=True)
        fn(Ad, Td, o)
        torch.cuda.synchronize()
        vr = Ad.cpu().numpy()
        outs.append({"V": np.tril(vr, -1) + np.eye(mm, nn), "R": np.triu(vr[:nn]),
                     "T": Td.cpu().numpy()})
    return outs


@pytest.mark.parametrize("layout", ["full", "blocked"])
def test_noalloc_matches_qr_factor_twice(miqr, layout):
    m_, h = miqr
    kw = {} if layout == "full" else dict(t_layout=m_.T_BLOCKED, nb=128)
    for (mm, nn, seed) in [(6000, 300, 701), (2500, 150, 702)]:
        A = synth.gaussian(mm, nn, seed)
        g, z = both(m_, h, A, kw)
        assert rel(oracle.normalize(z["R"])[0], oracle.normalize(g["R"])[0]) <= 1e-13
        assert rel(z["V"], g["V"]) <= 1e-12
        assert rel(z["T"], g["T"]) <= 1e-12
        f = oracle.qr(A)
        if layout == "full":
            check_against_oracle(A, z, f=f)
        else:
            check_elementwise(A, f, z["R"], z["V"])
            for j in range(0, nn, 128):
                w = min(128, nn - j)
                assert rel(z["T"][:w, j:j + w], f.T[j:j + w, j:j + w]) <= 1e-12
                assert np.all(np.tril(z["T"][:w, j:j + w], -1) == 0.0)


def test_noalloc_rejects_oversized(miqr):
    m_, h = miqr
    A = m_.colmajor(2_000_000, 64)
    T = m_.colmajor(64, 64)
    with pytest.raises(m_.MiqrError) as ei:
        h.factor_noalloc(A, T)
    assert ei.value.status == m_.EINVAL
