"""Host-side plan of the library (no GPU): the Alg. 2 recursion it will run,
the workspace regions it sizes for it, the T layouts and the tuning the cost
model picks.  Read through qr_plan, which needs no device.

* Every recursion node's M1..M4 temporaries (n1 x n2 doubles) fit the EG
  regions, whatever the width (the widths whose left child is wider than the
  root's split included), and every base case is a TSQR panel of width <= b*.
* The nodes of a top-level panel tile its columns exactly (children widths add
  up, the left child keeps the rows, the right child starts n1 rows lower).
* BLOCKED plans cut the columns into panels of nb, and T has nb rows.
* The tuning keeps what the caller fixed, is deterministic, and rejects
  options out of range.
"""
import ctypes
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def m_():
    import paper_1805_05278_amd as m
    if not os.path.exists(m.LIB_PATH):
        pytest.skip("libmiqr.so not built")
    return m


def walk(nodes, c0, rows, width, bstar, wa, out):
    """Check the subtree rooted at (c0, rows, width) in pre-order; return the
    index past it."""
    node = nodes[out["i"]]
    out["i"] += 1
    assert node[:3] == [c0, rows, width], (node, c0, rows, width)
    n1 = node[3]
    if n1 == 0:
        assert width <= bstar
        out["panels"].append((c0, rows, width))
        return
    n2 = width - n1
    assert 0 < n1 < width
    assert n1 * n2 <= wa, (node, wa)
    walk(nodes, c0, rows, n1, bstar, wa, out)
    walk(nodes, c0 + n1, rows - n1, n2, bstar, wa, out)


def check_plan(p, m, n):
    t = p["tuning"]
    nb = t["nb"] if t["t_layout"] == 1 else n
    out = {"i": 0, "panels": []}
    for j in range(0, n, nb):
        walk(p["nodes"], j, m - j, min(nb, n - j), t["bstar"], p["layout"]["wa"], out)
    assert out["i"] == len(p["nodes"])
    # TSQR panels cover the columns in order, each at its diagonal row.
    assert [x[0] for x in out["panels"]] == sorted(x[0] for x in out["panels"])
    assert sum(x[2] for x in out["panels"]) == n
    assert [tuple(x[:3]) for x in p["panels"]] == out["panels"]
    for pan in p["panels"]:
        c0, rows, w, leaf, chain, arity, levels = pan
        assert leaf in (128, 256) and chain >= 1 and arity >= 2 and levels >= 0
        assert (arity - 1) * w <= 256  # stacked children fit a tree node
    L = p["layout"]
    assert all(L[k] >= 0 for k in L)
    assert L["total"] >= sum(L[k] for k in L if k != "total")


@pytest.mark.parametrize("b", [16, 32, 48, 64])
def test_every_node_fits_its_workspace(m_, b):
    """All widths 1..400 and b in {16, 32, 48, 64}: in particular n in
    [2b + 2, 2.5b), where the left child (2b wide) splits into b x b, more
    than the root's n1 x n2."""
    o = m_.Handle.opts(b=b)
    for n in range(1, 401):
        p = m_.Handle.plan(max(n, 300), n, o)
        assert p["tuning"]["b"] == min(b, n) and p["tuning"]["bstar"] == min(b, n)
        check_plan(p, max(n, 300), n)


@pytest.mark.parametrize("n,b", [(130, 64), (135, 64), (159, 64), (66, 32), (70, 32)])
def test_wide_left_child_sizes(m_, n, b):
    p = m_.Handle.plan(1000, n, m_.Handle.opts(b=b))
    worst = max(nd[3] * (nd[2] - nd[3]) for nd in p["nodes"] if nd[3])
    root = p["nodes"][0]
    assert worst > root[3] * (root[2] - root[3])  # the root is not the largest
    assert p["layout"]["wa"] >= worst


@pytest.mark.parametrize("m,n,nb", [(5000, 1000, 256), (3000, 3000, 512), (900, 700, 128),
                                    (4096, 513, 200)])
def test_blocked_plan(m_, m, n, nb):
    o = m_.Handle.opts(t_layout=m_.T_BLOCKED, nb=nb, b=64)
    p = m_.Handle.plan(m, n, o)
    assert p["tuning"]["t_layout"] == 1 and p["tuning"]["nb"] == nb
    check_plan(p, m, n)
    assert m_.Handle.t_rows(m, n, o) == nb
    assert m_.Handle.t_rows(m, n, m_.Handle.opts(b=64)) == n
    # The look-ahead stream's temporaries hold one panel against every
    # column after the first panel.
    assert p["layout"]["ua1"] >= nb * (n - nb)
    assert p["layout"]["u1"] >= nb * nb


def test_b_above_64_uses_64_wide_panels(m_):
    """b = 128 (the paper's Alg. 2 threshold above 1D-CAQR-EG's b*): nodes up
    to 128 wide are base cases, themselves split down to 64-wide TSQR."""
    p = m_.Handle.plan(20000, 1000, m_.Handle.opts(b=128))
    assert p["tuning"]["b"] == 128 and p["tuning"]["bstar"] == 64
    check_plan(p, 20000, 1000)
    assert max(x[2] for x in p["panels"]) == 64


@pytest.mark.parametrize("m,n", [(1024, 64), (1048576, 64), (262144, 256), (16384, 16384),
                                 (65536, 8192), (65536, 2048), (5000, 150)])
def test_autotuned_plans_are_valid_and_deterministic(m_, m, n):
    for lstsq in (False, True):
        p = m_.Handle.plan(m, n, None, lstsq)
        check_plan(p, m, n)
        assert p == m_.Handle.plan(m, n, None, lstsq)
        t = p["tuning"]
        assert t["b"] in (32, 64, 128) and t["bstar"] in (32, 64) and t["bstar"] <= t["b"]
        assert p["cost"]["seconds"] > 0
        if not lstsq:
            assert t["t_layout"] == 0  # qr_factor returns the full T unless asked


def test_fixed_fields_are_kept(m_):
    o = m_.Handle.opts(b=32, leaf_rows=256, chain=3, arity=3)
    p = m_.Handle.plan(100000, 200, o)
    t = p["tuning"]
    assert (t["b"], t["bstar"], t["leaf_rows"], t["chain"], t["arity"]) == (32, 32, 256, 3, 3)
    assert all(x[3:6] == [256, 3, 3] for x in p["panels"])


@pytest.mark.parametrize("kw", [dict(b=5000), dict(bstar=65), dict(b=32, bstar=64), dict(nb=5000),
                                dict(t_layout=2), dict(leaf_rows=64), dict(arity=1)])
def test_rejected_options(m_, kw):
    o = m_.Handle.opts(**kw)
    lib = m_.lib()
    assert lib.qr_plan(1000, 100, ctypes.byref(o), 0, None, 0) == -1
    assert lib.qr_t_rows(1000, 100, ctypes.byref(o)) == 0
    assert lib.qr_workspace_size(1000, 100, ctypes.byref(o)) == 0


def test_cost_model_prefers_blocked_for_square(m_):
    full = m_.Handle.plan(16384, 16384, m_.Handle.opts(t_layout=m_.T_FULL))
    blk = m_.Handle.plan(16384, 16384, m_.Handle.opts(t_layout=m_.T_BLOCKED))
    assert blk["cost"]["gemm_flops"] < 0.5 * full["cost"]["gemm_flops"]
    assert blk["cost"]["seconds"] < full["cost"]["seconds"]
