"""C-ABI checks that need no GPU: the library loads, exports every function
that include/miqr.h declares, and rejects bad arguments before touching a
device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "miqr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)) - {"sizeof"})


@pytest.fixture(scope="module")
def lib():
    import paper_1805_05278_amd as m
    if not os.path.exists(m.LIB_PATH):
        pytest.skip("libmiqr.so not built")
    return m.lib()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for f in ("miqr_create", "miqr_destroy", "qr_factor", "qr_apply_q", "qr_lstsq",
              "qr_form_q", "qr_solve_r", "qr_workspace_size", "miqr_status_string"):
        assert f in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), "missing export %s" % name


def test_status_strings(lib):
    for s in range(8):
        assert lib.miqr_status_string(s)
    assert lib.miqr_status_string(99) == b"unknown status"


def test_null_handle_is_einval(lib):
    import paper_1805_05278_amd as m
    assert lib.qr_factor(None, None, 10, 5, None, 10, None, 5, None) == m.EINVAL
    assert lib.qr_apply_q(None, None, b"T", 10, 5, 1, None, 10, None, 5, None, 10) == m.EINVAL
    assert lib.qr_lstsq(None, None, 10, 5, 1, None, 10, None, 10, None, None) == m.EINVAL
    assert lib.miqr_destroy(None) == m.EINVAL
    assert lib.miqr_create(None, 0) == m.EINVAL


def test_workspace_size_is_host_only(lib):
    assert lib.qr_workspace_size(1000, 64, None) > 0
    assert lib.qr_workspace_size(10, 20, None) == 0
    big = lib.qr_workspace_size(1 << 20, 64, None)
    assert 0 < big < (4 << 30)


def test_binding_rejects_non_colmajor():
    import numpy as np
    import paper_1805_05278_amd as m
    with pytest.raises((TypeError, ValueError)):
        m._mat(np.zeros((3, 3)), "A")
