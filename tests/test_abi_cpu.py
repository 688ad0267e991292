"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects invalid arguments before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fcrkpm.h")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fcrkpm_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2403_19854_amd import fcrkpm
    if not os.path.exists(fcrkpm.LIB_PATH):
        from paper_2403_19854_amd import build
        build.build()
    return fcrkpm.load_library()


def test_header_symbols_exported(lib):
    names = declared_symbols()
    assert {"fcrkpm_setup", "fcrkpm_apply", "fcrkpm_solve", "fcrkpm_adjoint"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    from paper_2403_19854_amd import fcrkpm
    assert set(fcrkpm.EXPORTS) == set(names)


def test_version_and_status_strings(lib):
    assert lib.fcrkpm_version() >= 100
    assert lib.fcrkpm_status_str(0) == b"FCRKPM_OK"
    assert lib.fcrkpm_status_str(2) == b"FCRKPM_ERR_SINGULAR"
    assert lib.fcrkpm_basis_size(None) == -1
    lib.fcrkpm_destroy(None)


def _setup(lib, dim=3, n=(16, 16, 16), h=(0.1, 0.1, 0.1), support=(2.5, 2.5, 2.5), degree=1,
           kernel=0, flags=0, mask=1):
    from paper_2403_19854_amd.fcrkpm import Grid
    g = Grid()
    g.dim = dim
    for k in range(3):
        g.n[k] = n[k]
        g.h[k] = h[k]
    g.dirichlet = None
    g.vol = None
    g.flags = flags
    out = C.c_void_p()
    sup = (C.c_double * 3)(*support)
    # the mask pointer is never dereferenced: every case below fails validation first
    st = lib.fcrkpm_setup(C.byref(g), C.c_void_p(mask) if mask else None, kernel, sup, degree,
                          None, C.byref(out))
    return st, out.value, lib.fcrkpm_last_error(None).decode()


@pytest.mark.parametrize("kw,frag", [
    (dict(dim=4), "dim"),
    (dict(degree=3), "degree"),
    (dict(kernel=7), "kernel"),
    (dict(flags=1), "flags"),
    (dict(n=(11 * 8, 16, 16)), "factor"),
    (dict(n=(2, 16, 16)), "box size"),
    (dict(support=(0.5, 2.5, 2.5)), "support"),
    (dict(n=(8, 8, 8), support=(4.5, 2.5, 2.5)), "support too large"),
    (dict(dim=2, n=(16, 16, 4)), "unused axes"),
    (dict(h=(0.0, 0.1, 0.1)), "spacing"),
    (dict(mask=0), "NULL"),
])
def test_setup_rejects_bad_arguments(lib, kw, frag):
    st, h, msg = _setup(lib, **kw)
    assert st == 1, (st, msg)
    assert h is None
    assert frag in msg


def test_null_context_calls(lib):
    assert lib.fcrkpm_apply(None, 0, 0, 1, None, None, None) == 1
    assert lib.fcrkpm_solve(None, 0, 1, None, None, None, None, 1e-8, 10, None, None) == 1
    assert lib.fcrkpm_adjoint(None, 0, 1, None, None, 1e-8, 10, None, None) == 1
    assert lib.fcrkpm_get_coeffs(None, 0, None, None) == 1
