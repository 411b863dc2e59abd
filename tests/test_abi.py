"""The C-ABI library loads and exports every entry point include/hs.h declares;
host-only calls validate their arguments (no GPU needed)."""
import os
import re

import numpy as np
import pytest

from oracle import summaries as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"^\s*(?:hs_status|const char\*)\s+(hs_\w+)\s*\(", text, re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    from paper_2212_13297_amd import hs
    lib = hs.load()
    names = declared_functions()
    assert len(names) >= 9
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) <= set(hs._SIGS)


def test_breakpoints_are_float32_roundings_of_normal_quantiles():
    from paper_2212_13297_amd import hs
    b = hs.hs_breakpoints(8)
    ref = S.breakpoints(256)[1:-1]
    np.testing.assert_array_equal(b, ref.astype(np.float32))
    with pytest.raises(hs.HSError):
        hs.hs_breakpoints(4)


def test_index_bytes_and_param_validation():
    from paper_2212_13297_amd import hs
    p = hs.Params(w=16, leaf_size=1000).c(256)
    N = 1000
    nb = hs.hs_index_bytes(N, p)
    assert nb >= N * 256 * 4 + N * 4 + N * 16
    assert hs.hs_index_bytes(N, hs.Params(w=8).c(200)) >= N * 256 * 4     # rows padded to 64 points
    for bad in (hs.Params(w=7).c(256), hs.Params(w=16, card_bits=4).c(256), hs.Params(leaf_size=0).c(256),
                hs.Params(l_max=-1).c(256), hs.Params(w=16).c(0), hs.Params(w=65).c(65 * 2),
                hs.Params(eapca_th=float("nan")).c(256)):
        with pytest.raises(hs.HSError) as e:
            hs.hs_index_bytes(N, bad)
        assert e.value.code == hs.HS_EINVAL
    for badN in (0, -5, 1 << 32):
        with pytest.raises(hs.HSError):
            hs.hs_index_bytes(badN, p)
    assert "N=" in hs.hs_last_error()


def test_read_probe_rejects_bad_arguments():
    import ctypes
    from paper_2212_13297_amd import hs
    lib = hs.load()
    ms = ctypes.c_double()
    sink = ctypes.c_uint32()
    # argument errors are reported before any device call
    assert lib.hs_read_probe(None, 1 << 20, 1, ctypes.addressof(sink), None, ctypes.byref(ms)) == -1
    assert lib.hs_read_probe(ctypes.addressof(sink), 1 << 20, 1, None, None, ctypes.byref(ms)) == -1
    assert lib.hs_read_probe(ctypes.addressof(sink), 1000, 1, ctypes.addressof(sink), None, ctypes.byref(ms)) == -1
    assert lib.hs_read_probe(ctypes.addressof(sink), 1 << 20, 0, ctypes.addressof(sink), None, ctypes.byref(ms)) == -1


def test_lds_probe_rejects_bad_arguments():
    import ctypes
    from paper_2212_13297_amd import hs
    lib = hs.load()
    out = ctypes.c_double()
    sink = ctypes.c_uint32()
    # argument errors are reported before any device call
    assert lib.hs_lds_probe(0, 16, 1, None, None, ctypes.byref(out)) == -1
    assert lib.hs_lds_probe(0, 16, 1, ctypes.addressof(sink), None, None) == -1
    assert lib.hs_lds_probe(2, 16, 1, ctypes.addressof(sink), None, ctypes.byref(out)) == -1
    assert lib.hs_lds_probe(0, 0, 1, ctypes.addressof(sink), None, ctypes.byref(out)) == -1
    assert lib.hs_lds_probe(1, (1 << 20) + 1, 1, ctypes.addressof(sink), None, ctypes.byref(out)) == -1
    assert lib.hs_lds_probe(1, 16, 0, ctypes.addressof(sink), None, ctypes.byref(out)) == -1
    assert "pattern" in hs.hs_last_error()
