"""Host-side checks of the C ABI: the library loads, exports every function
that include/hisq.h declares, and validates arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_1712_00143_amd import hisq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "hisq.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hisq_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ["hisq_create", "hisq_load_links", "hisq_dslash", "hisq_cg", "hisq_multishift_cg",
              "hisq_batch_cg", "hisq_cg_learned"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    L = hisq.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert set(_declared()) <= set(hisq.EXPORTS)


def test_status_strings():
    assert hisq.hisq_status_string(0) == "ok"
    assert "reconstruct" in hisq.hisq_status_string(hisq.HISQ_ERR_RECON)


def test_create_rejects_odd_extents_without_gpu():
    h = ctypes.c_void_p()
    for dims in [(3, 4, 4, 4), (4, 4, 4, 0), (4, 4, 5, 4)]:
        d = (ctypes.c_int * 4)(*dims)
        st = hisq.lib().hisq_create(d, 0, None, ctypes.byref(h))
        assert st == hisq.HISQ_ERR_ARG
        assert "even" in hisq.hisq_last_error(None)


def test_default_params():
    p = hisq.hisq_default_params()
    assert p.tol == 1e-10 and p.sloppy == hisq.HISQ_F64 and p.recon == 18 and p.delta == 0.1


def test_null_handle_calls_fail_cleanly():
    L = hisq.lib()
    assert L.hisq_destroy(None) == hisq.HISQ_ERR_ARG
    assert L.hisq_prepare_links(None, 1, 18) == hisq.HISQ_ERR_ARG
