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
    assert "file" in hisq.hisq_status_string(hisq.HISQ_ERR_IO)
    # every declared status has its own message
    codes = [0, -1, -2, -3, -4, -5, -6, -7, -8]
    assert len({hisq.hisq_status_string(c) for c in codes}) == len(codes)


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
    n = ctypes.c_int(0)
    assert L.hisq_residual_history(None, 0, None, 0, ctypes.byref(n)) == hisq.HISQ_ERR_ARG
    assert L.hisq_ptc_save(None, b"x") == hisq.HISQ_ERR_ARG
    assert L.hisq_ptc_load(None, b"x") == hisq.HISQ_ERR_ARG
    assert L.hisq_ptc_set_loss(None, 0) == hisq.HISQ_ERR_ARG
    assert L.hisq_ptc_init_polynomial(None, ctypes.c_double(4.0), ctypes.c_double(1.2), 30, None) == \
        hisq.HISQ_ERR_ARG


def test_bench_refuses_several_gpus():
    """The benchmark runs on one GPU; asking for more exits with a message
    (before it touches a GPU)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr
