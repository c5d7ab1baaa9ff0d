"""The C ABI library loads and exports every symbol the header declares, and
argument validation answers before any GPU work (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsrad.h")
LIB = os.path.join(ROOT, "paper_2509_18497_amd", "libgsrad.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gsrad_[A-Za-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        pytest.fail("libgsrad.so is not built (python -m paper_2509_18497_amd.build)")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n


def test_binding_lists_every_symbol():
    from paper_2509_18497_amd import gsrad
    assert sorted(gsrad.EXPORTS) == _declared()


def test_null_arguments_are_einval(L):
    L.gsrad_build_bvh.restype = ctypes.c_int32
    L.gsrad_last_error.restype = ctypes.c_char_p
    assert L.gsrad_build_bvh(None, None, None) == -1
    assert b"null" in L.gsrad_last_error()
    L.gsrad_form_factors.restype = ctypes.c_int32
    assert L.gsrad_form_factors(None, None, None, None) == -1
    L.gsrad_transport_solve.restype = ctypes.c_int32
    assert L.gsrad_transport_solve(None, None, None, 1, 1, 1, 0, None, None, None) == -1
    L.gsrad_ff_info.restype = ctypes.c_int32
    assert L.gsrad_ff_info(None, None, None) == -1
    L.gsrad_version.restype = ctypes.c_char_p
    assert L.gsrad_version().startswith(b"gsrad")


def test_bad_surfel_count_is_einval(L):
    from paper_2509_18497_amd.gsrad import _Surfels
    s = _Surfels(*([None] * 15), 0)
    L.gsrad_build_bvh.restype = ctypes.c_int32
    h = ctypes.c_void_p()
    assert L.gsrad_build_bvh(ctypes.byref(s), ctypes.byref(h), None) == -1
    s = _Surfels(*([None] * 15), 10)
    assert L.gsrad_build_bvh(ctypes.byref(s), ctypes.byref(h), None) == -1
    assert h.value is None


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asking for several exits with a
    message instead of reporting a figure."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert not r.stdout.strip().startswith("{")
