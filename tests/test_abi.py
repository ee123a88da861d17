"""The C ABI: every function declared in include/*.h is exported by
libcorr.so, and the Python binding declares exactly those (CPU only: no
compute call is made here)."""
import ctypes
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(\w+)\s*\(", text, flags=re.M):
            name = m.group(1)
            if name not in ("if", "sizeof", "defined"):
                names.add(name)
    return names


@pytest.fixture(scope="module")
def libpath():
    import __graft_entry__ as g
    g._ensure_built()
    from paper_2309_03308_amd import _lib
    return _lib.LIB_PATH


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for n in ("corr_pearson_pairs", "corr_ksg_mi_pairs", "corr_region_max", "corr_create", "corr_destroy"):
        assert n in names


def test_every_declared_symbol_is_exported(libpath):
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = sorted(declared_functions() - exported)
    assert not missing, missing


def test_binding_matches_header(libpath):
    from paper_2309_03308_amd import _lib
    L = _lib.load(libpath)
    assert set(_lib.SIGNATURES) == declared_functions()
    for n in _lib.SIGNATURES:
        assert hasattr(L, n)
    assert L.corr_status_str(1) == b"invalid argument"


def test_struct_layouts():
    from paper_2309_03308_amd import _lib
    assert ctypes.sizeof(_lib.corr_field) == 40
    assert ctypes.sizeof(_lib.corr_region) == 24
    assert ctypes.sizeof(_lib.corr_max) == 24


def test_null_context_rejected_without_gpu(libpath):
    # argument validation happens on the host before any device work
    from paper_2309_03308_amd import _lib
    L = _lib.load(libpath)
    st = L.corr_pearson_pairs(None, None, None, None, 0, 0, None, None)
    assert st == _lib.CORR_EINVAL
    assert b"context" in L.corr_last_error()
