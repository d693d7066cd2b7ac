"""The C-ABI library loads and exports every entry point declared in
include/unimgs.h; argument validation that needs no device is exercised."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "unimgs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(umgs_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("umgs_create", "umgs_destroy", "umgs_project", "umgs_bin", "umgs_sort", "umgs_blend",
              "umgs_bind_transfer", "umgs_bind_raycast", "umgs_set_proxy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2601_19233_amd import _lib
    lib = _lib.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding attaches a prototype to each of them
    assert set(declared_functions()) <= set(_lib.PROTOTYPES)


def test_option_validation_without_device():
    from paper_2601_19233_amd import _lib, render
    lib = _lib.load()
    h = C.c_void_p()
    assert lib.umgs_create(None, None, None) == -1
    bad = [dict(tile=(16, 8)), dict(frag_batch=100), dict(sh_degree=4), dict(k_bind=2), dict(mode=7)]
    for kw in bad:
        o = render.make_options(**kw)
        assert lib.umgs_create(C.byref(h), C.byref(o), None) == -1, kw
        assert not h.value
    d = _lib.Options()
    lib.umgs_default_options(C.byref(d))
    assert (d.tile_w, d.tile_h, d.frag_batch, d.k_bind) == (16, 16, 128, 8)
    assert lib.umgs_last_error(None) == b""
