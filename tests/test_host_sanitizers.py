"""The C ABI layer's host code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only: the paths that need no device).

The library is rebuilt with both sanitizers on its host code
(paper_2601_19233_amd/build_sanitized.py) and loaded into a child Python
process that preloads the clang ASan runtime; the child drives the argument
validation of every entry point, context creation and destruction and the
option checks, and any sanitizer report fails the test.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import ctypes as C, sys
sys.path.insert(0, sys.argv[1])
from paper_2601_19233_amd import _lib, render
_lib.LIB_PATH = sys.argv[2]
lib = _lib.load()
h = C.c_void_p()
assert lib.umgs_create(None, None, None) == -1
for kw in [dict(tile=(16, 8)), dict(frag_batch=100), dict(sh_degree=4), dict(k_bind=2), dict(mode=7)]:
    o = render.make_options(**kw)
    assert lib.umgs_create(C.byref(h), C.byref(o), None) == -1, kw
    assert not h.value
d = _lib.Options()
lib.umgs_default_options(C.byref(d))
assert (d.tile_w, d.tile_h, d.frag_batch, d.k_bind) == (16, 16, 128, 8)
# a valid request without a device: the context is allocated, then freed
st = lib.umgs_create(C.byref(h), C.byref(d), None)
assert st in (-3, 0), st
if st == 0:
    lib.umgs_destroy(h)
lib.umgs_destroy(None)
assert lib.umgs_last_error(None) == b""
cam = (C.c_float * 3)(0.0, 0.0, 3.0)
n = 0
for name, (res, args) in _lib.PROTOTYPES.items():
    if name in ("umgs_default_options", "umgs_create", "umgs_destroy", "umgs_last_error"):
        continue
    vals = []
    for a in args:
        if a is _lib.I32 or a is C.c_int32:
            vals.append(0)
        elif a is _lib.I64:
            vals.append(0)
        elif a is C.POINTER(C.c_float):
            vals.append(cam)
        else:
            vals.append(None)
    assert getattr(lib, name)(*vals) == -1, name       # NULL context
    n += 1
print("checked", n, "entry points")
'''


@pytest.mark.slow
def test_abi_host_code_under_asan_and_ubsan(tmp_path):
    from paper_2601_19233_amd import build_sanitized as BS
    if not os.path.exists(BS.HIPCC):
        pytest.skip("hipcc not found")
    lib = BS.build()
    rt = BS.runtime()
    assert rt and os.path.exists(rt), "clang ASan runtime not found"
    env = dict(os.environ, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               HIP_VISIBLE_DEVICES=os.environ.get("HIP_VISIBLE_DEVICES", ""))
    script = tmp_path / "child.py"
    script.write_text(CHILD)
    r = subprocess.run([sys.executable, str(script), ROOT, lib], env=env, capture_output=True,
                       text=True, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "checked" in r.stdout
