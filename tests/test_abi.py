"""The C-ABI library loads on a machine without a GPU and exports every function the headers
declare; the Python binding declares exactly that set (no compute calls here)."""
import ctypes
import glob
import os
import re

from paper_1801_04070_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"^[A-Za-z_][\w \*]*?\b(gq_\w+)\s*\(", src, flags=re.M))
    return names


def test_headers_declare_functions():
    d = _declared()
    assert "gq_eval" in d and "gq_mlp_train_step" in d and len(d) >= 20


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_headers():
    assert set(_lib.EXPORTED) | set(_lib.EXPORTED_MLP) == _declared()
    L = _lib.load()
    for n in _lib.EXPORTED + _lib.EXPORTED_MLP:
        assert getattr(L, n).argtypes is not None, n
