"""The C ABI: libfftc.so loads on a machine without a GPU and exports every
function that include/*.h declares; the Python binding names each of them."""
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for path in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(path).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        text = "\n".join(l for l in text.splitlines() if not l.lstrip().startswith("#"))
        for m in re.finditer(r"\b(fftc_\w+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_headers_declare_entry_points():
    names = _declared()
    for must in ("fftc_create", "fftc_solve", "fftc_batch_solve", "fftc_nn_train_step", "fftc_solve_judged"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2607_26082_amd as F
    if not os.path.exists(F.LIB_PATH):
        from paper_2607_26082_amd import build
        build.build()
    lib = F.load()
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing
    unbound = [n for n in sorted(_declared()) if n not in F.exported_symbols()]
    assert not unbound, unbound
