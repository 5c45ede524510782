"""CPU checks of the C-ABI library: it loads and exports every function that include/*.h
declares (no compute call: there is no GPU here)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(sa_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("sa_setup", "sa_solve", "sa_destroy", "sa_hierarchy_info",
                     "sa_export_level"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2103_10476_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_default_options_roundtrip():
    """sa_default_options needs no GPU: it fills the struct with the paper's defaults."""
    from paper_2103_10476_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    o = _lib.SaOptions()
    _lib.lib().sa_default_options(ctypes.byref(o))
    assert o.struct_size == ctypes.sizeof(_lib.SaOptions)
    assert o.theta == 0.02 and o.tau == 1.1 and o.max_coarse == 1000 and o.degree == 2
    assert o.cheb_ratio == 10.0 and o.power_iters == 10
    assert o.dist_power == 1 and o.coarse_solver == 0  # 1/d weights; Cholesky


def test_status_strings():
    from paper_2103_10476_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    for code in _lib.STATUS_NAMES:
        assert _lib.lib().sa_status_string(code)


def test_product_path_never_loads_oracle():
    """The package must not import or load anything under oracle/."""
    pkg = os.path.join(ROOT, "paper_2103_10476_amd")
    for path in glob.glob(os.path.join(pkg, "**", "*"), recursive=True):
        if path.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
            text = open(path).read()
            assert not re.search(r"import\s+oracle|from\s+oracle|liboracle|oracle/", text), path
