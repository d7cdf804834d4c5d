"""CPU-side checks of the C ABI: the library loads and exports every symbol the
header declares, option defaults match the header, NULL arguments fail cleanly.
No GPU work is launched here."""
import ctypes
import os
import re

import pytest

from paper_2507_00129_amd import lya as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "lya.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lya_[a-z0-9_]+)\s*\(", text)))


def test_header_symbols_exported():
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(L.LIB_PATH)
    names = _declared_functions()
    assert {"lya_create", "lya_xi", "lya_dmat", "lya_xi_backward", "lya_last_error",
            "lya_xi_subsamples", "lya_xi_covariance", "lya_xi_means", "lya_xi3"} <= set(names)
    for n in names:
        assert hasattr(lib, n), f"{n} declared in lya.h but not exported"


def test_struct_layouts_match_header():
    assert ctypes.sizeof(L.lya_forests) == 8 * 10 + 8
    assert ctypes.sizeof(L.lya_grid) == 24
    assert ctypes.sizeof(L.lya_grid3) == 4 * 3 + 4 + 3 * 8
    assert ctypes.sizeof(L.lya_options) == 4 * 8 + 8 + 8 + 8
    assert L.lya_options.deterministic.offset == 48
    assert L.lya_options.dmat_keep_fraction.offset == 32
    assert ctypes.sizeof(L.lya_stats) == 3 * 8 + 2 * 4 + 4 * 4 + 3 * 8


def test_defaults_and_null_arguments():
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("library not built")
    lib = L.load_library()
    o = L.lya_options()
    lib.lya_options_default(ctypes.byref(o))
    assert (o.precision, o.eta, o.project_deltas, o.autotune, o.validate) == (L.FP32_COMP, L.ETA_MEAN_SLOPE, 0, 1, 1)
    assert o.dmat_keep_fraction == 1.0 and o.variant == -1
    assert lib.lya_xi(None, None, None, None, None, None, None, None, None) == L.LYA_E_INVALID
    assert lib.lya_xi_noalloc(None, None, None, None, None, None, None, None, None) == L.LYA_E_INVALID
    assert lib.lya_measure_peaks(None, None, None) == L.LYA_E_INVALID
    assert lib.lya_dmat(None, None, None, None, None, None, None) == L.LYA_E_INVALID
    assert lib.lya_xi_backward(None, None, None, None, None, None, None, None, None, None) == L.LYA_E_INVALID
    assert lib.lya_xi_subsamples(None, None, None, None, None, None, 1, None, None, None, None) == L.LYA_E_INVALID
    assert lib.lya_xi_covariance(None, None, None, 1, 1, None, None, None) == L.LYA_E_INVALID
    assert lib.lya_xi_means(None, None, None, None, None, None, None, None, None, None, None, None) == L.LYA_E_INVALID
    assert lib.lya_xi3(None, None, None, None, None, None, None, None, None) == L.LYA_E_INVALID
    assert lib.lya_xi3_subsamples(None, None, None, None, None, None, 1, None, None, None, None) == L.LYA_E_INVALID
    assert o.counters == 0 and o.deterministic == 0
    assert lib.lya_variant_name(0, 0) and lib.lya_variant_name(1, 0)
    assert lib.lya_variant_name(0, -1) is None and lib.lya_variant_name(1, 99) is None
    assert lib.lya_variant_name(2, 0) is None
    assert lib.lya_create(None, 0) == L.LYA_E_INVALID
    assert lib.lya_last_error(None) == b"NULL context"
