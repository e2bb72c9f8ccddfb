"""The C-ABI library loads on the CPU and exports every symbol the header declares (no compute)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fhe_spmspm.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(fhe_[a-z_0-9]+)\s*\(", txt)) - {"fhe_alloc_fn", "fhe_free_fn"})


def test_library_exports_every_declared_symbol():
    from paper_2604_11659_amd import fhe
    lib = ctypes.CDLL(fhe.LIB_PATH)
    names = _declared()
    assert len(names) >= 25
    for name in names:
        assert hasattr(lib, name), name
    # the binding wraps every declared entry point
    assert set(names) <= set(fhe.exported_symbols())


def test_error_path_without_device_work():
    from paper_2604_11659_amd import fhe
    d = fhe.fhe_params_desc(9, 4, 50, 1, 60, 1, 1, 40, 10, 0)  # log_n 9 is out of range
    out = ctypes.c_void_p()
    rc = fhe._lib.fhe_params_create(ctypes.byref(d), ctypes.byref(out))
    assert rc == -1 and out.value is None
    assert b"log_n" in fhe._lib.fhe_last_error()


def test_too_few_q_primes_is_a_level_error():
    """FHE_ELEVEL: the method needs two rescales, so a parameter set with fewer than 3 Q primes is
    refused before any device work."""
    from paper_2604_11659_amd import fhe
    d = fhe.fhe_params_desc(13, 2, 50, 1, 60, 1, 1, 40, 10, 0)
    out = ctypes.c_void_p()
    rc = fhe._lib.fhe_params_create(ctypes.byref(d), ctypes.byref(out))
    assert rc == -3 and out.value is None
    assert b"3 Q primes" in fhe._lib.fhe_last_error()
