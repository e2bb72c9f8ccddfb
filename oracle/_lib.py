"""ctypes loader for the plain C oracle (test infrastructure only).

Builds ``oracle/libckks_oracle.so`` from ``ckks_oracle.c`` with gcc when it is
missing (or when ``build_oracle(force=True)`` is called). Floating-point
contraction is disabled so that encoding and sampling evaluate exactly the
operation sequence written in the C source.

``build_oracle(sanitize=True)`` builds ``libckks_oracle_san.so`` with gcc's
AddressSanitizer and UndefinedBehaviorSanitizer; a process that sets
``FHE_ORACLE_SANITIZED=1`` (and preloads gcc's libasan) loads that one instead.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ckks_oracle.c")
_SO = os.path.join(_HERE, "libckks_oracle.so")
_SO_SAN = os.path.join(_HERE, "libckks_oracle_san.so")
_SAN = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]

_lib = None


def build_oracle(force: bool = False, sanitize: bool = False) -> str:
    so = _SO_SAN if sanitize else _SO
    if force or not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O1" if sanitize else "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
               *(_SAN if sanitize else []), "-o", so + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(so + ".tmp", so)
    return so


u64 = ctypes.c_uint64
u64p = ctypes.POINTER(ctypes.c_uint64)
i64p = ctypes.POINTER(ctypes.c_int64)
dblp = ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "or_mulmod": ([u64, u64, u64], u64),
    "or_addmod": ([u64, u64, u64], u64),
    "or_submod": ([u64, u64, u64], u64),
    "or_powmod": ([u64, u64, u64], u64),
    "or_invmod_prime": ([u64, u64], u64),
    "or_is_prime": ([u64], ctypes.c_int),
    "or_find_primes": ([ctypes.c_int, ctypes.c_int, u64, u64p], ctypes.c_int),
    "or_primitive_2n_root": ([u64, u64], u64),
    "or_poly_mul_schoolbook": ([u64p, u64p, u64p, u64, u64], None),
    "or_ntt_forward": ([u64p, u64, u64], None),
    "or_ntt_inverse": ([u64p, u64, u64], None),
    "or_poly_mul": ([u64p, u64p, u64p, u64, u64], None),
    "or_splitmix_first": ([u64, u64, u64, u64p], u64),
    "or_sample_uniform": ([u64, u64, u64, u64, u64p], None),
    "or_sample_ternary": ([u64, u64, u64, i64p], None),
    "or_sample_gauss": ([u64, u64, u64, ctypes.c_double, ctypes.c_int64, i64p], None),
    "or_encode": ([dblp, u64, ctypes.c_double, u64, i64p], None),
    "or_decode_slots": ([dblp, u64, ctypes.c_double, i64p, u64, dblp], None),
    "or_signed_to_limbs": ([i64p, u64, u64p, u64, u64p], None),
    "or_automorph": ([u64p, u64p, u64, u64, u64p, u64], None),
    "or_automorph_signed": ([i64p, i64p, u64, u64], None),
    "or_tag": ([u64, u64, u64, u64], u64),
    "or_keygen_switch": ([u64, u64, i64p, u64p, u64, u64p, u64, u64, u64, u64p], None),
    "or_encrypt": ([u64, u64, i64p, i64p, u64, u64p, u64, u64p], None),
    "or_decrypt_limbs": ([u64p, u64, u64, i64p, u64, u64p, u64p], None),
    "or_crt2_centered": ([u64p, u64p, u64, u64, u64, dblp], None),
    "or_modup": ([u64p, u64, u64, u64, u64p, u64, u64, u64p], None),
    "or_moddown": ([u64p, u64, u64p, u64, u64, u64p], None),
    "or_keyswitch": ([u64p, u64, u64p, u64, u64, u64, u64, u64p, u64p], None),
    "or_rescale": ([u64p, u64, u64, u64, u64p, u64p], None),
    "or_tensor": ([u64p, u64p, u64, u64, u64p, u64p], None),
    "or_mul_plain": ([u64p, u64, u64, i64p, u64, u64p, u64p], None),
    "or_add": ([u64p, u64p, u64, u64, u64, u64p, u64p], None),
}


def lib():
    global _lib
    if _lib is None:
        path = build_oracle(sanitize=os.environ.get("FHE_ORACLE_SANITIZED") == "1")
        handle = ctypes.CDLL(path)
        for name, (args, res) in _SIGS.items():
            fn = getattr(handle, name)
            fn.argtypes = args
            fn.restype = res
        _lib = handle
    return _lib


def P(a: np.ndarray):
    """Pointer to a C-contiguous numpy array (uint64, int64 or float64)."""
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    if a.dtype == np.uint64:
        return a.ctypes.data_as(u64p)
    if a.dtype == np.int64:
        return a.ctypes.data_as(i64p)
    if a.dtype == np.float64:
        return a.ctypes.data_as(dblp)
    raise TypeError(a.dtype)
