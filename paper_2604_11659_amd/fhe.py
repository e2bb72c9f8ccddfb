"""Python binding of libfhe_spmspm.so (ctypes; argument marshalling only).

Every operation runs in the HIP library; this module converts numpy arrays and
handles and raises ``FheError`` on a negative return code. Importing it fails
loudly when the library has not been built (``python -m paper_2604_11659_amd.build``).

Streams: calls take an optional ``stream`` (an int hipStream_t handle or a
``torch.cuda.Stream``); by default torch's current stream is used when torch
sees a GPU, else the HIP default stream. Device memory comes from torch's
caching allocator when ``Context(..., allocator="torch")`` is requested,
otherwise from hipMalloc.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# FHE_SPMSPM_LIB selects another build of the same library (the host-sanitizer build of the CPU tests)
LIB_PATH = os.environ.get("FHE_SPMSPM_LIB") or os.path.join(_HERE, "libfhe_spmspm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2604_11659_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

c_i32, c_i64, c_u64, c_sz, c_dbl, c_vp = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t,
                                          ctypes.c_double, ctypes.c_void_p)
P_i32, P_i64, P_u64, P_dbl = (ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                              ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_double))
PP = ctypes.POINTER(ctypes.c_void_p)
P_u8 = ctypes.POINTER(ctypes.c_uint8)

FHE_ERRORS = {-1: "EINVAL", -2: "ESHAPE", -3: "ELEVEL", -4: "EKEY", -5: "ENOMEM", -6: "EAGAIN", -7: "EDEVICE",
              -8: "ECANCELED"}


class fhe_params_desc(ctypes.Structure):
    _fields_ = [("log_n", c_i32), ("n_q", c_i32), ("q_bits", c_i32), ("n_p", c_i32), ("p_bits", c_i32),
                ("alpha", c_i32), ("rot_digits", c_i32), ("log_delta", c_i32), ("mask_bits", c_i32),
                ("device", c_i32)]


class fhe_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", c_i64), ("total_ms", c_dbl), ("bytes", c_dbl),
                ("mulmods", c_dbl)]


class fhe_server_info(ctypes.Structure):
    _fields_ = [("p50_s", c_dbl), ("p99_s", c_dbl), ("completed", c_i64), ("failed", c_i64), ("cancelled", c_i64),
                ("inflight", c_i64), ("queued", c_i64), ("steps", c_i64), ("max_merged", c_i64),
                ("max_step_requests", c_i64), ("budget_bytes", c_sz), ("fixed_bytes", c_sz),
                ("inflight_bytes", c_sz)]


ALLOC_FN = ctypes.CFUNCTYPE(c_vp, c_sz, c_vp, c_vp)
FREE_FN = ctypes.CFUNCTYPE(None, c_vp, c_vp, c_vp)

_SIGS = {
    "fhe_set_allocator": ([ALLOC_FN, FREE_FN, c_vp], c_i32),
    "fhe_params_create": ([ctypes.POINTER(fhe_params_desc), PP], c_i32),
    "fhe_ctx_free": ([c_vp], None),
    "fhe_ctx_primes": ([c_vp, P_u64, c_sz], c_i32),
    "fhe_keygen": ([c_vp, c_u64, c_vp, PP], c_i32),
    "fhe_sk_free": ([c_vp], None),
    "fhe_keygen_rotations": ([c_vp, c_vp, P_i32, c_sz, c_vp], c_i32),
    "fhe_encrypt_csr": ([c_vp, c_vp, c_i32, c_i32, P_i32, P_i32, P_dbl, c_u64, c_vp, PP], c_i32),
    "fhe_encrypt_csc": ([c_vp, c_vp, c_i32, c_i32, P_i32, P_i32, P_dbl, c_u64, c_vp, PP], c_i32),
    "fhe_spmspm": ([c_vp, c_vp, c_vp, c_vp, PP], c_i32),
    "fhe_spmspm_pairs": ([c_vp, c_vp, c_vp, c_i64, c_i64, c_vp, PP], c_i32),
    "fhe_spmspm_batch": ([c_vp, c_sz, PP, PP, c_vp, PP], c_i32),
    "fhe_spmspm_batch_pairs": ([c_vp, c_sz, PP, PP, P_i64, P_i64, c_vp, PP], c_i32),
    "fhe_plan_stats": ([c_vp, c_vp, c_vp, P_i64], c_i32),
    "fhe_spmspm_plan": ([c_vp, c_sz, PP, PP, P_i64, P_i64, c_i32, c_vp, PP], c_i32),
    "fhe_plan_groups": ([c_vp, c_vp, c_vp, P_i64], c_i32),
    "fhe_spmspm_naive_sparse": ([c_vp, c_vp, c_vp, P_u8, P_u8, c_vp, PP], c_i32),
    "fhe_plan_stats_naive_sparse": ([c_vp, c_vp, c_vp, P_u8, P_u8, P_i64], c_i32),
    "fhe_autotune": ([c_vp, c_vp, c_vp, c_vp, c_i64, c_i32, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32),
                      ctypes.POINTER(c_dbl), ctypes.POINTER(c_i32), P_i32, P_i32, P_dbl, c_i32], c_i32),
    "fhe_plan_pattern": ([c_i32, c_i32, c_i32, c_i32, c_i32, P_i32, P_i32, P_i32, P_i32, P_i64], c_i32),
    "fhe_plan_rotations": ([c_vp, c_vp, c_vp, P_i32, c_sz, ctypes.POINTER(c_sz)], c_i32),
    "fhe_decrypt_decode": ([c_vp, c_vp, c_vp, c_vp, P_dbl, c_sz], c_i32),
    "fhe_mat_info": ([c_vp, P_i32, P_i32, P_i32, P_i32, P_i32, P_dbl], c_i32),
    "fhe_mat_export": ([c_vp, c_vp, c_i32, P_u64, c_sz, c_vp], c_i32),
    "fhe_mat_free": ([c_vp], None),
    "fhe_ct_import": ([c_vp, P_u64, c_i32, c_i32, c_dbl, c_vp, PP], c_i32),
    "fhe_ct_export": ([c_vp, c_vp, P_u64, c_sz, c_vp], c_i32),
    "fhe_ct_info": ([c_vp, P_i32, P_i32, P_dbl], c_i32),
    "fhe_ct_rotate": ([c_vp, c_vp, c_i32, c_vp, PP], c_i32),
    "fhe_ct_rotate_into": ([c_vp, c_vp, c_i32, c_vp, c_vp], c_i32),
    "fhe_ct_mult_relin": ([c_vp, c_vp, c_vp, c_vp, PP], c_i32),
    "fhe_ct_rescale": ([c_vp, c_vp, c_vp, PP], c_i32),
    "fhe_ct_mask": ([c_vp, c_vp, c_i32, c_vp, PP], c_i32),
    "fhe_ct_add": ([c_vp, c_vp, c_vp, c_vp, PP], c_i32),
    "fhe_ct_free": ([c_vp], None),
    "fhe_server_create": ([PP, c_sz, c_sz, c_sz, c_i32, c_i32, c_i32, PP], c_i32),
    "fhe_server_submit": ([c_vp, c_i32, c_vp, c_vp, ctypes.POINTER(c_u64)], c_i32),
    "fhe_server_set_plan": ([c_vp, c_i32], c_i32),
    "fhe_server_poll": ([c_vp, c_u64, c_i32, PP, P_dbl], c_i32),
    "fhe_server_stats": ([c_vp, ctypes.POINTER(fhe_server_info)], c_i32),
    "fhe_server_cancel": ([c_vp, c_u64], c_i32),
    "fhe_server_free": ([c_vp], None),
    "fhe_profile_enable": ([ctypes.c_int], c_i32),
    "fhe_profile_read": ([ctypes.POINTER(fhe_kernel_stat), c_sz], c_i32),
    "fhe_bench_mulmod": ([c_i32, c_i32, c_i32, c_vp, P_dbl], c_i32),
    "fhe_last_error": ([], ctypes.c_char_p),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


def exported_symbols():
    return sorted(_SIGS)


class FheError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"FHE_{FHE_ERRORS.get(code, code)}: {msg}")
        self.code = code


def _check(rc):
    if rc is not None and rc < 0:
        raise FheError(rc, _lib.fhe_last_error().decode())
    return rc


def _stream(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream
        except Exception:
            pass
        return None
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


def _arr(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def profile_enable(on: bool = True):
    """Start (clearing earlier records) or stop per-kernel HIP-event timing."""
    _check(_lib.fhe_profile_enable(1 if on else 0))


def profile_read() -> dict:
    """{kernel: dict(launches, total_ms, bytes, mulmods)} for the records since the last profile_enable(True)."""
    n = _check(_lib.fhe_profile_read(None, 0))
    arr = (fhe_kernel_stat * max(1, n))()
    _check(_lib.fhe_profile_read(arr, n))
    return {arr[i].name.decode(): dict(launches=arr[i].launches, total_ms=arr[i].total_ms, bytes=arr[i].bytes,
                                       mulmods=arr[i].mulmods)
            for i in range(n)}


def bench_mulmod(kind: int, iters: int = 4096, device: int = 0, stream=None) -> float:
    """Modular products per second of one form (0: FP64 for Q primes, 1: Shoup, 2: Montgomery for the
    60-bit special primes), from the library's throughput probe."""
    v = c_dbl()
    _check(_lib.fhe_bench_mulmod(device, kind, iters, _stream(stream), ctypes.byref(v)))
    return v.value


_TORCH_HOOKS = None


def use_torch_allocator():
    """Route the library's device allocations through torch's caching allocator."""
    global _TORCH_HOOKS
    import torch

    def _alloc(size, stream, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(size), stream=int(stream or 0))
        except Exception:
            return None

    def _free(ptr, stream, user):
        try:
            torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:
            pass

    _TORCH_HOOKS = (ALLOC_FN(_alloc), FREE_FN(_free))
    _check(_lib.fhe_set_allocator(_TORCH_HOOKS[0], _TORCH_HOOKS[1], None))


class _Handle:
    _free_fn = None

    def __init__(self, ptr, owner=None):
        self._ptr = ptr
        self._owner = owner

    def close(self):
        if self._ptr:
            type(self)._free_fn(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SecretKey(_Handle):
    _free_fn = staticmethod(_lib.fhe_sk_free)


class Matrix(_Handle):
    """Encrypted matrix handle (CSR operand, CSC operand or dense result)."""
    _free_fn = staticmethod(_lib.fhe_mat_free)

    def info(self):
        kind, rows, cols, chunks, limbs = (c_i32() for _ in range(5))
        scale = c_dbl()
        _check(_lib.fhe_mat_info(self._ptr, ctypes.byref(kind), ctypes.byref(rows), ctypes.byref(cols),
                                 ctypes.byref(chunks), ctypes.byref(limbs), ctypes.byref(scale)))
        return dict(kind=kind.value, rows=rows.value, cols=cols.value, chunks=chunks.value, limbs=limbs.value,
                    scale=scale.value)


class Ciphertext(_Handle):
    _free_fn = staticmethod(_lib.fhe_ct_free)

    def info(self):
        ncomp, limbs = c_i32(), c_i32()
        scale = c_dbl()
        _check(_lib.fhe_ct_info(self._ptr, ctypes.byref(ncomp), ctypes.byref(limbs), ctypes.byref(scale)))
        return dict(ncomp=ncomp.value, limbs=limbs.value, scale=scale.value)


@dataclass
class PlanStats:
    matched_pairs: int
    products: int
    align_keyswitches: int
    relin_keyswitches: int
    target_keyswitches: int
    result_chunks: int

    @property
    def keyswitches(self) -> int:
        return self.align_keyswitches + self.relin_keyswitches + self.target_keyswitches


def plan_pattern(log_n: int, rot_digits: int, m: int, k: int, n: int, csr_a, csc_b) -> "PlanStats":
    """Host-only plan statistics from the public patterns (csr_a = (indptr, indices) of A, csc_b of B)."""
    ipa, ixa = _arr(csr_a[0], np.int32), _arr(csr_a[1], np.int32)
    ipb, ixb = _arr(csc_b[0], np.int32), _arr(csc_b[1], np.int32)
    c = np.zeros(6, np.int64)
    _check(_lib.fhe_plan_pattern(log_n, rot_digits, m, k, n, _ptr(ipa, c_i32), _ptr(ixa, c_i32), _ptr(ipb, c_i32),
                                 _ptr(ixb, c_i32), _ptr(c, c_i64)))
    return PlanStats(*[int(x) for x in c])


class Context(_Handle):
    """Parameter set, device tables and evaluation keys on one GPU."""
    _free_fn = staticmethod(_lib.fhe_ctx_free)

    def __init__(self, log_n: int, n_q: int, n_p: int, alpha: int, rot_digits: int, q_bits: int = 50,
                 p_bits: int = 60, log_delta: int = 40, mask_bits: int = 10, device: int = 0,
                 allocator: str = "hip"):
        if allocator == "torch":
            use_torch_allocator()
        d = fhe_params_desc(log_n, n_q, q_bits, n_p, p_bits, alpha, rot_digits, log_delta, mask_bits, device)
        out = c_vp()
        _check(_lib.fhe_params_create(ctypes.byref(d), ctypes.byref(out)))
        super().__init__(out.value)
        self.log_n, self.n_q, self.n_p, self.alpha, self.rot_digits = log_n, n_q, n_p, alpha, rot_digits
        self.N = 1 << log_n
        self.S = self.N // 2

    @property
    def primes(self):
        n = _check(_lib.fhe_ctx_primes(self._ptr, None, 0))
        out = np.zeros(n, np.uint64)
        _check(_lib.fhe_ctx_primes(self._ptr, _ptr(out, c_u64), n))
        return [int(x) for x in out]

    def keygen(self, seed: int, stream=None) -> SecretKey:
        out = c_vp()
        _check(_lib.fhe_keygen(self._ptr, seed, _stream(stream), ctypes.byref(out)))
        return SecretKey(out.value, self)

    def keygen_rotations(self, sk: SecretKey, amounts, stream=None):
        a = _arr(list(amounts), np.int32)
        _check(_lib.fhe_keygen_rotations(self._ptr, sk._ptr, _ptr(a, c_i32), a.size, _stream(stream)))

    def _encrypt(self, fn, sk, rows, cols, indptr, indices, values, seed, stream):
        ip, ix, va = _arr(indptr, np.int32), _arr(indices, np.int32), _arr(values, np.float64)
        out = c_vp()
        _check(fn(self._ptr, sk._ptr, rows, cols, _ptr(ip, c_i32), _ptr(ix, c_i32), _ptr(va, c_dbl), seed,
                  _stream(stream), ctypes.byref(out)))
        return Matrix(out.value, self)

    def encrypt_csr(self, sk, rows, cols, indptr, indices, values, seed, stream=None) -> Matrix:
        return self._encrypt(_lib.fhe_encrypt_csr, sk, rows, cols, indptr, indices, values, seed, stream)

    def encrypt_csc(self, sk, rows, cols, indptr, indices, values, seed, stream=None) -> Matrix:
        return self._encrypt(_lib.fhe_encrypt_csc, sk, rows, cols, indptr, indices, values, seed, stream)

    def spmspm(self, A: Matrix, B: Matrix, stream=None, grouped: bool = False, graph: bool = False,
               tree: bool = False, hoist: bool = False) -> Matrix:
        """C = A B. grouped: pairs sharing (result chunk, target rotation) share one second rescale
        and one target rotation (FHE_PLAN_GROUPED); tree: grouped, with the target rotations shared
        digit by digit (FHE_PLAN_TREE). graph: record / replay the call as a HIP graph. hoist: hoisted
        alignment rotations (FHE_PLAN_HOIST)."""
        if grouped or graph or tree or hoist:
            return self.spmspm_batch([A], [B], stream, grouped=grouped, graph=graph, tree=tree, hoist=hoist)[0]
        out = c_vp()
        _check(_lib.fhe_spmspm(self._ptr, A._ptr, B._ptr, _stream(stream), ctypes.byref(out)))
        return Matrix(out.value, self)

    def spmspm_batch(self, As, Bs, stream=None, pair_ranges=None, grouped: bool = False,
                     graph: bool = False, tree: bool = False, hoist: bool = False) -> list:
        """[A_i B_i] in one merged launch stream (bit-identical to one-at-a-time spmspm).

        pair_ranges: optional [(begin, end)] per matmul, restricting each to those matched pairs.
        grouped: the grouped plan mode (FHE_PLAN_GROUPED). graph: FHE_PLAN_GRAPH (record the launch
        stream as a HIP graph on first use, replay it on later calls with the same operands)."""
        n = len(As)
        assert len(Bs) == n
        pa = (c_vp * max(1, n))(*[a._ptr for a in As])
        pb = (c_vp * max(1, n))(*[b._ptr for b in Bs])
        out = (c_vp * max(1, n))()
        if pair_ranges is None:
            lo = hi = None
        else:
            assert len(pair_ranges) == n
            lo = np.asarray([r[0] for r in pair_ranges] or [0], np.int64)
            hi = np.asarray([r[1] for r in pair_ranges] or [0], np.int64)
        _check(_lib.fhe_spmspm_plan(self._ptr, n, ctypes.cast(pa, PP), ctypes.cast(pb, PP),
                                    None if lo is None else _ptr(lo, c_i64), None if hi is None else _ptr(hi, c_i64),
                                    (2 if tree else 1 if grouped else 0) | (256 if graph else 0) | (512 if hoist else 0),
                                    _stream(stream),
                                    ctypes.cast(out, PP)))
        return [Matrix(out[i], self) for i in range(n)]

    def spmspm_pairs(self, A: Matrix, B: Matrix, begin: int, end: int, stream=None, grouped: bool = False,
                     tree: bool = False, hoist: bool = False) -> Matrix:
        if grouped or tree or hoist:
            return self.spmspm_batch([A], [B], stream, pair_ranges=[(begin, end)], grouped=grouped, tree=tree,
                                     hoist=hoist)[0]
        out = c_vp()
        _check(_lib.fhe_spmspm_pairs(self._ptr, A._ptr, B._ptr, begin, end, _stream(stream), ctypes.byref(out)))
        return Matrix(out.value, self)

    def autotune(self, A: Matrix | None = None, B: Matrix | None = None, pairs: int = 2000,
                 batch: int | None = None, stream=None) -> dict:
        """Pick the fastest NTT split and row-phase workgroup shape for this context (results are
        unchanged); returns the timings, keyed "k1/row threads".

        With A and B: times the first `pairs` matched pairs of A B; else synthetic key switches."""
        if batch is None:
            batch = {12: 256, 13: 256, 14: 256, 15: 128, 16: 32}.get(self.N.bit_length() - 1, 12)
        k1, rows, ms, n = c_i32(), c_i32(), c_dbl(), c_i32()
        cap = 32
        kt = np.zeros(cap, np.int32)
        rt = np.zeros(cap, np.int32)
        mt = np.zeros(cap, np.float64)
        _check(_lib.fhe_autotune(self._ptr, _stream(stream), A._ptr if A else None, B._ptr if B else None, pairs,
                                 batch, ctypes.byref(k1), ctypes.byref(rows), ctypes.byref(ms), ctypes.byref(n),
                                 _ptr(kt, c_i32), _ptr(rt, c_i32), _ptr(mt, c_dbl), cap))
        m = min(n.value, cap)
        return {"k1": k1.value, "row_threads": rows.value, "ms": ms.value, "mode": "plan" if A else "keyswitch",
                "pairs" if A else "batch": pairs if A else batch,
                "tried": {f"{int(kt[i])}/{int(rt[i])}": round(float(mt[i]), 3) for i in range(m)}}

    def plan_stats(self, A: Matrix, B: Matrix, nonzero_a=None, nonzero_b=None) -> PlanStats:
        """Plan counts of A B; with nonzero_a / nonzero_b, of the naive sparse plan (see spmspm_naive_sparse)."""
        c = np.zeros(6, np.int64)
        if nonzero_a is None and nonzero_b is None:
            _check(_lib.fhe_plan_stats(self._ptr, A._ptr, B._ptr, _ptr(c, c_i64)))
        else:
            za, zb = _arr(nonzero_a, np.uint8), _arr(nonzero_b, np.uint8)
            _check(_lib.fhe_plan_stats_naive_sparse(self._ptr, A._ptr, B._ptr, _ptr(za, ctypes.c_uint8),
                                                    _ptr(zb, ctypes.c_uint8), _ptr(c, c_i64)))
        return PlanStats(*[int(x) for x in c])

    def spmspm_naive_sparse(self, A: Matrix, B: Matrix, nonzero_a, nonzero_b, stream=None) -> Matrix:
        """The naive sparse method on operands that store every entry: a product runs unless both of its
        entries are zero. nonzero_a / nonzero_b: one flag per stored entry of A / B in packing order."""
        za, zb = _arr(nonzero_a, np.uint8), _arr(nonzero_b, np.uint8)
        out = c_vp()
        _check(_lib.fhe_spmspm_naive_sparse(self._ptr, A._ptr, B._ptr, _ptr(za, ctypes.c_uint8),
                                            _ptr(zb, ctypes.c_uint8), _stream(stream), ctypes.byref(out)))
        return Matrix(out.value, self)

    def plan_groups(self, A: Matrix, B: Matrix) -> tuple:
        """(groups, target-rotation key switches grouped, same with the digit tree) of A B."""
        c = np.zeros(3, np.int64)
        _check(_lib.fhe_plan_groups(self._ptr, A._ptr, B._ptr, _ptr(c, c_i64)))
        return int(c[0]), int(c[1]), int(c[2])

    def plan_rotations(self, A: Matrix, B: Matrix):
        n = c_sz()
        _check(_lib.fhe_plan_rotations(self._ptr, A._ptr, B._ptr, None, 0, ctypes.byref(n)))
        out = np.zeros(max(1, n.value), np.int32)
        _check(_lib.fhe_plan_rotations(self._ptr, A._ptr, B._ptr, _ptr(out, c_i32), out.size, ctypes.byref(n)))
        return [int(x) for x in out[: n.value]]

    def decrypt_decode(self, sk: SecretKey, M: Matrix, stream=None) -> np.ndarray:
        inf = M.info()
        if inf["kind"] == 2:
            shape, count = (inf["rows"], inf["cols"]), inf["rows"] * inf["cols"]
        else:
            count = None
            shape = None
        if count is None:
            count = inf["chunks"] * self.S
        out = np.zeros(max(1, count), np.float64)
        _check(_lib.fhe_decrypt_decode(self._ptr, sk._ptr, M._ptr, _stream(stream), _ptr(out, c_dbl), out.size))
        return out[:count].reshape(shape) if shape else out

    def export(self, M: Matrix, chunk: int, stream=None) -> np.ndarray:
        inf = M.info()
        out = np.zeros((2, inf["limbs"], self.N), np.uint64)
        _check(_lib.fhe_mat_export(self._ptr, M._ptr, chunk, _ptr(out, c_u64), out.size, _stream(stream)))
        return out

    # --- single-ciphertext operations -----------------------------------------------------------
    def ct_import(self, coeffs: np.ndarray, scale: float, stream=None) -> Ciphertext:
        a = _arr(coeffs, np.uint64)
        assert a.ndim == 3 and a.shape[2] == self.N
        out = c_vp()
        _check(_lib.fhe_ct_import(self._ptr, _ptr(a, c_u64), a.shape[0], a.shape[1], scale, _stream(stream),
                                  ctypes.byref(out)))
        return Ciphertext(out.value, self)

    def ct_export(self, ct: Ciphertext, stream=None) -> np.ndarray:
        inf = ct.info()
        out = np.zeros((inf["ncomp"], inf["limbs"], self.N), np.uint64)
        _check(_lib.fhe_ct_export(self._ptr, ct._ptr, _ptr(out, c_u64), out.size, _stream(stream)))
        return out

    def _ct1(self, fn, *args, stream=None):
        out = c_vp()
        _check(fn(self._ptr, *args, _stream(stream), ctypes.byref(out)))
        return Ciphertext(out.value, self)

    def ct_rotate(self, ct: Ciphertext, r: int, stream=None) -> Ciphertext:
        return self._ct1(_lib.fhe_ct_rotate, ct._ptr, r, stream=stream)

    def ct_rotate_into(self, ct: Ciphertext, r: int, out: Ciphertext, stream=None) -> Ciphertext:
        """ct_rotate into the existing `out` (same limb count) with no device allocation."""
        _check(_lib.fhe_ct_rotate_into(self._ptr, ct._ptr, r, out._ptr, _stream(stream)))
        return out

    def ct_mult_relin(self, a: Ciphertext, b: Ciphertext, stream=None) -> Ciphertext:
        return self._ct1(_lib.fhe_ct_mult_relin, a._ptr, b._ptr, stream=stream)

    def ct_rescale(self, ct: Ciphertext, stream=None) -> Ciphertext:
        return self._ct1(_lib.fhe_ct_rescale, ct._ptr, stream=stream)

    def ct_mask(self, ct: Ciphertext, slot: int, stream=None) -> Ciphertext:
        return self._ct1(_lib.fhe_ct_mask, ct._ptr, slot, stream=stream)

    def ct_add(self, a: Ciphertext, b: Ciphertext, stream=None) -> Ciphertext:
        return self._ct1(_lib.fhe_ct_add, a._ptr, b._ptr, stream=stream)


class Server(_Handle):
    """Continuous-batching request loop over one or more Contexts on one GPU (worker thread + own HIP
    stream), with one HBM budget shared by all of them."""
    _free_fn = staticmethod(_lib.fhe_server_free)

    def __init__(self, ctxs, hbm_budget: int, max_inflight: int = 8, slice_products: int = 64,
                 max_queue: int = 1024, grouped: bool = False, tree: bool = False, hoist: bool = False,
                 workspace_bytes: int = 0):
        if isinstance(ctxs, Context):
            ctxs = [ctxs]
        self._ctxs = list(ctxs)
        arr = (c_vp * len(self._ctxs))(*[c._ptr for c in self._ctxs])
        out = c_vp()
        _check(_lib.fhe_server_create(ctypes.cast(arr, PP), len(self._ctxs), hbm_budget, workspace_bytes,
                                      max_inflight, slice_products, max_queue, ctypes.byref(out)))
        super().__init__(out.value, self._ctxs)
        self._keep = {}
        if grouped or tree or hoist:
            _check(_lib.fhe_server_set_plan(self._ptr, (2 if tree else 1 if grouped else 0) | (512 if hoist else 0)))

    def submit(self, A: Matrix, B: Matrix, ctx_id: int = 0) -> int:
        t = c_u64()
        _check(_lib.fhe_server_submit(self._ptr, ctx_id, A._ptr, B._ptr, ctypes.byref(t)))
        self._keep[t.value] = (ctx_id, A, B)  # operands must outlive the request
        return t.value

    def poll(self, ticket: int, wait_ms: int = 0):
        """(Matrix, latency_s) when done, None while running; raises FheError if the request failed
        or was cancelled (code -8)."""
        out = c_vp()
        lat = c_dbl()
        rc = _lib.fhe_server_poll(self._ptr, ticket, wait_ms, ctypes.byref(out), ctypes.byref(lat))
        if rc == -6:
            return None
        ctx_id = self._keep.pop(ticket, (0,))[0]
        if rc < 0:
            raise FheError(rc, "request cancelled" if rc == -8 else "request failed")
        return Matrix(out.value, self._ctxs[ctx_id]), lat.value

    def cancel(self, ticket: int):
        """Cancel a queued request at once, an in-flight one at the next step boundary."""
        _check(_lib.fhe_server_cancel(self._ptr, ticket))

    def stats(self) -> dict:
        info = fhe_server_info()
        _check(_lib.fhe_server_stats(self._ptr, ctypes.byref(info)))
        return {name: getattr(info, name) for name, _ in fhe_server_info._fields_}
