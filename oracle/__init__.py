"""Plain CPU oracle for sparse x sparse RNS-CKKS ciphertext matmul.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``, never by the product library. It
shares no code with the HIP path; only the seeded input generators in
``paper_2604_11659_amd.synth`` (which hold none of the method's arithmetic)
serve both.

Parity status: every function is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py`` (schoolbook products, big-integer CRT identities,
decrypt-after-operation invariants, a slot-level simulator of the plan and the
FP64 matmul).
"""
from . import ckks, spmspm  # noqa: F401
from ._lib import build_oracle, lib  # noqa: F401
