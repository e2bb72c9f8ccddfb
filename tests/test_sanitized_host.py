"""Host code under AddressSanitizer + UndefinedBehaviorSanitizer (CPU only, no GPU).

* The library's host code (built with the sanitizers behind -Xarch_host; device code as usual) runs
  its host-only entry points in a child process that preloads clang's ASan runtime: the planner on
  random and workload-sized patterns against the oracle's Algorithm 1 traversal, its malformed-pattern
  rejections, the ABI export check and the parameter checks of context creation.
* The C oracle (built with gcc's sanitizers) runs its arithmetic, sampling, encoding and operation
  pins in a child process that preloads gcc's libasan.
A sanitizer report aborts the child (halt_on_error, no recovery from undefined behaviour).
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.slow

_ASAN = "detect_leaks=0:halt_on_error=1:abort_on_error=1"


def _child(env_extra, tests):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = _ASAN
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu", *tests]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    return out


def _probe(env_extra, code):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = _ASAN
    return subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=300)


def test_library_host_code_under_asan_ubsan():
    from paper_2604_11659_amd import build
    lib = build.build(sanitize=True)
    env = {"LD_PRELOAD": build.host_asan_runtime(), "FHE_SPMSPM_LIB": lib}
    # the child really loads the sanitized build next to the ASan runtime
    r = _probe(env, "from paper_2604_11659_amd import fhe; maps = open('/proc/self/maps').read(); "
                    "assert fhe.LIB_PATH.endswith('_san.so') and fhe.LIB_PATH in maps, fhe.LIB_PATH; "
                    "assert 'libclang_rt.asan' in maps; print('ok')")
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr
    out = _child(env, ["tests/test_planner_host.py", "tests/test_library_abi.py"])
    assert " passed" in out


def test_oracle_under_asan_ubsan():
    from oracle import _lib
    _lib.build_oracle(force=True, sanitize=True)
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    assert os.path.isabs(libasan), libasan
    env = {"LD_PRELOAD": os.path.realpath(libasan), "FHE_ORACLE_SANITIZED": "1"}
    # positive control: the sanitized oracle is the one loaded, and a modulus of 0 (a division by zero
    # in the mulmod definition) is reported and aborts
    r = _probe(env, "from oracle import lib; l = lib(); print('loaded', flush=True); l.or_mulmod(1, 1, 0)")
    assert "loaded" in r.stdout and r.returncode != 0 and "division by zero" in r.stderr, r.stdout + r.stderr
    out = _child(env, ["tests/test_oracle_arith.py", "tests/test_oracle_sampling_encoding.py",
                       "tests/test_oracle_ops.py"])
    assert " passed" in out
