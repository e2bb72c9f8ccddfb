"""Pins of the oracle's scalar arithmetic, prime search and negacyclic products.

Everything here is checked against Python big integers or against the
definition of the negacyclic product (schoolbook convolution with X^N = -1),
never against the oracle itself.
"""
import numpy as np
import pytest

from oracle._lib import P
from tests.bigint import is_prime, negacyclic_mul

Q50 = 1125899906826241  # a 50-bit prime = 1 mod 2^15
EDGE = [0, 1, 2, Q50 - 1, Q50 - 2, 1 << 49, (1 << 50) - 1]


def test_mulmod_matches_python(oracle_lib):
    rng = np.random.default_rng(0)
    for q in [Q50, 1152921504606830593, 97, (1 << 61) - 1]:
        vals = [v % q for v in EDGE] + [int(x) % q for x in rng.integers(0, 2**63, 200, dtype=np.uint64)]
        for a in vals[:40]:
            for b in vals[-40:]:
                assert oracle_lib.or_mulmod(a, b, q) == (a * b) % q
                assert oracle_lib.or_addmod(a, b, q) == (a + b) % q
                assert oracle_lib.or_submod(a, b, q) == (a - b) % q


def test_inverse_and_power(oracle_lib):
    for q in [Q50, 1152921504606830593]:
        for a in [1, 2, 3, 12345678901, q - 1]:
            inv = oracle_lib.or_invmod_prime(a, q)
            assert (inv * a) % q == 1
            assert oracle_lib.or_powmod(a, 1000003, q) == pow(a, 1000003, q)


@pytest.mark.parametrize("bits,count,log_n", [(50, 6, 13), (60, 3, 16), (50, 4, 15), (30, 5, 10)])
def test_find_primes_descending_and_complete(oracle_lib, bits, count, log_n):
    m = 2 << log_n
    out = np.zeros(count, np.uint64)
    assert oracle_lib.or_find_primes(bits, count, m, P(out)) == count
    ps = [int(x) for x in out]
    assert ps == sorted(ps, reverse=True)
    for p in ps:
        assert p < (1 << bits) and p % m == 1 and is_prime(p)
    # nothing skipped: every candidate = 1 mod m between 2^bits and the last prime that is
    # not in the list is composite
    cand = ((1 << bits) - 2) // m * m + 1
    listed = set(ps)
    while cand >= ps[-1]:
        assert is_prime(cand) == (cand in listed), cand
        cand -= m


def test_primitive_root(oracle_lib):
    for log_n in [3, 10, 13, 16]:
        N = 1 << log_n
        out = np.zeros(1, np.uint64)
        oracle_lib.or_find_primes(50, 1, 2 * N, P(out))
        q = int(out[0])
        psi = oracle_lib.or_primitive_2n_root(N, q)
        assert pow(psi, N, q) == q - 1 and pow(psi, 2 * N, q) == 1


@pytest.mark.parametrize("log_n", [2, 3, 4, 5, 6])
def test_poly_mul_equals_schoolbook_definition(oracle_lib, log_n):
    N = 1 << log_n
    rng = np.random.default_rng(log_n)
    for q in [int(x) for x in _primes(oracle_lib, 50, 2, N)] + [int(x) for x in _primes(oracle_lib, 60, 1, N)]:
        a = rng.integers(0, q, N, dtype=np.uint64)
        b = rng.integers(0, q, N, dtype=np.uint64)
        ref = negacyclic_mul([int(x) for x in a], [int(x) for x in b], q)
        c1 = np.zeros(N, np.uint64)
        c2 = np.zeros(N, np.uint64)
        oracle_lib.or_poly_mul(P(a), P(b), P(c1), N, q)
        oracle_lib.or_poly_mul_schoolbook(P(a), P(b), P(c2), N, q)
        assert [int(x) for x in c1] == ref
        assert [int(x) for x in c2] == ref


def test_poly_mul_special_cases(oracle_lib):
    """X^(N-1) * X = X^N = -1 and products with 1 are the identity."""
    N = 64
    q = int(_primes(oracle_lib, 50, 1, N)[0])
    a = np.zeros(N, np.uint64)
    a[N - 1] = 1
    b = np.zeros(N, np.uint64)
    b[1] = 1
    c = np.zeros(N, np.uint64)
    oracle_lib.or_poly_mul(P(a), P(b), P(c), N, q)
    expect = np.zeros(N, np.uint64)
    expect[0] = q - 1
    assert (c == expect).all()
    one = np.zeros(N, np.uint64)
    one[0] = 1
    r = np.random.default_rng(1).integers(0, q, N, dtype=np.uint64)
    oracle_lib.or_poly_mul(P(r), P(one), P(c), N, q)
    assert (c == r).all()


@pytest.mark.parametrize("log_n", [3, 5, 6])
def test_ntt_is_evaluation_at_odd_powers(oracle_lib, log_n):
    """Forward transform = evaluations at psi^(2i+1) (Horner with Python ints)."""
    N = 1 << log_n
    q = int(_primes(oracle_lib, 50, 1, N)[0])
    psi = oracle_lib.or_primitive_2n_root(N, q)
    a = np.random.default_rng(2).integers(0, q, N, dtype=np.uint64)
    f = a.copy()
    oracle_lib.or_ntt_forward(P(f), N, q)
    for i in range(N):
        x = pow(psi, 2 * i + 1, q)
        acc = 0
        for k in reversed(range(N)):
            acc = (acc * x + int(a[k])) % q
        assert int(f[i]) == acc
    oracle_lib.or_ntt_inverse(P(f), N, q)
    assert (f == a).all()


def test_ntt_roundtrip_large(oracle_lib):
    N = 1 << 13
    q = int(_primes(oracle_lib, 50, 1, N)[0])
    a = np.random.default_rng(3).integers(0, q, N, dtype=np.uint64)
    f = a.copy()
    oracle_lib.or_ntt_forward(P(f), N, q)
    assert not (f == a).all()
    oracle_lib.or_ntt_inverse(P(f), N, q)
    assert (f == a).all()


def _primes(lib, bits, count, N):
    out = np.zeros(count, np.uint64)
    lib.or_find_primes(bits, count, 2 * N, P(out))
    return out
