"""Pins of the oracle's sampling and canonical-embedding encode/decode."""
import math
import os

import numpy as np
import pytest

from oracle import ckks
from oracle._lib import P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_kat.txt")


def _kat():
    seed, vals = None, []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("seed"):
            seed = int(line.split()[1])
        else:
            vals.append(int(line))
    return seed, vals


def test_splitmix64_known_answer(oracle_lib):
    seed, vals = _kat()
    out = np.zeros(len(vals), np.uint64)
    oracle_lib.or_splitmix_first(seed, 0, len(vals), P(out))  # tag 0: state0 = seed
    assert [int(x) for x in out] == vals


def test_stream_tags_are_distinct(oracle_lib):
    a = np.zeros(4, np.uint64)
    b = np.zeros(4, np.uint64)
    oracle_lib.or_splitmix_first(42, ckks.tag(2, 0, 1, 3), 4, P(a))
    oracle_lib.or_splitmix_first(42, ckks.tag(2, 0, 1, 4), 4, P(b))
    assert not (a == b).any()


def test_ternary_distribution():
    s = ckks.sample_ternary(7, ckks.tag(1), 1 << 16)
    vals, counts = np.unique(s, return_counts=True)
    assert list(vals) == [-1, 0, 1]
    expect = (1 << 16) / 3
    chi2 = float(((counts - expect) ** 2 / expect).sum())
    assert chi2 < 20.0  # 2 dof, p ~ 5e-5


def test_gaussian_moments_and_bound():
    e = ckks.sample_gauss(7, ckks.tag(5), 1 << 17)
    assert np.abs(e).max() <= 19
    assert abs(e.mean()) < 0.05
    # rounding adds variance 1/12
    assert abs(e.std() - math.sqrt(3.2 ** 2 + 1 / 12)) < 0.05


def test_uniform_range_and_mean():
    q = 1125899906826241
    u = ckks.sample_uniform(9, ckks.tag(4, 0, 0, 1), q, 1 << 16)
    assert int(u.max()) < q
    assert abs(float(u.mean()) / q - 0.5) < 0.01


def test_encode_constant_vector_closed_form():
    """Encoding of the all-c vector over every slot is c*Delta in coefficient 0 and 0 elsewhere:
    the cosines of the non-zero coefficients sum to zero over the S conjugate pairs."""
    N = 1 << 10
    delta = 2.0 ** 40
    m = ckks.encode(np.full(N // 2, 0.75), delta, N)
    assert m[0] == round(0.75 * delta)
    assert (m[1:] == 0).all()


def test_decode_monomial_closed_form():
    """Slot t of the monomial X is Re(zeta^(5^t)) = cos(pi 5^t / N)."""
    N = 1 << 8
    mono = np.zeros(N)
    mono[1] = 1.0
    slots = np.arange(N // 2)
    out = ckks.decode_poly(mono, 1.0, slots)
    ref = np.array([math.cos(math.pi * pow(5, int(t), 2 * N) / N) for t in slots])
    assert np.abs(out - ref).max() < 1e-12


@pytest.mark.parametrize("log_n", [6, 10, 13])
def test_encode_decode_roundtrip(log_n):
    N = 1 << log_n
    rng = np.random.default_rng(log_n)
    z = rng.uniform(-1, 1, N // 2)
    z[rng.random(N // 2) < 0.3] = 0.0
    delta = 2.0 ** 40
    m = ckks.encode(z, delta, N)
    out = ckks.decode_poly(m.astype(np.float64), delta, np.arange(N // 2))
    assert np.abs(out - z).max() < 1e-9


def test_rotation_is_automorphism_on_encodings():
    """tau_(5^r) turns slot t into slot t + r (left rotation) on the encoding."""
    N = 1 << 9
    S = N // 2
    z = np.random.default_rng(4).uniform(-1, 1, S)
    delta = 2.0 ** 40
    m = ckks.encode(z, delta, N)
    for r in [1, 5, S - 1, 77]:
        mr = ckks.automorph_signed(m, pow(5, r, 2 * N))
        out = ckks.decode_poly(mr.astype(np.float64), delta, np.arange(S))
        assert np.abs(out - np.roll(z, -r)).max() < 1e-9


def test_mask_decodes_to_one_hot():
    params = ckks.Params(log_n=10, n_q=4, n_p=1, alpha=1, rot_digits=1)
    S = params.S
    for p in [0, 1, 17, S - 1]:
        mk = ckks.mask(params, p)
        out = ckks.decode_poly(mk.astype(np.float64), params.delta_mask, np.arange(S))
        ref = np.zeros(S)
        ref[p] = 1.0
        assert np.abs(out - ref).max() < 2.0 ** -30
