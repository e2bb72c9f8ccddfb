"""Plain RNS-CKKS oracle (test infrastructure only).

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may use
this module. It wraps the C definitions in ``ckks_oracle.c`` and follows the
paper's description of CKKS (Section 2.1) and the operations issued by its
Algorithm 2: EvalMult + Relinearize + Rescale, plaintext mask multiply,
EvalRotate (automorphism + key switch) and EvalAdd.

Readings of points the paper leaves open (each is stated in the design notes):
  * parameters: Q primes are the n_q largest primes below 2^q_bits with
    q = 1 (mod 2N), descending; P primes likewise below 2^p_bits;
  * hybrid key switching with alpha primes per digit (digits truncate at lower
    levels), ModUp/ModDown fast base conversion on [0, q) representatives;
  * rescale with nearest (centred) rounding of the dropped limb;
  * rotation by r is a left rotation (slot t receives slot t + r), realised
    with tau_g, g = 5^r mod 2N, and decomposed into at most ``rot_digits``
    power-of-2^b steps;
  * operand A encoded at 2^log_delta, operand B at exactly q_top, mask at
    2^mask_bits * q_(top-1), so the result scale is exactly 2^(log_delta+mask_bits).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from ._lib import P, lib

TAG_SECRET = 1
TAG_RELIN_A, TAG_RELIN_E = 2, 3
TAG_ENC_A, TAG_ENC_E = 4, 5
TAG_ROT_A, TAG_ROT_E = 6, 7


def tag(kind: int, sub1: int = 0, sub2: int = 0, sub3: int = 0) -> int:
    return (kind << 56) | (sub1 << 32) | (sub2 << 16) | sub3


def find_primes(bits: int, count: int, modulus: int) -> list[int]:
    out = np.zeros(count, np.uint64)
    got = lib().or_find_primes(bits, count, modulus, P(out))
    if got != count:
        raise ValueError("not enough primes")
    return [int(x) for x in out]


@dataclass
class Params:
    log_n: int
    n_q: int
    n_p: int
    alpha: int
    rot_digits: int
    q_bits: int = 50
    p_bits: int = 60
    log_delta: int = 40
    mask_bits: int = 10
    N: int = field(init=False)
    S: int = field(init=False)
    q: tuple = field(init=False)
    p: tuple = field(init=False)
    primes: np.ndarray = field(init=False, repr=False)

    def __post_init__(self):
        self.N = 1 << self.log_n
        self.S = self.N // 2
        self.q = tuple(find_primes(self.q_bits, self.n_q, 2 * self.N))
        cand = find_primes(self.p_bits, self.n_p + self.n_q, 2 * self.N)
        self.p = tuple([x for x in cand if x not in self.q][: self.n_p])
        self.primes = np.array(self.q + self.p, dtype=np.uint64)

    @property
    def top(self) -> int:  # top level index L (n_q - 1 limbs below it)
        return self.n_q - 1

    def qp(self, nl: int) -> np.ndarray:
        """Moduli of the first nl Q limbs."""
        return np.ascontiguousarray(self.primes[:nl])

    @property
    def delta_a(self) -> float:
        return float(2 ** self.log_delta)

    @property
    def delta_b(self) -> float:
        return float(self.q[self.n_q - 1])

    @property
    def delta_mask(self) -> float:
        return float(2 ** self.mask_bits) * float(self.q[self.n_q - 2])

    @property
    def delta_out(self) -> float:
        return float(2 ** (self.log_delta + self.mask_bits))

    def rot_step_bits(self) -> int:
        return -(-int(math.log2(self.S)) // self.rot_digits)


@dataclass
class Ct:
    data: np.ndarray  # uint64 [ncomp][nl][N], coefficient domain
    scale: float

    @property
    def nl(self) -> int:
        return self.data.shape[1]


def _u64(shape) -> np.ndarray:
    return np.zeros(shape, dtype=np.uint64)


# ----------------------------------------------------------------------------------------------
# Sampling / encoding
# ----------------------------------------------------------------------------------------------

def sample_ternary(seed: int, t: int, N: int) -> np.ndarray:
    out = np.zeros(N, np.int64)
    lib().or_sample_ternary(seed, t, N, P(out))
    return out


def sample_gauss(seed: int, t: int, N: int) -> np.ndarray:
    out = np.zeros(N, np.int64)
    lib().or_sample_gauss(seed, t, N, 3.2, 19, P(out))
    return out


def sample_uniform(seed: int, t: int, q: int, N: int) -> np.ndarray:
    out = _u64(N)
    lib().or_sample_uniform(seed, t, q, N, P(out))
    return out


def encode(z, delta: float, N: int) -> np.ndarray:
    z = np.ascontiguousarray(np.asarray(z, dtype=np.float64))
    assert z.size <= N // 2
    m = np.zeros(N, np.int64)
    lib().or_encode(P(z), z.size, delta, N, P(m))
    return m


def decode_poly(mpoly: np.ndarray, delta: float, slots) -> np.ndarray:
    """mpoly: real message coefficients (float64, already centred)."""
    slots = np.ascontiguousarray(np.asarray(slots, dtype=np.int64))
    out = np.zeros(slots.size, np.float64)
    mpoly = np.ascontiguousarray(mpoly, dtype=np.float64)
    lib().or_decode_slots(P(mpoly), mpoly.size, delta, P(slots), slots.size, P(out))
    return out


def automorph_signed(v: np.ndarray, g: int) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.int64)
    out = np.zeros_like(v)
    lib().or_automorph_signed(P(v), P(out), v.size, g)
    return out


def signed_to_limbs(v: np.ndarray, moduli: np.ndarray) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.int64)
    moduli = np.ascontiguousarray(moduli, dtype=np.uint64)
    out = _u64((moduli.size, v.size))
    lib().or_signed_to_limbs(P(v), v.size, P(moduli), moduli.size, P(out))
    return out


def poly_mul(a: np.ndarray, b: np.ndarray, q: int) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    out = np.zeros_like(a)
    lib().or_poly_mul(P(a), P(b), P(out), a.size, q)
    return out


# ----------------------------------------------------------------------------------------------
# Keys
# ----------------------------------------------------------------------------------------------

class Keys:
    """Secret key, relinearisation key and lazily generated rotation keys.

    A switching key array has shape [beta_top][2][n_q + n_p][N]: component 0
    is b_j, component 1 is a_j, over limbs q_0..q_L, p_0..p_(K-1).
    """

    def __init__(self, params: Params, seed: int):
        self.params = params
        self.seed = seed
        N = params.N
        self.s = sample_ternary(seed, tag(TAG_SECRET), N)
        s_l = signed_to_limbs(self.s, params.primes)
        s2 = np.stack([poly_mul(s_l[i], s_l[i], int(params.primes[i])) for i in range(len(params.primes))])
        self.relin = self._switch_key(0, s2)
        self._rot: dict[int, np.ndarray] = {}

    def _switch_key(self, key_id: int, sprime_limbs: np.ndarray) -> np.ndarray:
        pr = self.params
        beta = -(-pr.n_q // pr.alpha)
        key = _u64((beta, 2, pr.n_q + pr.n_p, pr.N))
        sp = np.ascontiguousarray(sprime_limbs, dtype=np.uint64)
        lib().or_keygen_switch(self.seed, key_id, P(self.s), P(sp), pr.N, P(pr.primes), pr.n_q, pr.n_p,
                               pr.alpha, P(key))
        return key

    def rot_key(self, g: int) -> np.ndarray:
        if g not in self._rot:
            target = automorph_signed(self.s, g)
            self._rot[g] = self._switch_key(g, signed_to_limbs(target, self.params.primes))
        return self._rot[g]


# ----------------------------------------------------------------------------------------------
# Ciphertext operations
# ----------------------------------------------------------------------------------------------

def encrypt(params: Params, keys: Keys, m: np.ndarray, seed: int, chunk: int, scale: float) -> Ct:
    ct = _u64((2, params.n_q, params.N))
    m = np.ascontiguousarray(m, dtype=np.int64)
    lib().or_encrypt(seed, chunk, P(m), P(keys.s), params.N, P(params.primes), params.n_q, P(ct))
    return Ct(ct, scale)


def decrypt_message(params: Params, keys: Keys, ct: Ct) -> np.ndarray:
    """Centred message coefficients (float64) from limbs q_0, q_1 by exact CRT."""
    nl = ct.nl
    assert nl >= 2
    d = np.ascontiguousarray(ct.data)
    lim = _u64((2, params.N))
    lib().or_decrypt_limbs(P(d), nl, 2, P(keys.s), params.N, P(params.primes), P(lim))
    out = np.zeros(params.N, np.float64)
    lib().or_crt2_centered(P(np.ascontiguousarray(lim[0])), P(np.ascontiguousarray(lim[1])), params.N,
                           params.q[0], params.q[1], P(out))
    return out


def decrypt_decode(params: Params, keys: Keys, ct: Ct, slots) -> np.ndarray:
    return decode_poly(decrypt_message(params, keys, ct), ct.scale, slots)


def automorph(params: Params, ct: Ct, g: int) -> Ct:
    ncomp, nl, N = ct.data.shape
    out = np.zeros_like(ct.data)
    for c in range(ncomp):
        src = np.ascontiguousarray(ct.data[c])
        dst = _u64((nl, N))
        lib().or_automorph(P(src), P(dst), N, g, P(params.qp(nl)), nl)
        out[c] = dst
    return Ct(out, ct.scale)


def keyswitch(params: Params, d: np.ndarray, key: np.ndarray) -> np.ndarray:
    """d: [nl][N] -> (u0, u1) as [2][nl][N]."""
    nl = d.shape[0]
    d = np.ascontiguousarray(d, dtype=np.uint64)
    out = _u64((2, nl, params.N))
    lib().or_keyswitch(P(d), nl, P(key), params.n_q, params.n_p, params.alpha, params.N, P(params.primes), P(out))
    return out


def add(params: Params, a: Ct, b: Ct) -> Ct:
    assert a.data.shape == b.data.shape
    ncomp, nl, N = a.data.shape
    out = np.zeros_like(a.data)
    lib().or_add(P(np.ascontiguousarray(a.data)), P(np.ascontiguousarray(b.data)), ncomp, nl, N,
                 P(params.qp(nl)), P(out))
    return Ct(out, a.scale)


def rotate_single(params: Params, keys: Keys, ct: Ct, r: int) -> Ct:
    """One key switch: left rotation by r (0 < r < S) via tau_g, g = 5^r mod 2N."""
    g = pow(5, r, 2 * params.N)
    t = automorph(params, ct, g)
    u = keyswitch(params, t.data[1], keys.rot_key(g))
    c0 = add(params, Ct(t.data[0:1].copy(), ct.scale), Ct(u[0:1].copy(), ct.scale)).data[0]
    return Ct(np.stack([c0, u[1]]), ct.scale)


def ext_moduli(params: Params, nl: int) -> np.ndarray:
    """Moduli of the extended basis at nl limbs: q_0 .. q_(nl-1), then p_0 .. p_(K-1)."""
    return np.ascontiguousarray(np.concatenate([params.primes[:nl], params.primes[params.n_q:]]))


def modup_digits(params: Params, d: np.ndarray) -> list:
    """ModUp of every digit of d ([nl][N], coefficient domain): the list over digits j of the
    extended polynomials ([nl + K][N]) that the key switch multiplies by the key's digit j."""
    nl = d.shape[0]
    d = np.ascontiguousarray(d, dtype=np.uint64)
    em = ext_moduli(params, nl)
    out = []
    for j in range(-(-nl // params.alpha)):
        lo, hi = j * params.alpha, min((j + 1) * params.alpha, nl)
        ext = _u64((nl + params.n_p, params.N))
        lib().or_modup(P(d), nl, lo, hi, P(em), params.n_p, params.N, P(ext))
        out.append(ext)
    return out


def keyswitch_digits(params: Params, exts: list, key: np.ndarray, nl: int, g: int = 1) -> np.ndarray:
    """Inner product and ModDown from given extended digits, each first mapped by tau_g (applied limb
    by limb over the extended basis): u_c = sum_j tau_g(ext_j) (*) key_(j,c); out_c = ModDown(u_c).
    With g = 1 and exts = modup_digits(d) this is keyswitch(d). -> [2][nl][N]."""
    N, nk = params.N, params.n_p
    nxt = nl + nk
    em = ext_moduli(params, nl)
    u = np.zeros((2, nxt, N), dtype=np.uint64)
    prod = _u64(N)
    for j, ext in enumerate(exts):
        if g != 1:
            eg = _u64((nxt, N))
            lib().or_automorph(P(np.ascontiguousarray(ext)), P(eg), N, g, P(em), nxt)
        else:
            eg = ext
        for c in range(2):
            for e in range(nxt):
                limb = e if e < nl else params.n_q + (e - nl)
                lib().or_poly_mul(P(np.ascontiguousarray(eg[e])), P(np.ascontiguousarray(key[j, c, limb])), P(prod),
                                  N, int(em[e]))
                u[c, e] = (u[c, e] + prod) % em[e]
    out = _u64((2, nl, N))
    for c in range(2):
        o = _u64((nl, N))
        lib().or_moddown(P(np.ascontiguousarray(u[c])), nl, P(em), nk, N, P(o))
        out[c] = o
    return out


def rotate_single_hoisted(params: Params, keys: Keys, ct: Ct, r: int, exts: list | None = None) -> Ct:
    """Left rotation by r with the automorphism moved past ModUp (hoisting): the key switch uses
    tau_g(ModUp_j(c1)), which agrees with ModUp_j(tau_g(c1)) modulo each digit's modulus (tau_g is a
    ring automorphism modulo every prime), so the result decrypts to the same rotation; ModUp of c1
    depends on ct alone and can serve every rotation of ct. `exts` = modup_digits(ct's c1) if known."""
    g = pow(5, r, 2 * params.N)
    nl = ct.data.shape[1]
    if exts is None:
        exts = modup_digits(params, ct.data[1])
    u = keyswitch_digits(params, exts, keys.rot_key(g), nl, g)
    t0 = automorph(params, Ct(ct.data[0:1].copy(), ct.scale), g)
    c0 = add(params, t0, Ct(u[0:1].copy(), ct.scale)).data[0]
    return Ct(np.stack([c0, u[1]]), ct.scale)


def rotate_hoisted(params: Params, keys: Keys, ct: Ct, r: int) -> Ct:
    """Rotation by r as its digit steps (as rotate), each step hoisted."""
    for step in rotation_steps(params, r):
        ct = rotate_single_hoisted(params, keys, ct, step)
    return ct


def rotation_steps(params: Params, r: int) -> list[int]:
    """Decomposition of a left rotation by r into key-switched steps r_t * 2^(b t), t ascending."""
    S = params.S
    r %= S
    if r == 0:
        return []
    b = params.rot_step_bits()
    steps = []
    for t in range(params.rot_digits):
        rt = (r >> (b * t)) & ((1 << b) - 1)
        if rt:
            steps.append(rt << (b * t))
    return steps


def rotate(params: Params, keys: Keys, ct: Ct, r: int) -> Ct:
    for step in rotation_steps(params, r):
        ct = rotate_single(params, keys, ct, step)
    return ct


def mult_relin(params: Params, keys: Keys, a: Ct, b: Ct) -> Ct:
    """EvalMult followed by Relinearize (key switch of d2 with the s^2 key)."""
    assert a.nl == b.nl
    nl = a.nl
    d = _u64((3, nl, params.N))
    lib().or_tensor(P(np.ascontiguousarray(a.data)), P(np.ascontiguousarray(b.data)), nl, params.N,
                    P(params.qp(nl)), P(d))
    u = keyswitch(params, d[2], keys.relin)
    scale = a.scale * b.scale
    return add(params, Ct(np.ascontiguousarray(d[0:2]), scale), Ct(u, scale))


def rescale(params: Params, ct: Ct) -> Ct:
    ncomp, nl, N = ct.data.shape
    out = _u64((ncomp, nl - 1, N))
    lib().or_rescale(P(np.ascontiguousarray(ct.data)), ncomp, nl, N, P(params.qp(nl)), P(out))
    return Ct(out, ct.scale / float(params.q[nl - 1]))


def base_mask(params: Params) -> np.ndarray:
    """Encoding of the one-hot vector e_0 at scale 2^mask_bits * q_(top-1)."""
    return encode(np.array([1.0]), params.delta_mask, params.N)


def mask(params: Params, p: int) -> np.ndarray:
    """One-hot mask at slot p: tau_(g_p) applied to the base mask, g_p = 5^((S - p) mod S) mod 2N."""
    g = pow(5, (params.S - p) % params.S, 2 * params.N)
    return automorph_signed(base_mask(params), g)


def mul_plain(params: Params, ct: Ct, m: np.ndarray, m_scale: float) -> Ct:
    ncomp, nl, N = ct.data.shape
    out = np.zeros_like(ct.data)
    lib().or_mul_plain(P(np.ascontiguousarray(ct.data)), ncomp, nl, P(np.ascontiguousarray(m, dtype=np.int64)), N,
                       P(params.qp(nl)), P(out))
    return Ct(out, ct.scale * m_scale)


def zero_ct(params: Params, nl: int, scale: float) -> Ct:
    return Ct(_u64((2, nl, params.N)), scale)
