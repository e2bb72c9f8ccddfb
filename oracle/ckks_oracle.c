/*
 * Plain CPU oracle for RNS-CKKS sparse x sparse ciphertext matmul.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library may include,
 * link or call this file; only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it. It shares no code, header,
 * table or constant generator with the HIP library: every definition below
 * is written out again from the mathematics, deliberately slow and plain.
 *
 * Conventions
 *   - Residues are uint64 in [0, q). Products use unsigned __int128 and '%'.
 *   - Polynomials live in the coefficient domain, one limb = N uint64.
 *     Multi-limb arrays are limb-major: a[limb * N + k].
 *   - The NTT here exists only to evaluate negacyclic products
 *     (Z_q[X]/(X^N + 1)); its output order is never observable outside.
 *
 * The CKKS definitions follow the paper's background on CKKS (Section 2.1:
 * packing, rescaling, relinearisation) and the operations its Algorithm 2
 * issues (EvalMult, Relinearize, Rescale, plaintext mask multiply,
 * EvalRotate, EvalAdd). Every choice the paper leaves open (sampling,
 * encoding rounding, base-conversion representatives, rescale rounding,
 * key-digit layout) is fixed by the readings listed in the design notes and
 * restated at each function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;
typedef __int128 i128;

/* ------------------------------------------------------------------ */
/* Scalar modular arithmetic: the definitions, written with '%'.       */
/* ------------------------------------------------------------------ */

uint64_t or_mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a * b) % q); }

uint64_t or_addmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + b) % q); }

uint64_t or_submod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + q - b) % q); }

uint64_t or_powmod(uint64_t a, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  a %= q;
  while (e) {
    if (e & 1) r = or_mulmod(r, a, q);
    a = or_mulmod(a, a, q);
    e >>= 1;
  }
  return r;
}

/* Inverse modulo a prime by Fermat's little theorem. */
uint64_t or_invmod_prime(uint64_t a, uint64_t q) { return or_powmod(a, q - 2, q); }

/* Signed integer -> residue in [0, q). */
static uint64_t from_signed(int64_t v, uint64_t q) {
  i128 r = (i128)v % (i128)q;
  if (r < 0) r += q;
  return (uint64_t)r;
}

/* Deterministic Miller-Rabin for n < 2^64 (the first twelve prime bases suffice). */
int or_is_prime(uint64_t n) {
  static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return 0;
  for (int i = 0; i < 12; ++i) {
    if (n == bases[i]) return 1;
    if (n % bases[i] == 0) return 0;
  }
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  for (int i = 0; i < 12; ++i) {
    uint64_t x = or_powmod(bases[i], d, n);
    if (x == 1 || x == n - 1) continue;
    int composite = 1;
    for (int r = 1; r < s; ++r) {
      x = or_mulmod(x, x, n);
      if (x == n - 1) { composite = 0; break; }
    }
    if (composite) return 0;
  }
  return 1;
}

/* The `count` largest primes q < 2^bits with q = 1 (mod m), in descending order. */
int or_find_primes(int bits, int count, uint64_t m, uint64_t* out) {
  uint64_t top = (bits >= 64) ? UINT64_MAX : (((uint64_t)1 << bits) - 1);
  uint64_t k = (top - 1) / m;  /* largest k with k*m + 1 <= top */
  int found = 0;
  while (found < count && k > 0) {
    uint64_t x = k * m + 1;
    if (or_is_prime(x)) out[found++] = x;
    --k;
  }
  return found;
}

/* A primitive 2N-th root of unity mod q (q = 1 mod 2N, N a power of two):
 * psi = x^((q-1)/2N) for the first x = 2, 3, ... with psi^N = -1. */
uint64_t or_primitive_2n_root(uint64_t N, uint64_t q) {
  for (uint64_t x = 2;; ++x) {
    uint64_t psi = or_powmod(x, (q - 1) / (2 * N), q);
    if (or_powmod(psi, N, q) == q - 1) return psi;
  }
}

/* ------------------------------------------------------------------ */
/* Negacyclic products.                                                */
/* ------------------------------------------------------------------ */

/* Schoolbook product in Z_q[X]/(X^N+1): the definition itself. O(N^2). */
void or_poly_mul_schoolbook(const uint64_t* a, const uint64_t* b, uint64_t* out, uint64_t N, uint64_t q) {
  for (uint64_t k = 0; k < N; ++k) out[k] = 0;
  for (uint64_t i = 0; i < N; ++i)
    for (uint64_t j = 0; j < N; ++j) {
      uint64_t p = or_mulmod(a[i], b[j], q);
      uint64_t idx = i + j;
      if (idx < N) out[idx] = or_addmod(out[idx], p, q);
      else out[idx - N] = or_submod(out[idx - N], p, q); /* X^N = -1 */
    }
}

static uint64_t bit_reverse(uint64_t x, int bits) {
  uint64_t r = 0;
  for (int i = 0; i < bits; ++i) { r = (r << 1) | (x & 1); x >>= 1; }
  return r;
}

/* Textbook iterative radix-2 cyclic DFT over Z_q with root w (order N):
 * A[i] = sum_k a[k] w^(i k). Bit-reversal permutation, then butterflies. */
static void cyclic_dft(uint64_t* a, uint64_t N, uint64_t q, uint64_t w) {
  int logn = 0;
  while (((uint64_t)1 << logn) < N) ++logn;
  for (uint64_t i = 0; i < N; ++i) {
    uint64_t j = bit_reverse(i, logn);
    if (i < j) { uint64_t t = a[i]; a[i] = a[j]; a[j] = t; }
  }
  for (uint64_t len = 2; len <= N; len <<= 1) {
    uint64_t wl = or_powmod(w, N / len, q); /* primitive len-th root */
    for (uint64_t start = 0; start < N; start += len) {
      uint64_t wj = 1;
      for (uint64_t j = 0; j < len / 2; ++j) {
        uint64_t u = a[start + j];
        uint64_t v = or_mulmod(a[start + j + len / 2], wj, q);
        a[start + j] = or_addmod(u, v, q);
        a[start + j + len / 2] = or_submod(u, v, q);
        wj = or_mulmod(wj, wl, q);
      }
    }
  }
}

/* Forward negacyclic transform: A[i] = a(psi^(2i+1)) = sum_k (a_k psi^k) (psi^2)^(ik). */
void or_ntt_forward(uint64_t* a, uint64_t N, uint64_t q) {
  uint64_t psi = or_primitive_2n_root(N, q);
  uint64_t pk = 1;
  for (uint64_t k = 0; k < N; ++k) { a[k] = or_mulmod(a[k], pk, q); pk = or_mulmod(pk, psi, q); }
  cyclic_dft(a, N, q, or_mulmod(psi, psi, q));
}

/* Inverse of or_ntt_forward: a_k = N^-1 psi^-k sum_i A_i (psi^-2)^(ik). */
void or_ntt_inverse(uint64_t* a, uint64_t N, uint64_t q) {
  uint64_t psi = or_primitive_2n_root(N, q);
  uint64_t psi_inv = or_invmod_prime(psi, q);
  cyclic_dft(a, N, q, or_mulmod(psi_inv, psi_inv, q));
  uint64_t n_inv = or_invmod_prime(N % q, q);
  uint64_t pk = n_inv;
  for (uint64_t k = 0; k < N; ++k) { a[k] = or_mulmod(a[k], pk, q); pk = or_mulmod(pk, psi_inv, q); }
}

/* Negacyclic product through the transform (a library step, pinned to the schoolbook). */
void or_poly_mul(const uint64_t* a, const uint64_t* b, uint64_t* out, uint64_t N, uint64_t q) {
  uint64_t* fa = (uint64_t*)malloc(N * 8);
  uint64_t* fb = (uint64_t*)malloc(N * 8);
  memcpy(fa, a, N * 8);
  memcpy(fb, b, N * 8);
  or_ntt_forward(fa, N, q);
  or_ntt_forward(fb, N, q);
  for (uint64_t i = 0; i < N; ++i) fa[i] = or_mulmod(fa[i], fb[i], q);
  or_ntt_inverse(fa, N, q);
  memcpy(out, fa, N * 8);
  free(fa);
  free(fb);
}

/* ------------------------------------------------------------------ */
/* Sampling: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014).             */
/* One stream per sampled object: state0 = seed XOR tag * 0x9E3779B97F4A7C15. */
/* ------------------------------------------------------------------ */

static uint64_t splitmix_next(uint64_t* s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

uint64_t or_splitmix_first(uint64_t seed, uint64_t tag, uint64_t count, uint64_t* out) {
  uint64_t s = seed ^ (tag * 0x9E3779B97F4A7C15ULL);
  for (uint64_t i = 0; i < count; ++i) out[i] = splitmix_next(&s);
  return s;
}

/* Uniform residues mod q, coefficient k = 0..N-1: draw x, accept if x < floor(2^64/q)*q, return x mod q. */
void or_sample_uniform(uint64_t seed, uint64_t tag, uint64_t q, uint64_t N, uint64_t* out) {
  uint64_t s = seed ^ (tag * 0x9E3779B97F4A7C15ULL);
  uint64_t bound = (uint64_t)((((u128)1 << 64) / q) * q);
  for (uint64_t k = 0; k < N; ++k) {
    uint64_t x;
    do { x = splitmix_next(&s); } while (x >= bound);
    out[k] = x % q;
  }
}

/* Uniform ternary: draw x, accept if x < floor(2^64/3)*3; x mod 3 = 0 -> 0, 1 -> +1, 2 -> -1. */
void or_sample_ternary(uint64_t seed, uint64_t tag, uint64_t N, int64_t* out) {
  uint64_t s = seed ^ (tag * 0x9E3779B97F4A7C15ULL);
  uint64_t bound = (UINT64_MAX / 3) * 3;
  for (uint64_t k = 0; k < N; ++k) {
    uint64_t x;
    do { x = splitmix_next(&s); } while (x >= bound);
    uint64_t r = x % 3;
    out[k] = (r == 0) ? 0 : (r == 1 ? 1 : -1);
  }
}

/* Rounded Gaussian: Box-Muller (cosine branch) on two 53-bit uniforms,
 * u1 = ((x1 >> 11) + 1) 2^-53 in (0,1], u2 = (x2 >> 11) 2^-53 in [0,1),
 * v = sigma * (sqrt(-2 ln u1) * cos(2 pi u2)), e = round-half-away(v),
 * redrawn while |e| > bound. */
void or_sample_gauss(uint64_t seed, uint64_t tag, uint64_t N, double sigma, int64_t bound, int64_t* out) {
  uint64_t s = seed ^ (tag * 0x9E3779B97F4A7C15ULL);
  const double two_pi = 6.283185307179586476925286766559;
  const double inv53 = 1.0 / 9007199254740992.0;
  for (uint64_t k = 0; k < N; ++k) {
    int64_t e;
    do {
      uint64_t x1 = splitmix_next(&s);
      uint64_t x2 = splitmix_next(&s);
      double u1 = (double)((x1 >> 11) + 1) * inv53;
      double u2 = (double)(x2 >> 11) * inv53;
      double r = sqrt(-2.0 * log(u1));
      double c = cos(two_pi * u2);
      double v = sigma * (r * c);
      e = (int64_t)round(v);
    } while (e > bound || e < -bound);
    out[k] = e;
  }
}

/* ------------------------------------------------------------------ */
/* Encoding / decoding (canonical embedding, slot t <-> zeta^(5^t),    */
/* zeta = exp(i pi / N), S = N/2 slots, real slot values).             */
/* ------------------------------------------------------------------ */

/* cos(pi j / N) for j in [0, 2N), evaluated as cos((pi * j) / N). */
static double cos_tab(uint64_t j, uint64_t N) {
  const double pi = 3.14159265358979323846264338327950288;
  return cos((pi * (double)j) / (double)N);
}

/* m_k = round-half-away( (delta * (2/N)) * acc_k ),
 * acc_k = sum over t ascending with z_t != 0 of z_t * cos(pi ((5^t k) mod 2N) / N),
 * each step acc = acc + z_t * c with two roundings (no fused multiply-add). */
void or_encode(const double* z, uint64_t nz, double delta, uint64_t N, int64_t* m) {
  uint64_t two_n = 2 * N;
  double* tab = (double*)malloc(two_n * sizeof(double));
  for (uint64_t j = 0; j < two_n; ++j) tab[j] = cos_tab(j, N);
  uint64_t* g = (uint64_t*)malloc((nz ? nz : 1) * 8);
  uint64_t gt = 1;
  for (uint64_t t = 0; t < nz; ++t) { g[t] = gt; gt = (gt * 5) % two_n; }
  double scale = delta * (2.0 / (double)N);
  for (uint64_t k = 0; k < N; ++k) {
    double acc = 0.0;
    for (uint64_t t = 0; t < nz; ++t) {
      if (z[t] == 0.0) continue;
      double p = z[t] * tab[(g[t] * k) % two_n];
      acc = acc + p;
    }
    double v = scale * acc;
    m[k] = (int64_t)round(v);
  }
  free(tab);
  free(g);
}

/* Decode selected slots of a real message polynomial given as doubles:
 * z_t = (sum_k m_k cos(pi ((5^t k) mod 2N) / N)) / delta. Plain O(N) per slot. */
void or_decode_slots(const double* m, uint64_t N, double delta, const int64_t* slots, uint64_t nslots, double* out) {
  uint64_t two_n = 2 * N;
  double* tab = (double*)malloc(two_n * sizeof(double));
  for (uint64_t j = 0; j < two_n; ++j) tab[j] = cos_tab(j, N);
  for (uint64_t s = 0; s < nslots; ++s) {
    uint64_t g = or_powmod(5, (uint64_t)slots[s], two_n);
    double acc = 0.0;
    for (uint64_t k = 0; k < N; ++k) acc += m[k] * tab[(g * k) % two_n];
    out[s] = acc / delta;
  }
  free(tab);
}

/* ------------------------------------------------------------------ */
/* Ring-level helpers over several limbs.                              */
/* ------------------------------------------------------------------ */

/* Reduce a signed small polynomial into limbs: out[i*N+k] = v_k mod primes[i]. */
void or_signed_to_limbs(const int64_t* v, uint64_t N, const uint64_t* primes, uint64_t nlimbs, uint64_t* out) {
  for (uint64_t i = 0; i < nlimbs; ++i)
    for (uint64_t k = 0; k < N; ++k) out[i * N + k] = from_signed(v[k], primes[i]);
}

/* Automorphism tau_g: X^k -> X^(k g mod 2N), with X^N = -1 (g odd). */
void or_automorph(const uint64_t* in, uint64_t* out, uint64_t N, uint64_t g, const uint64_t* primes, uint64_t nlimbs) {
  uint64_t two_n = 2 * N;
  for (uint64_t i = 0; i < nlimbs; ++i) {
    uint64_t q = primes[i];
    for (uint64_t k = 0; k < N; ++k) {
      uint64_t idx = (k * g) % two_n;
      uint64_t v = in[i * N + k];
      if (idx < N) out[i * N + idx] = v;
      else out[i * N + (idx - N)] = (v == 0) ? 0 : q - v;
    }
  }
}

/* Same map on a signed integer polynomial. */
void or_automorph_signed(const int64_t* in, int64_t* out, uint64_t N, uint64_t g) {
  uint64_t two_n = 2 * N;
  for (uint64_t k = 0; k < N; ++k) {
    uint64_t idx = (k * g) % two_n;
    if (idx < N) out[idx] = in[k];
    else out[idx - N] = -in[k];
  }
}

/* ------------------------------------------------------------------ */
/* Key material. A switching key for target secret s' has, for each    */
/* digit j of the top-level Q basis, a pair (b_j, a_j) over all limbs   */
/* q_0..q_L, p_0..p_{K-1}:                                              */
/*   a_j uniform (stream tag kind 2/6),                                 */
/*   b_j = -a_j s + e_j + [q_i in digit j] (P mod q_i) s'  (mod q_i),   */
/*   b_j = -a_j s + e_j                                    (mod p_k).   */
/* Layout: key[((j * 2 + c) * nall + limb) * N + k], c = 0 for b, 1 for a. */
/* ------------------------------------------------------------------ */

/* tag = kind << 56 | sub1 << 32 | sub2 << 16 | sub3 */
static uint64_t make_tag(uint64_t kind, uint64_t sub1, uint64_t sub2, uint64_t sub3) {
  return (kind << 56) | (sub1 << 32) | (sub2 << 16) | sub3;
}

uint64_t or_tag(uint64_t kind, uint64_t sub1, uint64_t sub2, uint64_t sub3) { return make_tag(kind, sub1, sub2, sub3); }

/* s: secret (ternary, int64[N]). sprime: target secret as residues on all limbs, [nall][N].
 * primes: q_0..q_L then p_0..p_{K-1} (nall = L+1+K). key_id: 0 relinearisation, g rotation. */
void or_keygen_switch(uint64_t seed, uint64_t key_id, const int64_t* s, const uint64_t* sprime, uint64_t N,
                      const uint64_t* primes, uint64_t nq, uint64_t nk, uint64_t alpha, uint64_t* key) {
  uint64_t nall = nq + nk;
  uint64_t beta = (nq + alpha - 1) / alpha;
  uint64_t* a = (uint64_t*)malloc(N * 8);
  uint64_t* slimb = (uint64_t*)malloc(N * 8);
  uint64_t* as = (uint64_t*)malloc(N * 8);
  int64_t* e = (int64_t*)malloc(N * 8);
  uint64_t kind_a = key_id == 0 ? 2 : 6, kind_e = key_id == 0 ? 3 : 7;
  for (uint64_t j = 0; j < beta; ++j) {
    or_sample_gauss(seed, make_tag(kind_e, key_id, j, 0), N, 3.2, 19, e);
    for (uint64_t i = 0; i < nall; ++i) {
      uint64_t q = primes[i];
      uint64_t* bj = key + ((j * 2 + 0) * nall + i) * N;
      uint64_t* aj = key + ((j * 2 + 1) * nall + i) * N;
      or_sample_uniform(seed, make_tag(kind_a, key_id, j, i), q, N, a);
      for (uint64_t k = 0; k < N; ++k) slimb[k] = from_signed(s[k], q);
      or_poly_mul(a, slimb, as, N, q);
      int in_digit = (i < nq) && (i / alpha == j);
      uint64_t pmod = 1;
      if (in_digit)
        for (uint64_t t = 0; t < nk; ++t) pmod = or_mulmod(pmod, primes[nq + t] % q, q);
      for (uint64_t k = 0; k < N; ++k) {
        uint64_t v = or_submod(from_signed(e[k], q), as[k], q);
        if (in_digit) v = or_addmod(v, or_mulmod(pmod, sprime[i * N + k], q), q);
        bj[k] = v;
        aj[k] = a[k];
      }
    }
  }
  free(a);
  free(slimb);
  free(as);
  free(e);
}

/* Secret-key encryption at the top level (limbs q_0..q_{nq-1}):
 * c1 = a (uniform, tag kind 4), c0 = -a s + e + m (e: tag kind 5). ct = [2][nq][N]. */
void or_encrypt(uint64_t seed, uint64_t chunk, const int64_t* m, const int64_t* s, uint64_t N,
                const uint64_t* primes, uint64_t nq, uint64_t* ct) {
  uint64_t* a = (uint64_t*)malloc(N * 8);
  uint64_t* slimb = (uint64_t*)malloc(N * 8);
  uint64_t* as = (uint64_t*)malloc(N * 8);
  int64_t* e = (int64_t*)malloc(N * 8);
  or_sample_gauss(seed, make_tag(5, chunk, 0, 0), N, 3.2, 19, e);
  for (uint64_t i = 0; i < nq; ++i) {
    uint64_t q = primes[i];
    or_sample_uniform(seed, make_tag(4, chunk, 0, i), q, N, a);
    for (uint64_t k = 0; k < N; ++k) slimb[k] = from_signed(s[k], q);
    or_poly_mul(a, slimb, as, N, q);
    for (uint64_t k = 0; k < N; ++k) {
      uint64_t v = or_submod(from_signed(e[k], q), as[k], q);
      ct[(0 * nq + i) * N + k] = or_addmod(v, from_signed(m[k], q), q);
      ct[(1 * nq + i) * N + k] = a[k];
    }
  }
  free(a);
  free(slimb);
  free(as);
  free(e);
}

/* Decryption on the first `nl` limbs: out[i] = c0_i + c1_i * s (mod q_i).
 * ct holds [2][nlimbs][N]. */
void or_decrypt_limbs(const uint64_t* ct, uint64_t nlimbs, uint64_t nl, const int64_t* s, uint64_t N,
                      const uint64_t* primes, uint64_t* out) {
  uint64_t* slimb = (uint64_t*)malloc(N * 8);
  uint64_t* cs = (uint64_t*)malloc(N * 8);
  for (uint64_t i = 0; i < nl; ++i) {
    uint64_t q = primes[i];
    for (uint64_t k = 0; k < N; ++k) slimb[k] = from_signed(s[k], q);
    or_poly_mul(ct + (1 * nlimbs + i) * N, slimb, cs, N, q);
    for (uint64_t k = 0; k < N; ++k) out[i * N + k] = or_addmod(ct[(0 * nlimbs + i) * N + k], cs[k], q);
  }
  free(slimb);
  free(cs);
}

/* Centred CRT of two limbs: x = the unique value in (-q0 q1 / 2, q0 q1 / 2] congruent to
 * (r0 mod q0, r1 mod q1); returned as a double. */
void or_crt2_centered(const uint64_t* r0, const uint64_t* r1, uint64_t N, uint64_t q0, uint64_t q1, double* out) {
  u128 Q = (u128)q0 * q1;
  uint64_t q0_inv_mod_q1 = or_invmod_prime(q0 % q1, q1);
  for (uint64_t k = 0; k < N; ++k) {
    /* x = r0 + q0 * ((r1 - r0) q0^-1 mod q1) */
    uint64_t t = or_mulmod(or_submod(r1[k], r0[k] % q1, q1), q0_inv_mod_q1, q1);
    u128 x = (u128)r0[k] + (u128)q0 * t;
    i128 v = (x > Q / 2) ? (i128)x - (i128)Q : (i128)x;
    out[k] = (double)v;
  }
}

/* ------------------------------------------------------------------ */
/* Key switching: ModUp per digit, inner product with the key, ModDown. */
/* ------------------------------------------------------------------ */

/* ModUp of one digit (fast base conversion, no correction term).
 * d: [nl][N] coefficient-domain limbs q_0..q_{nl-1}. The digit is q_lo..q_{hi-1}.
 * y_i = [d_i * (Dhat_i^-1 mod q_i)]_{q_i}, Dhat_i = prod of the other digit primes;
 * for every modulus t of the extended basis (q_0..q_{nl-1}, then the nk P primes)
 * outside the digit: ext_t = sum_i y_i * (Dhat_i mod t) mod t; inside: ext_t = d_t.
 * ext_moduli: [nl + nk]; ext: [nl + nk][N]. */
void or_modup(const uint64_t* d, uint64_t nl, uint64_t lo, uint64_t hi, const uint64_t* ext_moduli, uint64_t nk,
              uint64_t N, uint64_t* ext) {
  uint64_t next = nl + nk;
  uint64_t* y = (uint64_t*)malloc((hi - lo) * N * 8);
  for (uint64_t i = lo; i < hi; ++i) {
    uint64_t qi = ext_moduli[i];
    uint64_t dhat = 1;
    for (uint64_t i2 = lo; i2 < hi; ++i2)
      if (i2 != i) dhat = or_mulmod(dhat, ext_moduli[i2] % qi, qi);
    uint64_t dhat_inv = or_invmod_prime(dhat, qi);
    for (uint64_t k = 0; k < N; ++k) y[(i - lo) * N + k] = or_mulmod(d[i * N + k], dhat_inv, qi);
  }
  for (uint64_t e = 0; e < next; ++e) {
    uint64_t t = ext_moduli[e];
    if (e >= lo && e < hi) { memcpy(ext + e * N, d + e * N, N * 8); continue; }
    for (uint64_t k = 0; k < N; ++k) ext[e * N + k] = 0;
    for (uint64_t i = lo; i < hi; ++i) {
      uint64_t dhat_t = 1; /* Dhat_i mod t */
      for (uint64_t i2 = lo; i2 < hi; ++i2)
        if (i2 != i) dhat_t = or_mulmod(dhat_t, ext_moduli[i2] % t, t);
      for (uint64_t k = 0; k < N; ++k)
        ext[e * N + k] = or_addmod(ext[e * N + k], or_mulmod(y[(i - lo) * N + k] % t, dhat_t, t), t);
    }
  }
  free(y);
}

/* ModDown of one polynomial u over (q_0..q_{nl-1}, p_0..p_{nk-1}) to q_0..q_{nl-1}:
 * z_k = [u_{p_k} (P/p_k)^-1]_{p_k}, taken as the centred representative (z_k - p_k when
 * z_k > (p_k - 1)/2); conv_i = sum_k z_k (P/p_k mod q_i) mod q_i; out_i = (u_{q_i} - conv_i) P^-1 mod q_i.
 * Centring makes the rounding error of the division by P zero-mean; with [0, p_k) representatives it
 * has mean (K-1)/2 per coefficient, which adds the same slot pattern at every key switch.
 * ext_moduli: [nl + nk]; u: [nl+nk][N]; out: [nl][N]. */
void or_moddown(const uint64_t* u, uint64_t nl, const uint64_t* ext_moduli, uint64_t nk, uint64_t N, uint64_t* out) {
  const uint64_t* pm = ext_moduli + nl;
  uint64_t* z = (uint64_t*)malloc(nk * N * 8);
  for (uint64_t kk = 0; kk < nk; ++kk) {
    uint64_t pk = pm[kk];
    uint64_t phat = 1;
    for (uint64_t k2 = 0; k2 < nk; ++k2)
      if (k2 != kk) phat = or_mulmod(phat, pm[k2] % pk, pk);
    uint64_t phat_inv = or_invmod_prime(phat, pk);
    for (uint64_t k = 0; k < N; ++k) z[kk * N + k] = or_mulmod(u[(nl + kk) * N + k], phat_inv, pk);
  }
  for (uint64_t i = 0; i < nl; ++i) {
    uint64_t qi = ext_moduli[i];
    uint64_t pinv = 1;
    for (uint64_t kk = 0; kk < nk; ++kk) pinv = or_mulmod(pinv, pm[kk] % qi, qi);
    pinv = or_invmod_prime(pinv, qi);
    for (uint64_t k = 0; k < N; ++k) {
      uint64_t conv = 0;
      for (uint64_t kk = 0; kk < nk; ++kk) {
        uint64_t phat_q = 1; /* (P / p_kk) mod q_i */
        for (uint64_t k2 = 0; k2 < nk; ++k2)
          if (k2 != kk) phat_q = or_mulmod(phat_q, pm[k2] % qi, qi);
        uint64_t pk = pm[kk], zk = z[kk * N + k];
        int64_t zc = (zk > (pk - 1) / 2) ? (int64_t)zk - (int64_t)pk : (int64_t)zk;
        conv = or_addmod(conv, or_mulmod(from_signed(zc, qi), phat_q, qi), qi);
      }
      out[i * N + k] = or_mulmod(or_submod(u[i * N + k], conv, qi), pinv, qi);
    }
  }
  free(z);
}

/* KS_{s'}(d) at level nl - 1.
 * d: [nl][N] (coefficient domain). key: as written by or_keygen_switch with nq_top limbs
 * of Q. primes: q_0..q_{nq_top-1}, p_0..p_{nk-1}. out: [2][nl][N].
 * u_c = sum over digits j of ModUp_j(d) (*) key_{j,c} on the extended basis; out_c = ModDown(u_c). */
void or_keyswitch(const uint64_t* d, uint64_t nl, const uint64_t* key, uint64_t nq_top, uint64_t nk, uint64_t alpha,
                  uint64_t N, const uint64_t* primes, uint64_t* out) {
  uint64_t nall_key = nq_top + nk;
  uint64_t next = nl + nk;
  uint64_t beta = (nl + alpha - 1) / alpha;
  uint64_t* ext_mod = (uint64_t*)malloc(next * 8);
  uint64_t* ext = (uint64_t*)malloc(next * N * 8);
  uint64_t* u = (uint64_t*)calloc(2 * next * N, 8);
  uint64_t* prod = (uint64_t*)malloc(N * 8);
  for (uint64_t e = 0; e < next; ++e) ext_mod[e] = e < nl ? primes[e] : primes[nq_top + (e - nl)];
  for (uint64_t j = 0; j < beta; ++j) {
    uint64_t lo = j * alpha, hi = (j + 1) * alpha < nl ? (j + 1) * alpha : nl;
    or_modup(d, nl, lo, hi, ext_mod, nk, N, ext);
    for (uint64_t c = 0; c < 2; ++c)
      for (uint64_t e = 0; e < next; ++e) {
        uint64_t t = ext_mod[e];
        uint64_t key_limb = e < nl ? e : nq_top + (e - nl);
        const uint64_t* kp = key + ((j * 2 + c) * nall_key + key_limb) * N;
        or_poly_mul(ext + e * N, kp, prod, N, t);
        for (uint64_t k = 0; k < N; ++k) u[(c * next + e) * N + k] = or_addmod(u[(c * next + e) * N + k], prod[k], t);
      }
  }
  for (uint64_t c = 0; c < 2; ++c) or_moddown(u + c * next * N, nl, ext_mod, nk, N, out + c * nl * N);
  free(ext_mod);
  free(ext);
  free(u);
  free(prod);
}

/* ------------------------------------------------------------------ */
/* Rescale: drop the last limb q_l with nearest rounding.               */
/* v = c_l[k]; v' = v - q_l if v > (q_l - 1) / 2 else v;                */
/* c_i'[k] = (c_i[k] - (v' mod q_i)) * (q_l^-1 mod q_i) mod q_i.        */
/* in: [ncomp][nl][N] -> out: [ncomp][nl-1][N].                          */
/* ------------------------------------------------------------------ */
void or_rescale(const uint64_t* in, uint64_t ncomp, uint64_t nl, uint64_t N, const uint64_t* primes, uint64_t* out) {
  uint64_t ql = primes[nl - 1];
  for (uint64_t c = 0; c < ncomp; ++c)
    for (uint64_t i = 0; i + 1 < nl; ++i) {
      uint64_t qi = primes[i];
      uint64_t ql_inv = or_invmod_prime(ql % qi, qi);
      for (uint64_t k = 0; k < N; ++k) {
        uint64_t v = in[(c * nl + nl - 1) * N + k];
        int64_t vs = (v > (ql - 1) / 2) ? (int64_t)v - (int64_t)ql : (int64_t)v;
        uint64_t vm = from_signed(vs, qi);
        out[(c * (nl - 1) + i) * N + k] = or_mulmod(or_submod(in[(c * nl + i) * N + k], vm, qi), ql_inv, qi);
      }
    }
}

/* Ciphertext tensor product (a0, a1) x (b0, b1) -> (a0 b0, a0 b1 + a1 b0, a1 b1). a, b: [2][nl][N]; out: [3][nl][N]. */
void or_tensor(const uint64_t* a, const uint64_t* b, uint64_t nl, uint64_t N, const uint64_t* primes, uint64_t* out) {
  uint64_t* t = (uint64_t*)malloc(N * 8);
  for (uint64_t i = 0; i < nl; ++i) {
    uint64_t q = primes[i];
    const uint64_t *a0 = a + i * N, *a1 = a + (nl + i) * N, *b0 = b + i * N, *b1 = b + (nl + i) * N;
    or_poly_mul(a0, b0, out + i * N, N, q);
    or_poly_mul(a1, b1, out + (2 * nl + i) * N, N, q);
    or_poly_mul(a0, b1, out + (nl + i) * N, N, q);
    or_poly_mul(a1, b0, t, N, q);
    for (uint64_t k = 0; k < N; ++k) out[(nl + i) * N + k] = or_addmod(out[(nl + i) * N + k], t[k], q);
  }
  free(t);
}

/* Plaintext multiply by an integer polynomial m: each component and limb times (m mod q_i). */
void or_mul_plain(const uint64_t* in, uint64_t ncomp, uint64_t nl, const int64_t* m, uint64_t N, const uint64_t* primes,
                  uint64_t* out) {
  uint64_t* ml = (uint64_t*)malloc(N * 8);
  for (uint64_t i = 0; i < nl; ++i) {
    uint64_t q = primes[i];
    for (uint64_t k = 0; k < N; ++k) ml[k] = from_signed(m[k], q);
    for (uint64_t c = 0; c < ncomp; ++c) or_poly_mul(in + (c * nl + i) * N, ml, out + (c * nl + i) * N, N, q);
  }
  free(ml);
}

/* out = a + b limb-wise. */
void or_add(const uint64_t* a, const uint64_t* b, uint64_t ncomp, uint64_t nl, uint64_t N, const uint64_t* primes,
            uint64_t* out) {
  for (uint64_t c = 0; c < ncomp; ++c)
    for (uint64_t i = 0; i < nl; ++i)
      for (uint64_t k = 0; k < N; ++k)
        out[(c * nl + i) * N + k] = or_addmod(a[(c * nl + i) * N + k], b[(c * nl + i) * N + k], primes[i]);
}
