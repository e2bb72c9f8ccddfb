// Modular arithmetic on 64-bit residues for gfx950 (and the host, for table construction).
//
// All moduli are odd primes below 2^61. Three multiplication forms are used:
//   * Shoup (Harvey 2014): a * w mod q for a fixed operand w with the precomputed
//     companion w' = floor(w 2^64 / q); valid for any a < 2^64, result in [0, q).
//   * Montgomery (R = 2^64): a * b * R^-1 mod q for a, b < q; operands kept in
//     Montgomery form (x R mod q) where one side is a stored constant (keys, masks).
//   * plain add/sub with one conditional correction (inputs in [0, q)).
// On gfx950 the 64x64->128 products lower to v_mad_u64_u32 chains.
#pragma once
#include <stdint.h>

#include <hip/hip_runtime.h>

#define FHE_HD __host__ __device__ __forceinline__

namespace fhe {

typedef unsigned __int128 u128;

FHE_HD uint64_t mulhi64(uint64_t a, uint64_t b) { return (uint64_t)(((u128)a * b) >> 64); }

FHE_HD uint64_t add_mod(uint64_t a, uint64_t b, uint64_t q) {
  uint64_t s = a + b;
  return s >= q ? s - q : s;
}

FHE_HD uint64_t sub_mod(uint64_t a, uint64_t b, uint64_t q) { return a >= b ? a - b : a + q - b; }

FHE_HD uint64_t neg_mod(uint64_t a, uint64_t q) { return a == 0 ? 0 : q - a; }

// a * w mod q up to one multiple of q: the result is in [0, 2q) for any a < 2^64 (Shoup's
// estimate floor(a wp / 2^64) of floor(a w / q) is low by at most one).
FHE_HD uint64_t shoup_mul_lazy(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
  return a * w - mulhi64(a, wp) * q;
}

// a * w mod q, w < q, wp = floor(w * 2^64 / q).
FHE_HD uint64_t shoup_mul(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
  uint64_t qh = mulhi64(a, wp);
  uint64_t r = a * w - qh * q;
  return r >= q ? r - q : r;
}

// a * b * 2^-64 mod q for a * b < q 2^64; qinv = q^-1 mod 2^64.
FHE_HD uint64_t mont_mul(uint64_t a, uint64_t b, uint64_t q, uint64_t qinv) {
  u128 x = (u128)a * b;
  uint64_t lo = (uint64_t)x, hi = (uint64_t)(x >> 64);
  uint64_t m = lo * qinv;
  uint64_t mh = mulhi64(m, q);
  return hi >= mh ? hi - mh : hi - mh + q;
}

// Host-side helpers for constant tables.
inline uint64_t mulmod_host(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a * b) % q); }

inline uint64_t powmod_host(uint64_t a, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  a %= q;
  while (e) {
    if (e & 1) r = mulmod_host(r, a, q);
    a = mulmod_host(a, a, q);
    e >>= 1;
  }
  return r;
}

inline uint64_t invmod_host(uint64_t a, uint64_t q) { return powmod_host(a, q - 2, q); }

inline uint64_t shoup_prep(uint64_t w, uint64_t q) { return (uint64_t)(((u128)w << 64) / q); }

// q^-1 mod 2^64 by Newton iteration (q odd).
inline uint64_t mont_qinv(uint64_t q) {
  uint64_t x = q;  // correct to 3 bits
  for (int i = 0; i < 6; ++i) x *= 2 - q * x;
  return x;
}

// x R mod q (Montgomery form), R = 2^64.
inline uint64_t to_mont_host(uint64_t x, uint64_t q) { return (uint64_t)(((u128)x << 64) % q); }

// Per-modulus constants kept in device memory.
struct ModInfo {
  uint64_t q;
  uint64_t qinv;  // q^-1 mod 2^64 (Montgomery)
  uint64_t r2;    // 2^128 mod q (to enter Montgomery form with one mont_mul)
  uint64_t n_inv, n_inv_shoup;
  uint64_t pad[3];
};

}  // namespace fhe
