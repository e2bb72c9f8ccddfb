// Host-side number theory, sampling, encoding and decoding.
#pragma once
#include <stdint.h>

#include <vector>

namespace fhe {

// Largest `count` primes p < 2^bits with p = 1 (mod m), descending; fewer if the range runs out.
std::vector<uint64_t> primes_below(int bits, int count, uint64_t m);
bool is_prime_u64(uint64_t n);
// A primitive 2N-th root of unity modulo q (q = 1 mod 2N).
uint64_t root_2n(uint32_t N, uint64_t q);

// Object tags of the sampling streams: stream state0 = seed ^ (tag * 0x9E3779B97F4A7C15).
// tag = kind << 56 | sub1 << 32 | sub2 << 16 | sub3.
enum TagKind : uint64_t {
  kTagSecret = 1,
  kTagRelinA = 2,
  kTagRelinE = 3,
  kTagEncA = 4,
  kTagEncE = 5,
  kTagRotA = 6,
  kTagRotE = 7,
};
inline uint64_t stream_tag(uint64_t kind, uint64_t sub1, uint64_t sub2, uint64_t sub3) {
  return (kind << 56) | (sub1 << 32) | (sub2 << 16) | sub3;
}

// SplitMix64 samplers (Steele, Lea, Flood 2014), one stream per (seed, tag).
void sample_uniform(uint64_t seed, uint64_t tag, uint64_t q, uint32_t N, uint64_t* out);
void sample_ternary(uint64_t seed, uint64_t tag, uint32_t N, int64_t* out);
void sample_gauss(uint64_t seed, uint64_t tag, uint32_t N, int64_t* out);  // sigma 3.2, |e| <= 19

// CKKS encoding of real slots z[0..nz) (nz <= N/2) at scale delta:
// m_k = round-half-away((delta * 2/N) * sum_{t asc, z_t != 0} z_t cos(pi ((5^t k) mod 2N) / N)).
void encode_real(const double* z, uint32_t nz, double delta, uint32_t N, int64_t* m);

// Decoding of all S slots of a real message polynomial m (centred coefficients as doubles):
// z_t = Re(m(zeta^(5^t))) / delta, by a complex FFT of length N.
void decode_all(const double* m, uint32_t N, double delta, double* z);

}  // namespace fhe
