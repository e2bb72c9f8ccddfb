// Host-side number theory, SplitMix64 sampling, CKKS encoding and FFT decoding.
// Compiled without floating-point contraction so that encoding and sampling evaluate exactly the
// operation sequences written here.
#include "host_math.h"

#include <cmath>
#include <complex>
#include <thread>

namespace fhe {

namespace {

typedef unsigned __int128 u128;

uint64_t mm(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }

uint64_t pw(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  for (; e; e >>= 1) {
    if (e & 1) r = mm(r, a, m);
    a = mm(a, a, m);
  }
  return r;
}

struct SplitMix64 {
  uint64_t s;
  SplitMix64(uint64_t seed, uint64_t tag) : s(seed ^ (tag * 0x9E3779B97F4A7C15ULL)) {}
  uint64_t next() {
    s += 0x9E3779B97F4A7C15ULL;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
  }
};

unsigned worker_count() {
  unsigned n = std::thread::hardware_concurrency();
  if (n == 0) n = 1;
  if (n > 16) n = 16;
  return n;
}

template <class F>
void parallel_for(uint32_t n, F f) {
  unsigned w = worker_count();
  if (w <= 1 || n < 1024) {
    f(0u, n);
    return;
  }
  std::vector<std::thread> th;
  uint32_t step = (n + w - 1) / w;
  for (unsigned i = 0; i < w; ++i) {
    uint32_t lo = i * step, hi = std::min<uint32_t>(n, lo + step);
    if (lo >= hi) break;
    th.emplace_back([=] { f(lo, hi); });
  }
  for (auto& t : th) t.join();
}

}  // namespace

// Deterministic Miller-Rabin for 64-bit integers (Sinclair's seven bases).
bool is_prime_u64(uint64_t n) {
  if (n < 2) return false;
  static const uint64_t small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (uint64_t p : small) {
    if (n % p == 0) return n == p;
  }
  uint64_t d = n - 1;
  int r = 0;
  while (!(d & 1)) {
    d >>= 1;
    ++r;
  }
  static const uint64_t bases[] = {2, 325, 9375, 28178, 450775, 9780504, 1795265022};
  for (uint64_t a : bases) {
    uint64_t x = pw(a % n, d, n);
    if (a % n == 0 || x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < r && comp; ++i) {
      x = mm(x, x, n);
      if (x == n - 1) comp = false;
    }
    if (comp) return false;
  }
  return true;
}

std::vector<uint64_t> primes_below(int bits, int count, uint64_t m) {
  std::vector<uint64_t> out;
  uint64_t limit = bits >= 64 ? ~0ULL : ((1ULL << bits) - 1);
  for (uint64_t c = (limit - 1) / m; c > 0 && (int)out.size() < count; --c) {
    uint64_t x = c * m + 1;
    if (is_prime_u64(x)) out.push_back(x);
  }
  return out;
}

uint64_t root_2n(uint32_t N, uint64_t q) {
  for (uint64_t g = 2;; ++g) {
    uint64_t r = pw(g, (q - 1) / (2 * (uint64_t)N), q);
    if (pw(r, N, q) == q - 1) return r;
  }
}

void sample_uniform(uint64_t seed, uint64_t tag, uint64_t q, uint32_t N, uint64_t* out) {
  SplitMix64 g(seed, tag);
  const uint64_t accept = (uint64_t)((((u128)1 << 64) / q) * q);
  for (uint32_t k = 0; k < N; ++k) {
    uint64_t x = g.next();
    while (x >= accept) x = g.next();
    out[k] = x % q;
  }
}

void sample_ternary(uint64_t seed, uint64_t tag, uint32_t N, int64_t* out) {
  SplitMix64 g(seed, tag);
  const uint64_t accept = (~0ULL / 3) * 3;
  static const int64_t map3[3] = {0, 1, -1};
  for (uint32_t k = 0; k < N; ++k) {
    uint64_t x = g.next();
    while (x >= accept) x = g.next();
    out[k] = map3[x % 3];
  }
}

void sample_gauss(uint64_t seed, uint64_t tag, uint32_t N, int64_t* out) {
  SplitMix64 g(seed, tag);
  const double two_pi = 6.283185307179586476925286766559;
  const double ulp53 = 1.0 / 9007199254740992.0;
  const double sigma = 3.2;
  for (uint32_t k = 0; k < N; ++k) {
    int64_t v;
    for (;;) {
      const uint64_t x1 = g.next(), x2 = g.next();
      const double u1 = (double)((x1 >> 11) + 1) * ulp53;
      const double u2 = (double)(x2 >> 11) * ulp53;
      const double radius = std::sqrt(-2.0 * std::log(u1));
      const double c = std::cos(two_pi * u2);
      v = (int64_t)std::round(sigma * (radius * c));
      if (v <= 19 && v >= -19) break;
    }
    out[k] = v;
  }
}

void encode_real(const double* z, uint32_t nz, double delta, uint32_t N, int64_t* m) {
  const uint32_t two_n = 2 * N;
  const double pi = 3.14159265358979323846264338327950288;
  std::vector<double> cosv(two_n);
  for (uint32_t j = 0; j < two_n; ++j) cosv[j] = std::cos((pi * (double)j) / (double)N);
  std::vector<uint32_t> gen(nz ? nz : 1);  // 5^t mod 2N
  uint64_t g = 1;
  for (uint32_t t = 0; t < nz; ++t) {
    gen[t] = (uint32_t)g;
    g = g * 5 % two_n;
  }
  std::vector<uint32_t> live;  // slots with z_t != 0, ascending
  for (uint32_t t = 0; t < nz; ++t)
    if (z[t] != 0.0) live.push_back(t);
  const double scale = delta * (2.0 / (double)N);
  parallel_for(N, [&](uint32_t lo, uint32_t hi) {
    for (uint32_t k = lo; k < hi; ++k) {
      double acc = 0.0;
      for (uint32_t t : live) {
        const double term = z[t] * cosv[(uint32_t)(((uint64_t)gen[t] * k) % two_n)];
        acc = acc + term;
      }
      m[k] = (int64_t)std::round(scale * acc);
    }
  });
}

void decode_all(const double* m, uint32_t N, double delta, double* z) {
  // E[j] = sum_k (m_k zeta^k) w^(j k), w = exp(2 pi i / N): evaluation at zeta^(2j+1).
  typedef std::complex<double> cd;
  const double pi = 3.14159265358979323846264338327950288;
  std::vector<cd> a(N);
  for (uint32_t k = 0; k < N; ++k) a[k] = m[k] * std::polar(1.0, pi * (double)k / (double)N);
  uint32_t logn = 0;
  while ((1u << logn) < N) ++logn;
  for (uint32_t i = 0; i < N; ++i) {
    uint32_t r = 0, x = i;
    for (uint32_t b = 0; b < logn; ++b) {
      r = (r << 1) | (x & 1);
      x >>= 1;
    }
    if (i < r) std::swap(a[i], a[r]);
  }
  for (uint32_t len = 2; len <= N; len <<= 1) {
    const double ang = 2.0 * pi / (double)len;
    for (uint32_t j = 0; j < len / 2; ++j) {
      const cd w = std::polar(1.0, ang * (double)j);
      for (uint32_t s = 0; s < N; s += len) {
        cd u = a[s + j], v = a[s + j + len / 2] * w;
        a[s + j] = u + v;
        a[s + j + len / 2] = u - v;
      }
    }
  }
  const uint32_t S = N / 2;
  uint64_t g = 1;
  for (uint32_t t = 0; t < S; ++t) {
    z[t] = a[(uint32_t)((g - 1) / 2)].real() / delta;
    g = g * 5 % (2 * (uint64_t)N);
  }
}

}  // namespace fhe
