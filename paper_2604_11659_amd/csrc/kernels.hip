// gfx950 kernels for RNS-CKKS: negacyclic NTT, automorphism, tensor product, hybrid key switching
// (ModUp fast base conversion, key inner product, ModDown), rescale, one-hot mask multiply and
// accumulation. Residues are uint64 in [0, q), limb-major ([..][limb][coefficient]) so that a
// wavefront reads 64 consecutive coefficients of one limb (512 contiguous bytes).
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "kernels.h"

namespace fhe {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxAlpha = 8;
constexpr int kMaxK = 8;

__device__ __forceinline__ uint32_t brev_bits(uint32_t x, uint32_t bits) { return __brev(x) >> (32 - bits); }

__device__ __forceinline__ uint32_t mod_index(const LimbBatch& lb, uint32_t poly, uint32_t e) {
  if (e >= lb.n_first) return lb.p_base + (e - lb.n_first);
  if (lb.hole_items) {
    const uint32_t j = lb.hole_j0 + poly / lb.hole_items;
    if (e >= j * lb.hole_alpha) e += lb.hole_len;
  }
  return e;
}

// Index k' such that the NTT-domain value of tau_g(a) at position k is a[k'] (bit-reversed order:
// position k holds the evaluation at psi^(2 brv(k) + 1)).
__device__ __forceinline__ uint32_t automorph_src(uint32_t k, uint32_t g, uint32_t logN) {
  uint64_t e = 2ull * brev_bits(k, logN) + 1;
  uint32_t ge = (uint32_t)((e * g) & ((2ull << logN) - 1));
  return brev_bits((ge - 1) >> 1, logN);
}

inline uint32_t grid_for(uint64_t total) {
  uint64_t blocks = (total + kThreads - 1) / kThreads;
  if (blocks > (1u << 20)) blocks = 1u << 20;
  if (blocks == 0) blocks = 1;
  return (uint32_t)blocks;
}

// ------------------------------------------------------------------------------------------------
// NTT. Cooley-Tukey (forward) / Gentleman-Sande (inverse) with the 2N-th root psi merged into the
// twiddles: stage s pairs j and j + t (t = N / 2^(s+1)) with w = psi_rev[2^s + floor(j / 2t)].
// A limb is viewed as an N1 x N2 matrix (N1 = 2^k1 rows of N2 = 2^(logN-k1)). Phase 1 runs stages
// 0..k1-1 (pairs inside a column, stride N2); phase 2 runs stages k1..logN-1 (pairs inside a row).
// Each workgroup moves a 4096-element tile (several columns, resp. several contiguous rows) through
// LDS; inside a phase, stages are done in rounds of up to four: every thread gathers 16 elements
// whose row/column index differs only in the round's 4 bits, runs the 4 stages in registers and
// scatters back, so LDS is crossed once per 4 stages instead of once per stage. LDS rows are padded
// by one element per 16 to keep 64-bit accesses of a wavefront on distinct banks.
// Arithmetic: Q primes (< 2^50) use an exact FP64-FMA multiply (quotient from the product with
// w/q, remainder recovered exactly with two FMAs, one conditional correction); the special primes
// (< 2^61) use integer Shoup multiplication. Both return the same residue in [0, q).
// ------------------------------------------------------------------------------------------------

constexpr uint32_t kNttLogE = 12;
constexpr uint32_t kNttE = 1u << kNttLogE;
constexpr uint32_t kNttLdsElems = kNttE + (kNttE >> 4);

__device__ __forceinline__ uint32_t pad_idx(uint32_t i) { return i + (i >> 4); }

// LDS layouts of a tile: the default pads one word per 16 (rows of the row phase, columns of the
// standalone column phase); ColSwz<K1> is the column layout of the fused column kernels (2048-element
// tiles, 4 wavefronts, K1 column stages): column c of row x is stored at x C + (c ^ (h(x) Cw)), an
// XOR swizzle inside the row that sends the rows touched by one 16-lane LDS access to different
// banks (conflict-free for K1 = 6, 7; two-way for K1 = 8).
struct PadLayout {
  __device__ __forceinline__ static uint32_t idx(uint32_t i) { return i + (i >> 4); }
};
template <int K1>
struct ColSwz {
  static constexpr uint32_t kLogC = 11 - K1, kLogCw = kLogC - 2;
  __device__ __forceinline__ static uint32_t h(uint32_t x) {
    if (K1 == 6) return (x ^ (x >> 3)) & 1;
    if (K1 == 7) return (x ^ (x >> 1) ^ (x >> 3)) & 3;
    return (x ^ (x >> 2)) & 3;
  }
  __device__ __forceinline__ static uint32_t idx(uint32_t li) { return li ^ (h(li >> kLogC) << kLogCw); }
};

// A copy of x the compiler cannot see through: index arithmetic derived from it is recomputed
// where it is used instead of being kept live (in registers) across the transform rounds.
__device__ __forceinline__ uint32_t opaque(uint32_t x) {
  asm volatile("" : "+v"(x));
  return x;
}
__device__ __forceinline__ double opaque(double x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Pointers read from per-item device tables are generic pointers to the compiler, so accesses through
// them compile to flat instructions, which also count on the LDS counter: every wait for such a load
// then waits for the wavefront's LDS operations too (and the other way round), and LDS accesses cannot
// be moved past them. All of them point to global memory; this cast makes them global loads/stores.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// Workgroups are dealt to the eight XCDs in turn, each XCD with its own L2. For a grid of nitems x
// nrest workgroups this splits the block index into (item, rest) so that each XCD gets a contiguous
// share of the grid with the items innermost: the workgroups of all items that read the same
// per-(limb, tile) data (twiddles, and key tiles for items that share a key) run back to back on one
// XCD. A grid that is not a multiple of 8 keeps the plain order (rest innermost).
__device__ __forceinline__ void xcd_split(uint32_t nitems, uint32_t& item, uint32_t& rest) {
  const uint32_t wg = blockIdx.x;
  if ((gridDim.x & 7) == 0) {
    const uint32_t lg = (wg & 7) * (gridDim.x >> 3) + (wg >> 3);
    item = lg % nitems;
    rest = lg / nitems;
  } else {
    const uint32_t nrest = gridDim.x / nitems;
    item = wg / nrest;
    rest = wg - item * nrest;
  }
}

// Exact conversions between uint64 and double for integers in [0, 2^52): the double 2^52 + x has the
// bits of x as its mantissa, so each direction is one FP64 add and one bit operation (the generic
// 64-bit conversions take four to six instructions).
__device__ __forceinline__ double u52_to_f64(uint64_t x) {
  return __longlong_as_double((long long)(x | 0x4330000000000000ull)) - 0x1p52;
}
__device__ __forceinline__ uint64_t f64_to_u52(double x) {
  return (uint64_t)__double_as_longlong(x + 0x1p52) & 0x000FFFFFFFFFFFFFull;
}

// Integer arithmetic for the special primes (p < 2^61, so 4p < 2^63), with lazy reduction in the
// style of Harvey's NTT butterflies: forward butterflies keep values in [0, 4p) (the sum branch is
// brought below 2p before use, the twiddle product is left in [0, 2p)), inverse butterflies keep
// [0, 2p). Values leave the transform through lds_out / raw, which reduce to [0, p).
// Key-switching key words are in Montgomery form (x R mod p, R = 2^64); the key product accepts
// x < 4p since 4p * p < p * 2^64.
struct IntArith {
  typedef uint64_t T;
  typedef uint64_t W;
  typedef uint64_t Acc;
  uint64_t q, qinv, q2;
  __device__ __forceinline__ void init(const ModInfo& m) {
    q = m.q;
    qinv = m.qinv;
    q2 = 2 * m.q;
  }
  __device__ __forceinline__ uint64_t reduce4(uint64_t x) const {  // [0, 4p) -> [0, p)
    x = x >= q2 ? x - q2 : x;
    return x >= q ? x - q : x;
  }
  __device__ __forceinline__ uint64_t lds_in(uint64_t x) const { return x; }  // global -> LDS word
  __device__ __forceinline__ uint64_t lds_out(uint64_t x) const { return reduce4(x); }  // -> [0, p)
  __device__ __forceinline__ uint64_t raw(uint64_t x) const { return reduce4(x); }
  __device__ __forceinline__ T ld(uint64_t x) const { return x; }
  __device__ __forceinline__ uint64_t st(T x) const { return x; }
  __device__ __forceinline__ T from_u64(uint64_t x) const { return x; }
  __device__ __forceinline__ void round_end(T&) const {}
  __device__ __forceinline__ void ct(T& a, T& b, W w, W wx) const {
    const T x = a >= q2 ? a - q2 : a;           // [0, 2p)
    const T t = shoup_mul_lazy(b, w, wx, q);    // [0, 2p)
    a = x + t;                                  // [0, 4p)
    b = x - t + q2;                             // (0, 4p)
  }
  __device__ __forceinline__ void gs(T& a, T& b, W w, W wx) const {
    const T u = a, v = b;                       // [0, 2p)
    const T s = u + v;
    a = s >= q2 ? s - q2 : s;                   // [0, 2p)
    b = shoup_mul_lazy(u - v + q2, w, wx, q);   // [0, 2p)
  }
  // Key inner product: acc + x * key (key word in Montgomery form), in [0, p).
  __device__ __forceinline__ Acc kacc(Acc acc, T x, uint64_t kw) const {
    return add_mod(acc, mont_mul(x, kw, q, qinv), q);
  }
  __device__ __forceinline__ void kred(Acc&) const {}
  __device__ __forceinline__ uint64_t kfinal(Acc acc) const { return acc; }
};

// FP64 arithmetic for q < 2^50 on signed residues (doubles holding integers), lazily reduced.
//   mulc(a, w) (twiddle w in [0, q), wq = fl(w / q)): c = rint(a wq); a w = h + l exactly (FMA);
//     r = (h - c q) + l, both steps exact. The quotient estimate is off by at most 0.5 + |a| / 4q,
//     so |r| <= (0.5 + |a| / 4q) q, and every intermediate is an integer below 2^53 in magnitude.
//   red(x) = x - q rint(x / q) lies within [-q/2 - 2, q/2 + 2].
// Forward butterflies leave sums unreduced inside a round of at most four stages: from |x| <= q the
// magnitudes grow to at most 1.75q, 2.7q, 3.9q, 5.4q (< 2^53). Inverse butterflies reduce the sum
// branch every stage (|x| <= q throughout). Every round ends with red(); LDS holds the doubles'
// bits between rounds, and values leave LDS as [0, q) integers.
// Key-switching key words are the doubles' bits of plain residues in [0, q).
struct FpArith {
  typedef double T;
  typedef double W;
  typedef double Acc;
  double q, qinv;
  __device__ __forceinline__ void init(const ModInfo& m) {
    q = (double)m.q;
    qinv = 1.0 / q;
  }
  __device__ __forceinline__ uint64_t lds_in(uint64_t x) const { return __double_as_longlong(u52_to_f64(x)); }
  __device__ __forceinline__ uint64_t lds_out(uint64_t bits) const {
    const double x = __longlong_as_double((long long)bits);
    return f64_to_u52(x < 0.0 ? x + q : x);
  }
  __device__ __forceinline__ uint64_t raw(uint64_t bits) const { return bits; }  // internal form as is
  __device__ __forceinline__ T ld(uint64_t bits) const { return __longlong_as_double((long long)bits); }
  __device__ __forceinline__ uint64_t st(T x) const { return (uint64_t)__double_as_longlong(x); }
  __device__ __forceinline__ T from_u64(uint64_t x) const { return u52_to_f64(x); }
  __device__ __forceinline__ T red(T x) const { return __fma_rn(-rint(x * qinv), q, x); }
  __device__ __forceinline__ T mulc(T a, W w, W wq) const {
    const double c = rint(a * wq);
    const double h = a * w;
    const double l = __fma_rn(a, w, -h);
    return __fma_rn(-c, q, h) + l;
  }
  __device__ __forceinline__ void round_end(T& x) const { x = red(x); }
  __device__ __forceinline__ void ct(T& a, T& b, W w, W wq) const {
    const T t = mulc(b, w, wq);
    b = a - t;
    a = a + t;
  }
  __device__ __forceinline__ void gs(T& a, T& b, W w, W wq) const {
    const T d = a - b;
    a = red(a + b);
    b = mulc(d, w, wq);
  }
  // Key inner product: acc + x * k with |x| < q and k in [0, q). The quotient of h = fl(x k) by q is
  // estimated from fl(h / q) to within 0.875, so each term has |r| <= 0.875q; the sum is reduced every
  // four digits (kred), which keeps it below 4q + q/2 + 2 < 2^53.
  __device__ __forceinline__ Acc kacc(Acc acc, T x, uint64_t kw) const {
    const double k = __longlong_as_double((long long)kw);
    const double h = x * k;
    const double l = __fma_rn(x, k, -h);
    const double c = rint(h * qinv);
    return acc + (__fma_rn(-c, q, h) + l);
  }
  __device__ __forceinline__ void kred(Acc& acc) const { acc = red(acc); }
  __device__ __forceinline__ uint64_t kfinal(Acc acc) const {
    const double x = red(acc);
    return f64_to_u52(x < 0.0 ? x + q : x);
  }
};

// One round: bits [lo, lo + M) of the in-phase index x, with NT threads holding EPT elements each
// (NT * EPT = tile size). k = bits of x, logC = log2(sub-transforms per tile), sbase = global index of
// the phase's first stage, j0 = global index of the tile's first element.
// Thread group g holds x = (xh << (lo + M)) | (i << lo) | xl for i in [0, 2^M). At the stage on bit
// b = lo + bl the twiddle index 2^s + floor(j / 2^(b+1)) depends on i only through i >> (bl + 1), so
// each of the 2^(M - bl - 1) twiddles of the stage is loaded once and shared by 2^bl butterflies.
// kWave: every wavefront owns C / (NT / 64) of the tile's sub-transforms (columns in phase 1, rows in
// phase 2) and only touches their LDS slots, so rounds need a wavefront-level sync only.
template <int NT>
struct WaveSplit {
  static constexpr uint32_t kWaves = NT / 64;
  static constexpr uint32_t kLogWaves = kWaves == 1 ? 0 : kWaves == 2 ? 1 : kWaves == 4 ? 2 : kWaves == 8 ? 3 : 4;
};

template <int M, bool kInv, int kPhase, class A, int EPT, int NT, bool kWave, class L>
__device__ __forceinline__ void ntt_round(uint64_t* lds, const A& ar, const typename A::W* tw2, uint32_t lo,
                                          uint32_t k, uint32_t logC, uint32_t sbase, uint64_t j0) {
  constexpr uint32_t GM = 1u << M, G = EPT >> M;
  constexpr uint32_t TH = kWave ? 64 : NT, LW = kWave ? WaveSplit<NT>::kLogWaves : 0;
  const uint32_t lane = kWave ? (threadIdx.x & 63) : threadIdx.x;
  const uint32_t wbase = kWave ? (threadIdx.x >> 6) << (logC - LW) : 0;  // first sub-transform of this wave
  const uint32_t logCw = logC - LW;
  typename A::T r[EPT];
  uint32_t xh[G], xl[G], cc[G];
#pragma unroll
  for (uint32_t u = 0; u < G; ++u) {
    const uint32_t gid = u * TH + lane;
    if (kPhase == 1) {
      cc[u] = wbase + (gid & ((1u << logCw) - 1));
      const uint32_t rest = gid >> logCw;
      xl[u] = rest & ((1u << lo) - 1);
      xh[u] = rest >> lo;
    } else {
      xl[u] = gid & ((1u << lo) - 1);
      const uint32_t rest = gid >> lo, nh = k - lo - M;
      xh[u] = rest & ((1u << nh) - 1);
      cc[u] = wbase + (rest >> nh);
    }
    const uint32_t xb = (xh[u] << (lo + M)) | xl[u];
#pragma unroll
    for (uint32_t i = 0; i < GM; ++i) {
      const uint32_t x = xb | (i << lo);
      const uint32_t li = kPhase == 1 ? (x << logC) + cc[u] : (cc[u] << k) + x;
      r[u * GM + i] = ar.ld(lds[L::idx(li)]);
    }
  }
#pragma unroll
  for (uint32_t sb = 0; sb < M; ++sb) {
    const uint32_t bl = kInv ? sb : (M - 1 - sb);
    const uint32_t b = lo + bl;
    const uint32_t s = sbase + (k - 1 - b);
#pragma unroll
    for (uint32_t u = 0; u < G; ++u) {
      uint32_t base = (1u << s) + (xh[u] << (M - bl - 1));
      if (kPhase == 2) base += (uint32_t)(j0 >> (b + 1)) + (cc[u] << (k - b - 1));
#pragma unroll
      for (uint32_t t = 0; t < (1u << (M - bl - 1)); ++t) {
        const typename A::W W = tw2[2 * (base + t)], Wx = tw2[2 * (base + t) + 1];
#pragma unroll
        for (uint32_t low = 0; low < (1u << bl); ++low) {
          const uint32_t i = (t << (bl + 1)) | low, i2 = i | (1u << bl);
          if (kInv) ar.gs(r[u * GM + i], r[u * GM + i2], W, Wx);
          else ar.ct(r[u * GM + i], r[u * GM + i2], W, Wx);
        }
      }
    }
  }
#pragma unroll
  for (uint32_t u = 0; u < G; ++u) {
    const uint32_t xb = (xh[u] << (lo + M)) | xl[u];
#pragma unroll
    for (uint32_t i = 0; i < GM; ++i) {
      const uint32_t x = xb | (i << lo);
      const uint32_t li = kPhase == 1 ? (x << logC) + cc[u] : (cc[u] << k) + x;
      ar.round_end(r[u * GM + i]);
      lds[L::idx(li)] = ar.st(r[u * GM + i]);
    }
  }
}

// Wavefront-level sync for LDS data exchanged among the lanes of one wavefront.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool kInv, int kPhase, class A, int EPT, int NT, bool kWave = false, class L = PadLayout>
__device__ __forceinline__ void ntt_rounds(uint64_t* lds, const A& ar, const typename A::W* tw2, uint32_t k,
                                           uint32_t logC, uint32_t sbase, uint64_t j0) {
  // Rounds of MB = log2(EPT) bits. Forward: chunks from the top ([k-MB, k), [k-2MB, k-MB), ...,
  // [0, rem)); inverse: the same chunks in reverse order.
  constexpr uint32_t MB = EPT == 16 ? 4 : (EPT == 8 ? 3 : 2);
  const uint32_t nr = (k + MB - 1) / MB;
#pragma unroll
  for (uint32_t rr = 0; rr < nr; ++rr) {
    const uint32_t rf = kInv ? nr - 1 - rr : rr;
    const uint32_t hi = k - MB * rf;
    const uint32_t lo = hi >= MB ? hi - MB : 0;
    switch (hi - lo) {
      case 4:
        if constexpr (MB >= 4) ntt_round<4, kInv, kPhase, A, EPT, NT, kWave, L>(lds, ar, tw2, lo, k, logC, sbase, j0);
        break;
      case 3:
        if constexpr (MB >= 3) ntt_round<3, kInv, kPhase, A, EPT, NT, kWave, L>(lds, ar, tw2, lo, k, logC, sbase, j0);
        break;
      case 2: ntt_round<2, kInv, kPhase, A, EPT, NT, kWave, L>(lds, ar, tw2, lo, k, logC, sbase, j0); break;
      default: ntt_round<1, kInv, kPhase, A, EPT, NT, kWave, L>(lds, ar, tw2, lo, k, logC, sbase, j0); break;
    }
    if (kWave)
      wave_sync();
    else
      __syncthreads();
  }
}

// kSrcPtr: the first phase reads its input through lb.src_ptr / lb.src_gal (automorphism gather).
// KR: the row phase's stage count as a compile-time constant (0: logN - k1 at run time), so its
// rounds unroll and their index arithmetic folds.
template <bool kInv, int kPhase, class A, int NT, bool kSrcPtr = false, int KR = 0>
__global__ __launch_bounds__(NT) void k_ntt(LimbBatch lb, const ModInfo* __restrict__ mods,
                                                 const typename A::W* __restrict__ tw, uint32_t logN, uint32_t k1,
                                                 bool from_src) {
  extern __shared__ uint64_t lds[];
  constexpr uint32_t kPer = kNttE / NT;
  const uint32_t N = 1u << logN, tiles = N >> kNttLogE;
  uint32_t poly, e, tile;
  if (kPhase == 2) {  // rows: polynomials innermost per XCD (a limb's twiddles in one L2)
    uint32_t rest;
    xcd_split(lb.npoly, poly, rest);
    tile = rest % tiles;
    e = rest / tiles;
  } else {
    const uint32_t limb = blockIdx.x / tiles;
    tile = blockIdx.x - limb * tiles;
    poly = limb / lb.limbs;
    e = limb - poly * lb.limbs;
  }
  uint64_t* a = lb.base + (uint64_t)poly * lb.poly_stride + (uint64_t)e * N;
  const uint64_t* in = from_src && lb.src ? lb.src + (uint64_t)poly * lb.src_stride + (uint64_t)e * N : a;
  const uint32_t mi = mod_index(lb, poly, e);
  const ModInfo m = mods[mi];
  A ar;
  ar.init(m);
  const uint32_t k2 = KR ? KR : logN - k1, k = kPhase == 1 ? k1 : k2;
  const uint32_t logC = kNttLogE - k, C = 1u << logC;
  const uint32_t j0 = tile * kNttE;
  const uint64_t toff = (uint64_t)mi * 4 * N + (kInv ? 2 * (uint64_t)N : 0);
  if (kPhase == 2) {
    // rows are contiguous: every wavefront loads, transforms and stores its own rows
    const uint32_t wb = (threadIdx.x >> 6) * (kNttE / (NT / 64)), lane = threadIdx.x & 63;
    if (kSrcPtr) {
      // read through the automorphism: a wavefront's 64 indices map into one aligned 64-word block
      const auto sp = gmem(lb.src_ptr[poly] + (uint64_t)(lb.src_ptr_limb0 + e) * N);
      const uint32_t g = lb.src_gal[poly];
#pragma unroll
      for (uint32_t r_ = 0; r_ < kPer; ++r_) {
        const uint32_t idx = wb + lane + r_ * 64;
        lds[pad_idx(idx)] = ar.lds_in(sp[automorph_src(j0 + idx, g, logN)]);
      }
    } else {
#pragma unroll
      for (uint32_t r_ = 0; r_ < kPer; ++r_) {
        const uint32_t idx = wb + lane + r_ * 64;
        lds[pad_idx(idx)] = ar.lds_in(in[j0 + idx]);
      }
    }
    wave_sync();
    ntt_rounds<kInv, 2, A, kPer, NT, true>(lds, ar, tw + toff, k, logC, k1, j0);
    const uint32_t ln = opaque(lane);
#pragma unroll
    for (uint32_t r_ = 0; r_ < kPer; ++r_) {
      const uint32_t idx = wb + ln + r_ * 64;
      a[j0 + idx] = lb.raw_out ? ar.raw(lds[pad_idx(idx)]) : ar.lds_out(lds[pad_idx(idx)]);
    }
  } else {
    // columns are strided: coalesced loads and stores across the workgroup, rounds per wavefront
#pragma unroll
    for (uint32_t r_ = 0; r_ < kPer; ++r_) {
      const uint32_t idx = threadIdx.x + r_ * NT;
      lds[pad_idx(idx)] = ar.lds_in(in[((idx >> logC) << k2) + (tile << logC) + (idx & (C - 1))]);
    }
    __syncthreads();
    ntt_rounds<kInv, 1, A, kPer, NT, true>(lds, ar, tw + toff, k, logC, 0, 0);
    __syncthreads();
    const uint32_t tid = opaque(threadIdx.x);
#pragma unroll
    for (uint32_t r_ = 0; r_ < kPer; ++r_) {
      const uint32_t idx = tid + r_ * NT;
      uint64_t v = lb.raw_out ? ar.raw(lds[pad_idx(idx)]) : ar.lds_out(lds[pad_idx(idx)]);
      if (kInv) v = shoup_mul(v, m.n_inv, m.n_inv_shoup, m.q);
      a[((idx >> logC) << k2) + (tile << logC) + (idx & (C - 1))] = v;
    }
  }
}

// Row phase of the forward NTT of the ModUp digits fused with the key inner product.
// Workgroup (item b, extended limb e, tile), 512 threads holding 8 elements each: for every digit
// j, the digit's row for limb e (column phase already applied) goes through the row stages in LDS
// and is multiplied by the key tile; for the digit that contains e the NTT-domain input is used
// directly. Only u = sum_j ext_j * key_j (both components) is written, so the transformed digits
// never return to HBM.
constexpr int kInnerThreads = 512;
template <class A, bool kSrcPtr>
__device__ __forceinline__ void ntt_p2_inner_body(
    uint32_t B, uint32_t nl, uint32_t K, uint32_t nq, uint32_t alpha, uint32_t R, uint32_t e0, uint32_t ne,
    uint32_t logN, uint32_t k1, const ModInfo* __restrict__ mods, const typename A::W* __restrict__ tw,
    const uint64_t* __restrict__ in, uint64_t in_stride, const uint64_t* const* __restrict__ in_ptr,
    const uint32_t* __restrict__ in_gal, const uint64_t* __restrict__ ext,
    const uint64_t* const* __restrict__ keys, uint64_t* __restrict__ u) {
  extern __shared__ uint64_t lds[];
  constexpr uint32_t kPer = kNttE / kInnerThreads;
  const uint32_t N = 1u << logN, tiles = N >> kNttLogE;
  uint32_t tile, e, b;
  if (std::is_same<A, FpArith>::value) {  // items innermost per XCD (twiddles and shared keys in L2)
    uint32_t rest;
    xcd_split(B, b, rest);
    tile = rest % tiles;
    e = e0 + rest / tiles;
  } else {
    tile = blockIdx.x % tiles;
    const uint32_t be = blockIdx.x / tiles;
    e = e0 + be % ne;
    b = be / ne;
  }
  const uint32_t next = nl + K, beta = (nl + alpha - 1) / alpha, nall = nq + K;
  const uint32_t mi = e < nl ? e : nq + (e - nl);
  const ModInfo m = mods[mi];
  const uint64_t j0 = (uint64_t)tile * kNttE;
  const uint32_t k = logN - k1, logC = kNttLogE - k;
  const auto key = gmem(keys[b]);
  A ar;
  ar.init(m);
  const typename A::W* w = tw + (uint64_t)mi * 4 * N;
  // every wavefront owns whole rows of the tile (contiguous): loads, rounds, products and stores
  // stay inside the wavefront, so no workgroup barrier is needed
  const uint32_t wb = (threadIdx.x >> 6) * (kNttE / (kInnerThreads / 64)), lane = threadIdx.x & 63;
  typename A::Acc acc0[kPer], acc1[kPer];
#pragma unroll
  for (uint32_t r = 0; r < kPer; ++r) acc0[r] = acc1[r] = 0;
  for (uint32_t j = 0; j < beta; ++j) {
    const uint32_t lo = j * alpha, cnt = min(alpha, nl - lo);
    const auto kb = key + ((uint64_t)(j * 2 + 0) * nall + mi) * N + j0;
    const auto ka = key + ((uint64_t)(j * 2 + 1) * nall + mi) * N + j0;
    if (e >= lo && e < lo + cnt) {  // the digit's own limbs (Q limbs only)
      if (kSrcPtr) {  // the input read through its automorphism (rotation without a separate pass)
        const auto x = gmem(in_ptr[b] + (uint64_t)e * N);
        const uint32_t g = in_gal[b];
#pragma unroll
        for (uint32_t r = 0; r < kPer; ++r) {
          const uint32_t idx = wb + lane + r * 64;
          const typename A::T xv = ar.from_u64(x[automorph_src((uint32_t)j0 + idx, g, logN)]);
          acc0[r] = ar.kacc(acc0[r], xv, kb[idx]);
          acc1[r] = ar.kacc(acc1[r], xv, ka[idx]);
        }
      } else {
        const uint64_t* x = in + (uint64_t)b * in_stride + (uint64_t)e * N + j0;
#pragma unroll
        for (uint32_t r = 0; r < kPer; ++r) {
          const uint32_t idx = wb + lane + r * 64;
          const typename A::T xv = ar.from_u64(x[idx]);
          acc0[r] = ar.kacc(acc0[r], xv, kb[idx]);
          acc1[r] = ar.kacc(acc1[r], xv, ka[idx]);
        }
      }
    } else {
      const uint32_t row = e < lo ? e : e - cnt;
      const uint64_t* src = ext + (((uint64_t)j * B + b) * R + row) * N + j0;
#pragma unroll
      for (uint32_t r = 0; r < kPer; ++r) {
        const uint32_t idx = wb + lane + r * 64;
        lds[pad_idx(idx)] = src[idx];  // ext rows: internal form on Q primes, integers on P
      }
      wave_sync();
      ntt_rounds<false, 2, A, 8, kInnerThreads, true>(lds, ar, w, k, logC, k1, j0);
      const uint32_t ln = opaque(lane);
#pragma unroll
      for (uint32_t r = 0; r < kPer; ++r) {
        const uint32_t idx = wb + ln + r * 64;
        const typename A::T xv = ar.ld(lds[pad_idx(idx)]);
        acc0[r] = ar.kacc(acc0[r], xv, kb[idx]);
        acc1[r] = ar.kacc(acc1[r], xv, ka[idx]);
      }
      wave_sync();
    }
    if ((j & 3) == 3) {
#pragma unroll
      for (uint32_t r = 0; r < kPer; ++r) {
        ar.kred(acc0[r]);
        ar.kred(acc1[r]);
      }
    }
  }
  uint64_t* u0 = u + ((uint64_t)(b * 2 + 0) * next + e) * N + j0;
  uint64_t* u1 = u + ((uint64_t)(b * 2 + 1) * next + e) * N + j0;
#pragma unroll
  for (uint32_t r = 0; r < kPer; ++r) {
    const uint32_t idx = wb + lane + r * 64;
    u0[idx] = ar.kfinal(acc0[r]);
    u1[idx] = ar.kfinal(acc1[r]);
  }
}

// kSrcPtr: the input items are read through their automorphisms (in_ptr, in_gal; only the FP64
// instantiation reads the input at all).
template <class A, bool kSrcPtr>
__global__ __launch_bounds__(kInnerThreads) void k_ntt_p2_inner(
    uint32_t B, uint32_t nl, uint32_t K, uint32_t nq, uint32_t alpha, uint32_t R, uint32_t e0, uint32_t ne,
    uint32_t logN, uint32_t k1, const ModInfo* __restrict__ mods, const typename A::W* __restrict__ tw,
    const uint64_t* __restrict__ in, uint64_t in_stride, const uint64_t* const* __restrict__ in_ptr,
    const uint32_t* __restrict__ in_gal, const uint64_t* __restrict__ ext,
    const uint64_t* const* __restrict__ keys, uint64_t* __restrict__ u) {
  ntt_p2_inner_body<A, kSrcPtr>(B, nl, K, nq, alpha, R, e0, ne, logN, k1, mods, tw, in, in_stride, in_ptr, in_gal,
                                ext, keys, u);
}

// Hoisted rotations. The ModUp digits of S polynomials, column phase already applied
// (ext [beta][S][R][N], raw form), get their forward row phase in place, so that every rotation of a
// polynomial can read them through its automorphism afterwards. Workgroup (digit j, poly s, compact
// row r, tile); rows of Q primes (q_rows = true) and of special primes are separate launches. The
// compact row r of digit j is limb e = r (r < lo_j) or r + cnt_j, as the key-switch kernels map it.
template <class A, bool kQRows>
__global__ __launch_bounds__(kInnerThreads) void k_ext_rows(uint32_t S, uint32_t nl, uint32_t K, uint32_t nq,
                                                           uint32_t alpha, uint32_t R, uint32_t rows, uint32_t logN,
                                                           uint32_t k1, const ModInfo* __restrict__ mods,
                                                           const typename A::W* __restrict__ tw,
                                                           uint64_t* __restrict__ ext) {
  extern __shared__ uint64_t lds[];
  constexpr uint32_t kPer = kNttE / kInnerThreads;
  const uint32_t N = 1u << logN, tiles = N >> kNttLogE;
  const uint32_t tile = blockIdx.x % tiles, rest = blockIdx.x / tiles;
  const uint32_t rr = rest % rows, js = rest / rows, s = js % S, j = js / S;
  const uint32_t lo = j * alpha, cnt = min(alpha, nl - lo);
  const uint32_t nq_rows = nl - cnt;  // Q rows of this digit
  if (kQRows && rr >= nq_rows) return;  // the last digit may have fewer rows (whole workgroup exits)
  const uint32_t r = kQRows ? rr : nq_rows + rr;
  const uint32_t e = r < lo ? r : r + cnt;
  const uint32_t mi = e < nl ? e : nq + (e - nl);
  A ar;
  ar.init(mods[mi]);
  const uint32_t j0 = tile * kNttE, k = logN - k1, logC = kNttLogE - k;
  uint64_t* row = ext + (((uint64_t)j * S + s) * R + r) * N + j0;
  const uint32_t wb = (threadIdx.x >> 6) * (kNttE / (kInnerThreads / 64)), lane = threadIdx.x & 63;
#pragma unroll
  for (uint32_t r_ = 0; r_ < kPer; ++r_) {
    const uint32_t idx = wb + lane + r_ * 64;
    lds[pad_idx(idx)] = row[idx];  // raw form, as the column phase left it
  }
  wave_sync();
  ntt_rounds<false, 2, A, kPer, kInnerThreads, true>(lds, ar, tw + (uint64_t)mi * 4 * N, k, logC, k1, j0);
  const uint32_t ln = opaque(lane);
#pragma unroll
  for (uint32_t r_ = 0; r_ < kPer; ++r_) {
    const uint32_t idx = wb + ln + r_ * 64;
    row[idx] = ar.raw(lds[pad_idx(idx)]);
  }
}

// Key inner product of hoisted rotations: item b rotates polynomial state[b] by tau_(gal[b]). Per
// (item, extended limb e, tile): u_c = sum_j tau(ext_j)[e] * key_(j,c)[e], reading the transformed
// digits of the item's polynomial through the automorphism (a wavefront's 64 indices fall in one
// aligned 64-word block) and, for the digit that contains e, the NTT-domain input itself. No transform.
template <class A>
__global__ __launch_bounds__(kThreads) void k_hoisted_inner(
    uint32_t B, uint32_t S, uint32_t nl, uint32_t K, uint32_t nq, uint32_t alpha, uint32_t R, uint32_t e0,
    uint32_t ne, uint32_t logN, const ModInfo* __restrict__ mods, const uint32_t* __restrict__ state,
    const uint32_t* __restrict__ gal, const uint64_t* const* __restrict__ in_ptr, const uint64_t* __restrict__ ext,
    const uint64_t* const* __restrict__ keys, uint64_t* __restrict__ u) {
  constexpr uint32_t kPer = 8, kTile = kThreads * kPer;  // 2048 coefficients per workgroup
  const uint32_t N = 1u << logN, tiles = N / kTile;
  uint32_t tile, e, b;
  if (std::is_same<A, FpArith>::value) {  // items innermost per XCD (key tiles of items sharing a key in L2)
    uint32_t rest;
    xcd_split(B, b, rest);
    tile = rest % tiles;
    e = e0 + rest / tiles;
  } else {
    tile = blockIdx.x % tiles;
    const uint32_t be = blockIdx.x / tiles;
    e = e0 + be % ne;
    b = be / ne;
  }
  const uint32_t next = nl + K, beta = (nl + alpha - 1) / alpha, nall = nq + K;
  const uint32_t mi = e < nl ? e : nq + (e - nl);
  A ar;
  ar.init(mods[mi]);
  const uint32_t j0 = tile * kTile, g = gal[b], sb = state[b];
  const auto key = gmem(keys[b]);
  const uint32_t wb = (threadIdx.x >> 6) * (kTile / (kThreads / 64)), lane = threadIdx.x & 63;
  uint32_t src[kPer];
#pragma unroll
  for (uint32_t r = 0; r < kPer; ++r) src[r] = automorph_src(j0 + wb + lane + r * 64, g, logN);
  typename A::Acc acc0[kPer], acc1[kPer];
#pragma unroll
  for (uint32_t r = 0; r < kPer; ++r) acc0[r] = acc1[r] = 0;
  for (uint32_t j = 0; j < beta; ++j) {
    const uint32_t lo = j * alpha, cnt = min(alpha, nl - lo);
    const auto kb = key + ((uint64_t)(j * 2 + 0) * nall + mi) * N + j0 + wb;
    const auto ka = key + ((uint64_t)(j * 2 + 1) * nall + mi) * N + j0 + wb;
    if (e >= lo && e < lo + cnt) {  // the digit's own limbs (Q limbs only): the input itself
      const auto x = gmem(in_ptr[b] + (uint64_t)e * N);
#pragma unroll
      for (uint32_t r = 0; r < kPer; ++r) {
        const typename A::T xv = ar.from_u64(x[src[r]]);
        acc0[r] = ar.kacc(acc0[r], xv, kb[lane + r * 64]);
        acc1[r] = ar.kacc(acc1[r], xv, ka[lane + r * 64]);
      }
    } else {
      const uint32_t row = e < lo ? e : e - cnt;
      const uint64_t* x = ext + (((uint64_t)j * S + sb) * R + row) * N;
#pragma unroll
      for (uint32_t r = 0; r < kPer; ++r) {
        const typename A::T xv = ar.ld(x[src[r]]);
        acc0[r] = ar.kacc(acc0[r], xv, kb[lane + r * 64]);
        acc1[r] = ar.kacc(acc1[r], xv, ka[lane + r * 64]);
      }
    }
    if ((j & 3) == 3) {
#pragma unroll
      for (uint32_t r = 0; r < kPer; ++r) {
        ar.kred(acc0[r]);
        ar.kred(acc1[r]);
      }
    }
  }
  uint64_t* u0 = u + ((uint64_t)(b * 2 + 0) * next + e) * N + j0 + wb;
  uint64_t* u1 = u + ((uint64_t)(b * 2 + 1) * next + e) * N + j0 + wb;
#pragma unroll
  for (uint32_t r = 0; r < kPer; ++r) {
    u0[lane + r * 64] = ar.kfinal(acc0[r]);
    u1[lane + r * 64] = ar.kfinal(acc1[r]);
  }
}

// Row phase of the forward NTT of the ModDown conversion fused with the final combine:
// out[b][c][i] = add[2b+c][i] + (u[b][c][i] - NTT(conv)[b][c][i]) P^-1 (NTT domain).
// Workgroup (poly bc = 2b + c, limb i, tile); conv has had its column phase.
template <class A, int NT, int KR = 0>  // KR as in k_ntt
__global__ __launch_bounds__(NT) void k_ntt_p2_combine(uint32_t nl, uint32_t K, uint32_t nq, uint32_t logN,
                                                            uint32_t k1, const ModInfo* __restrict__ mods,
                                                            const typename A::W* __restrict__ tw,
                                                            const uint64_t* __restrict__ tab,
                                                            const uint64_t* __restrict__ u,
                                                            const uint64_t* __restrict__ conv,
                                                            const uint64_t* const* __restrict__ add,
                                                            const uint32_t* __restrict__ galois,
                                                            uint64_t* const* __restrict__ out) {
  extern __shared__ uint64_t lds[];
  const uint32_t N = 1u << logN, tiles = N >> kNttLogE, next = nl + K;
  // plain order: tiles of one row back to back (the per-item reads stream; the XCD-interleaved order
  // measured 5 % slower here)
  const uint32_t tile = blockIdx.x % tiles, li = blockIdx.x / tiles;
  const uint32_t i = li % nl, bc = li / nl, b = bc >> 1, c = bc & 1;
  const ModInfo m = mods[i];
  A ar;
  ar.init(m);
  const uint64_t j0 = (uint64_t)tile * kNttE;
  const uint32_t k = KR ? KR : logN - k1, logC = kNttLogE - k;
  const uint64_t* src = conv + ((uint64_t)bc * nl + i) * N + j0;
  constexpr uint32_t kPer = kNttE / NT;
  const uint32_t wb = (threadIdx.x >> 6) * (kNttE / (NT / 64)), lane = threadIdx.x & 63;
#pragma unroll
  for (uint32_t r_ = 0; r_ < kPer; ++r_) {
    const uint32_t idx = wb + lane + r_ * 64;
    lds[pad_idx(idx)] = src[idx];  // conv: internal FP64 form
  }
  wave_sync();
  const typename A::W* w = tw + (uint64_t)i * 4 * N;
  ntt_rounds<false, 2, A, kPer, NT, true>(lds, ar, w, k, logC, k1, j0);
  const uint64_t* pinv = tab + 2 * K + 2 * (uint64_t)K * nq + 2 * i;
  const uint64_t* uu = u + ((uint64_t)bc * next + i) * N + j0;
  auto ad = gmem(add[bc]);
  const uint32_t gal = galois ? galois[b] : 0;  // rotation form: the addend goes through tau_gal
  if (ad) ad += (uint64_t)i * N + (galois ? 0 : j0);
  const auto o = gmem(out[b] + ((uint64_t)c * nl + i) * N + j0);
  const uint32_t ln = opaque(lane);
  // exact FP64: |u - conv| < 1.5q + 2, so the product with P^-1 is below 0.9q and adding the
  // [0, q) addend keeps the sum below 2q before the final reduction
  const double pv = (double)pinv[0], pvq = pv * ar.qinv;
  // all loads first: `o` may alias the addend as far as the compiler knows, so a load placed after
  // a store would wait for it
  uint64_t uv[kPer], av[kPer];
#pragma unroll
  for (uint32_t r_ = 0; r_ < kPer; ++r_) uv[r_] = uu[wb + ln + r_ * 64];
  if (ad && galois) {  // uniform branches outside the unrolled loops
#pragma unroll
    for (uint32_t r_ = 0; r_ < kPer; ++r_) av[r_] = ad[automorph_src(j0 + wb + ln + r_ * 64, gal, logN)];
  } else if (ad) {
#pragma unroll
    for (uint32_t r_ = 0; r_ < kPer; ++r_) av[r_] = ad[wb + ln + r_ * 64];
  } else {
#pragma unroll
    for (uint32_t r_ = 0; r_ < kPer; ++r_) av[r_] = 0;
  }
#pragma unroll
  for (uint32_t r_ = 0; r_ < kPer; ++r_) {
    const uint32_t idx = wb + ln + r_ * 64;
    double v = ar.mulc(u52_to_f64(uv[r_]) - ar.ld(lds[pad_idx(idx)]), pv, pvq);
    v += u52_to_f64(av[r_]);  // zero without an addend
    v = ar.red(v);
    o[idx] = f64_to_u52(v < 0.0 ? v + ar.q : v);
  }
}

// ------------------------------------------------------------------------------------------------
// Element-wise kernels (grid-stride over flattened index spaces).
// ------------------------------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_automorph(uint32_t B, uint32_t ncomp, uint32_t nl, uint32_t logN,
                                                       const uint64_t* const* __restrict__ src,
                                                       const uint32_t* __restrict__ galois,
                                                       uint64_t* __restrict__ dst) {
  const uint32_t N = 1u << logN;
  const uint64_t total = (uint64_t)B << logN;
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < total; t += (uint64_t)gridDim.x * kThreads) {
    const uint32_t b = (uint32_t)(t >> logN), k = (uint32_t)t & (N - 1);
    const uint32_t ks = automorph_src(k, galois[b], logN);
    const auto s = gmem(src[b]);
    uint64_t* d = dst + (uint64_t)b * ncomp * nl * N;
    for (uint32_t r = 0; r < ncomp * nl; ++r) d[(uint64_t)r * N + k] = s[(uint64_t)r * N + ks];
  }
}

__global__ __launch_bounds__(kThreads) void k_tensor(uint32_t B, uint32_t nl, uint32_t logN,
                                                    const ModInfo* __restrict__ mods,
                                                    const uint64_t* const* __restrict__ A,
                                                    const uint64_t* const* __restrict__ Bc, uint64_t* __restrict__ out) {
  const uint32_t N = 1u << logN;
  const uint64_t total = (uint64_t)B * nl << logN;
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < total; t += (uint64_t)gridDim.x * kThreads) {
    const uint32_t k = (uint32_t)t & (N - 1);
    const uint64_t r = t >> logN;
    const uint32_t i = (uint32_t)(r % nl), b = (uint32_t)(r / nl);
    const ModInfo m = mods[i];
    const auto a = gmem(A[b]);
    const auto bb = gmem(Bc[b]);
    const uint64_t a0 = a[(uint64_t)i * N + k], a1 = a[(uint64_t)(nl + i) * N + k];
    const uint64_t b0 = bb[(uint64_t)i * N + k], b1 = bb[(uint64_t)(nl + i) * N + k];
    uint64_t* o = out + (uint64_t)b * 3 * nl * N;
    o[(uint64_t)i * N + k] = mont_mul(mont_mul(a0, b0, m.q, m.qinv), m.r2, m.q, m.qinv);
    const uint64_t x = add_mod(mont_mul(a0, b1, m.q, m.qinv), mont_mul(a1, b0, m.q, m.qinv), m.q);
    o[(uint64_t)(nl + i) * N + k] = mont_mul(x, m.r2, m.q, m.qinv);
    o[(uint64_t)(2 * nl + i) * N + k] = mont_mul(mont_mul(a1, b1, m.q, m.qinv), m.r2, m.q, m.qinv);
  }
}

// ModUp (coefficient domain): for item b, digit j, coefficient k. Only the limbs outside the digit are
// produced (the digit's own limbs are the input itself): compacted rows, row r -> extended-basis limb
// e = r (r < lo) or r + cnt, laid out [digit][item][row (stride R)][N].
// tab block of digit j: [alpha][2] (Dhat_i^-1 mod q_i, shoup) then [alpha][next][2] (Dhat_i mod t_e, shoup).
__global__ __launch_bounds__(kThreads) void k_modup(uint32_t B, uint32_t nl, uint32_t K, uint32_t nq, uint32_t alpha,
                                                   uint32_t R, uint32_t logN, const ModInfo* __restrict__ mods,
                                                   const uint64_t* __restrict__ tab, const uint64_t* __restrict__ dcoef,
                                                   uint64_t* __restrict__ ext) {
  const uint32_t N = 1u << logN;
  const uint32_t beta = (nl + alpha - 1) / alpha, next = nl + K;
  const uint64_t total = (uint64_t)B * beta << logN;
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < total; t += (uint64_t)gridDim.x * kThreads) {
    const uint32_t k = (uint32_t)t & (N - 1);
    const uint64_t r = t >> logN;
    const uint32_t b = (uint32_t)(r % B), j = (uint32_t)(r / B);
    const uint32_t lo = j * alpha, cnt = min(alpha, nl - lo);
    const uint64_t* blk = tab + (uint64_t)j * (2 * alpha + 2 * alpha * next);
    const uint64_t* d = dcoef + (uint64_t)b * nl * N;
    uint64_t y[kMaxAlpha];
    for (uint32_t i = 0; i < cnt; ++i)
      y[i] = shoup_mul(d[(uint64_t)(lo + i) * N + k], blk[2 * i], blk[2 * i + 1], mods[lo + i].q);
    uint64_t* o = ext + ((uint64_t)j * B + b) * R * N + k;
    for (uint32_t row = 0; row < next - cnt; ++row) {
      const uint32_t e = row < lo ? row : row + cnt;
      const uint64_t tq = mods[e < nl ? e : nq + (e - nl)].q;
      const uint64_t* mrow = blk + 2 * alpha + 2 * (uint64_t)e;
      uint64_t v = 0;
      for (uint32_t i = 0; i < cnt; ++i) {
        const uint64_t* c = mrow + (uint64_t)i * 2 * next;
        v = add_mod(v, shoup_mul(y[i], c[0], c[1], tq), tq);
      }
      o[(uint64_t)row * N] = v;
    }
  }
}

// ModDown base conversion P -> Q_l (coefficient domain) with centred representatives:
// z_k = [u_(p_k) (P/p_k)^-1]_(p_k) is used as z_k - p_k when z_k > (p_k - 1)/2, so the rounding error of
// the division by P is zero-mean. Since p_k (P/p_k) = P, each centred term subtracts P mod q_i.
// tab: [K][2] ((P/p_k)^-1 mod p_k), [K][nq][2] ((P/p_k) mod q_i), [nq][2] (P^-1 mod q_i), [nq] (P mod q_i).
__global__ __launch_bounds__(kThreads) void k_moddown_conv(uint32_t B, uint32_t nl, uint32_t K, uint32_t nq,
                                                          uint32_t logN, const ModInfo* __restrict__ mods,
                                                          const uint64_t* __restrict__ tab,
                                                          const uint64_t* __restrict__ u,
                                                          uint64_t* __restrict__ conv) {
  const uint32_t N = 1u << logN, next = nl + K;
  const uint64_t total = (uint64_t)B * 2 << logN;
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < total; t += (uint64_t)gridDim.x * kThreads) {
    const uint32_t k = (uint32_t)t & (N - 1);
    const uint32_t bc = (uint32_t)(t >> logN);
    uint64_t z[kMaxK];
    uint32_t nneg = 0;
    for (uint32_t kk = 0; kk < K; ++kk) {
      const uint64_t pk = mods[nq + kk].q;
      z[kk] = shoup_mul(u[((uint64_t)bc * next + nl + kk) * N + k], tab[2 * kk], tab[2 * kk + 1], pk);
      nneg += z[kk] > (pk - 1) / 2 ? 1u : 0u;
    }
    const uint64_t* pq = tab + 2 * K;
    const uint64_t* pmod = tab + 2 * K + 2 * (uint64_t)K * nq + 2 * nq;
    for (uint32_t i = 0; i < nl; ++i) {
      const uint64_t q = mods[i].q;
      uint64_t acc = 0;
      for (uint32_t kk = 0; kk < K; ++kk) {
        const uint64_t* c = pq + 2 * ((uint64_t)kk * nq + i);
        acc = add_mod(acc, shoup_mul(z[kk], c[0], c[1], q), q);
      }
      for (uint32_t n = 0; n < nneg; ++n) acc = sub_mod(acc, pmod[i], q);
      conv[((uint64_t)bc * nl + i) * N + k] = acc;
    }
  }
}

// Column-phase tiles of 2^LOG_E elements: 2^k1 rows (stride 2^(logN - k1)) by C = 2^(LOG_E - k1)
// adjacent columns.
// Column-phase slots owned by one wavefront in the fused column kernels (2048-element tiles, four
// wavefronts, ColSwz<K1> layout): wavefront w owns columns [w Cw, (w + 1) Cw) of the tile
// (Cw = C / 4) in every row; lane l handles slots l + 64 r (r < 8), i.e. row l / Cw + r 64 / Cw and
// column w Cw + l mod Cw. Consecutive r are 256 LDS words apart, and the swizzle depends on r only
// through r mod 2 (the row bits it reads above l / Cw are bit 0 of r, or none for K1 = 8), so two
// base indices kept in registers give every slot's LDS word with a constant offset that folds into
// the LDS instruction. The coefficient index advances by (64 / Cw) 2^k2 per r.
template <int K1>
struct ColSlots {
  static constexpr uint32_t kLogC = 11 - K1, kLogCw = kLogC - 2, kLogRows = 6 - kLogCw, kStep = 256, kEPT = 8;
  uint32_t lds_even, lds_odd, g0, gshift;
  __device__ __forceinline__ ColSlots(uint32_t lane, uint32_t wv, uint32_t k2, uint32_t tile) {
    const uint32_t row0 = lane >> kLogCw, col = (wv << kLogCw) + (lane & ((1u << kLogCw) - 1));
    const uint32_t li0 = (row0 << kLogC) + col;
    lds_even = ColSwz<K1>::idx(li0);
    lds_odd = ColSwz<K1>::idx(li0 + kStep) - kStep;
    g0 = (row0 << k2) + (tile << kLogC) + col;
    gshift = k2 + kLogRows;
  }
  // opaque bases: the per-slot sums are formed at each use instead of being kept live in registers
  __device__ __forceinline__ uint32_t lds(uint32_t r) const {
    return opaque((r & 1) ? lds_odd : lds_even) + r * kStep;
  }
  __device__ __forceinline__ uint32_t g(uint32_t r) const { return opaque(g0) + (r << gshift); }
  // work <- src over the lane's kEPT slots: every load is issued before the first LDS write, so the
  // wavefront waits for one memory latency instead of kEPT of them
  __device__ __forceinline__ void load(uint64_t* work, const uint64_t* src) const {
    uint64_t v[kEPT];
#pragma unroll
    for (uint32_t r = 0; r < kEPT; ++r) v[r] = src[g(r)];
#pragma unroll
    for (uint32_t r = 0; r < kEPT; ++r) work[lds(r)] = v[r];
  }
  // dst <- f(work) over the lane's kEPT slots, all LDS reads first
  template <class F>
  __device__ __forceinline__ void store(uint64_t* dst, const uint64_t* work, F f) const {
    uint64_t v[kEPT];
#pragma unroll
    for (uint32_t r = 0; r < kEPT; ++r) v[r] = f(work[lds(r)]);
#pragma unroll
    for (uint32_t r = 0; r < kEPT; ++r) dst[g(r)] = v[r];
  }
};

// ModUp fused with the column phases around it, per wavefront. Workgroup (digit j, item b, tile);
// every wavefront owns a group of the tile's columns: the digit's limbs (row phase of the inverse
// NTT already applied, in dc2 [B][nl][N]) go through the inverse column phase in LDS and are scaled
// to y_i = d_i Dhat_i^-1 mod q_i (N^-1 folded in), kept in registers; then for every limb t outside
// the digit the conversion sum_i y_i (Dhat_i mod t) mod t is formed (exact FP64 on Q primes,
// integer on special primes), goes through the forward column phase of t and is written to ext
// (layout as k_modup). No workgroup barrier; LDS holds one tile.
template <int LOG_E, int NT, int ALPHA, int K1>
__global__ __launch_bounds__(NT) void k_modup_cols(uint32_t B, uint32_t nl, uint32_t K, uint32_t nq, uint32_t alpha,
                                                  uint32_t R, uint32_t logN,
                                                  const ModInfo* __restrict__ mods, const double* __restrict__ twf,
                                                  const uint64_t* __restrict__ twi, const uint64_t* __restrict__ tab,
                                                  const uint64_t* __restrict__ dc2, uint64_t* __restrict__ ext) {
  constexpr uint32_t k1 = K1;  // column-phase stages (compile-time: round shapes and offsets fold)
  typedef ColSwz<K1> Lay;
  static_assert(LOG_E == 11 && NT == 256, "ColSwz assumes 2048-element tiles on 4 wavefronts");
  constexpr uint32_t E = 1u << LOG_E, EPT = E / NT;
  extern __shared__ uint64_t work[];
  const uint32_t N = 1u << logN, tiles = N >> LOG_E;
  const uint32_t tile = blockIdx.x % tiles, rest = blockIdx.x / tiles;
  const uint32_t b = rest % B, j = rest / B;
  const uint32_t next = nl + K, lo = j * alpha, cnt = min(alpha, nl - lo);
  const uint32_t k2 = logN - k1, logC = LOG_E - k1;
  const uint32_t wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const ColSlots<K1> cs(lane, wv, k2, tile);
  const uint64_t* blk = tab + (uint64_t)j * (2 * alpha + 2 * alpha * next);
  double y[ALPHA][EPT];
#pragma unroll
  for (uint32_t i = 0; i < ALPHA; ++i) {
    if (i >= cnt) {  // a short last digit: zero terms (their constants are zero too)
#pragma unroll
      for (uint32_t r = 0; r < EPT; ++r) y[i][r] = 0.0;
      continue;
    }
    const ModInfo m = mods[lo + i];
    FpArith ar;
    ar.init(m);
    const uint64_t* src = dc2 + ((uint64_t)b * nl + lo + i) * N;
    cs.load(work, src);  // row-phase output in internal FP64 form
    wave_sync();
    ntt_rounds<true, 1, FpArith, EPT, NT, true, Lay>(work, ar, twf + (uint64_t)(lo + i) * 4 * N + 2 * (uint64_t)N, k1,
                                                logC, 0, 0);
    const double c = (double)shoup_mul(m.n_inv, blk[2 * i], blk[2 * i + 1], m.q);
    const double cq = c / ar.q;
#pragma unroll
    for (uint32_t r = 0; r < EPT; ++r) {
      const double v = ar.mulc(ar.ld(work[cs.lds(r)]), c, cq);
      y[i][r] = v < 0.0 ? v + ar.q : v;  // [0, q_i)
    }
    wave_sync();
  }
  uint64_t* out = ext + ((uint64_t)j * B + b) * R * N;
#pragma unroll 1
  for (uint32_t row = 0; row < next - cnt; ++row) {
    const uint32_t e = row < lo ? row : row + cnt;
    const uint32_t mi = e < nl ? e : nq + (e - nl);
    const ModInfo m = mods[mi];
    const uint64_t* mrow = blk + 2 * alpha + 2 * (uint64_t)e;
    uint64_t* o = out + (uint64_t)row * N;
    if (e < nl) {
      FpArith ar;
      ar.init(m);
      double cw[ALPHA], cwq[ALPHA];
#pragma unroll
      for (uint32_t i = 0; i < ALPHA; ++i) {
        cw[i] = i < cnt ? (double)mrow[(uint64_t)i * 2 * next] : 0.0;
        cwq[i] = cw[i] * ar.qinv;
      }
#pragma unroll
      for (uint32_t r = 0; r < EPT; ++r) {
        double v = 0.0;
#pragma unroll
        for (uint32_t i = 0; i < ALPHA; ++i)
          if (i < cnt) v += ar.mulc(opaque(y[i][r]), cw[i], cwq[i]);
        work[cs.lds(r)] = ar.st(ar.red(v));
      }
      wave_sync();
      ntt_rounds<false, 1, FpArith, EPT, NT, true, Lay>(work, ar, twf + (uint64_t)mi * 4 * N, k1, logC, 0, 0);
      cs.store(o, work, [](uint64_t x) { return x; });  // internal FP64 form, read by the inner product
    } else {
      IntArith ar;
      ar.init(m);
      // constants of the digit's limbs (zero beyond cnt, so those terms vanish without a branch)
      uint64_t cw[ALPHA], cws[ALPHA];
#pragma unroll
      for (uint32_t i = 0; i < ALPHA; ++i) {
        cw[i] = i < cnt ? mrow[(uint64_t)i * 2 * next] : 0;
        cws[i] = i < cnt ? mrow[(uint64_t)i * 2 * next + 1] : 0;
      }
#pragma unroll
      for (uint32_t r = 0; r < EPT; ++r) {
        // lazy Shoup terms in [0, 2p) summed two at a time into [0, 4p), the forward butterflies'
        // input range (p < 2^61, so no sum wraps)
        uint64_t v = shoup_mul_lazy(f64_to_u52(opaque(y[0][r])), cw[0], cws[0], m.q);
#pragma unroll
        for (uint32_t i = 1; i < ALPHA; ++i) {
          const uint64_t t = shoup_mul_lazy(f64_to_u52(opaque(y[i][r])), cw[i], cws[i], m.q);
          v = (i == 1 ? v : (v >= ar.q2 ? v - ar.q2 : v)) + t;
        }
        work[cs.lds(r)] = v;
      }
      wave_sync();
      ntt_rounds<false, 1, IntArith, EPT, NT, true, Lay>(work, ar, twi + (uint64_t)mi * 4 * N, k1, logC, 0, 0);
      cs.store(o, work, [&ar](uint64_t x) { return ar.lds_out(x); });
    }
    wave_sync();
  }
}

// ModDown conversion fused with the column phases around it, per wavefront. Workgroup (item b,
// component c, tile): the K special-prime limbs of u (row phase of the inverse NTT already applied)
// go through the inverse column phase in LDS and are scaled to z_k = [u_(p_k) (P/p_k)^-1]_(p_k)
// (one Shoup product by N^-1 (P/p_k)^-1) and centred (z_k - p_k when z_k > (p_k - 1)/2), which
// accounts for the P mod q_i subtractions of k_moddown_conv. The centred z_k is kept in registers as two exact 30-bit
// halves (high part signed), so every Q limb's conversion sum_k zc_k (P/p_k mod q_i) is formed in
// exact FP64 from the constants c0 = (P/p_k) mod q_i and c1 = c0 2^30 mod q_i, goes through the
// forward column phase and is written to conv [B][2][nl][N] in the FP64 kernels' internal form.
template <int LOG_E, int NT, int KP, int K1>
__global__ __launch_bounds__(NT) void k_moddown_cols(uint32_t nl, uint32_t K, uint32_t nq, uint32_t logN,
                                                    const ModInfo* __restrict__ mods, const double* __restrict__ twf,
                                                    const uint64_t* __restrict__ twi, const uint64_t* __restrict__ tab,
                                                    const double* __restrict__ tabf, const uint64_t* __restrict__ u,
                                                    uint64_t* __restrict__ conv) {
  constexpr uint32_t k1 = K1;  // column-phase stages (compile-time: round shapes and offsets fold)
  typedef ColSwz<K1> Lay;
  static_assert(LOG_E == 11 && NT == 256, "ColSwz assumes 2048-element tiles on 4 wavefronts");
  constexpr uint32_t E = 1u << LOG_E, EPT = E / NT;
  extern __shared__ uint64_t work[];
  const uint32_t N = 1u << logN, tiles = N >> LOG_E;
  const uint32_t tile = blockIdx.x % tiles, bc = blockIdx.x / tiles;
  const uint32_t next = nl + K, k2 = logN - k1, logC = LOG_E - k1;
  const uint32_t wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const ColSlots<K1> cs(lane, wv, k2, tile);
  const uint64_t* tinv = tab + 2 * K + 2 * (uint64_t)K * nq + 3 * (uint64_t)nq;  // N^-1 (P/p_k)^-1 mod p_k
  int32_t zh[KP][EPT], zl[KP][EPT];
#pragma unroll
  for (uint32_t kk = 0; kk < KP; ++kk) {
    const ModInfo m = mods[nq + kk];
    const uint64_t half = (m.q - 1) / 2;
    IntArith ar;
    ar.init(m);
    const uint64_t* src = u + ((uint64_t)bc * next + nl + kk) * N;
    cs.load(work, src);
    wave_sync();
    ntt_rounds<true, 1, IntArith, EPT, NT, true, Lay>(work, ar, twi + (uint64_t)(nq + kk) * 4 * N + 2 * (uint64_t)N, k1,
                                                 logC, 0, 0);
#pragma unroll
    for (uint32_t r = 0; r < EPT; ++r) {
      const uint64_t z = shoup_mul(work[cs.lds(r)], tinv[2 * kk], tinv[2 * kk + 1], m.q);
      const int64_t zc = z > half ? (int64_t)z - (int64_t)m.q : (int64_t)z;
      zh[kk][r] = (int32_t)(zc >> 30);
      zl[kk][r] = (int32_t)(zc & 0x3FFFFFFF);
    }
    wave_sync();
  }
#pragma unroll 1
  for (uint32_t i = 0; i < nl; ++i) {
    const ModInfo m = mods[i];
    FpArith ar;
    ar.init(m);
    double c0[KP], c0q[KP], c1[KP], c1q[KP];
#pragma unroll
    for (uint32_t kk = 0; kk < KP; ++kk) {
      const double* f = tabf + 4 * ((uint64_t)kk * nq + i);
      c0[kk] = f[0];
      c0q[kk] = f[1];
      c1[kk] = f[2];
      c1q[kk] = f[3];
    }
#pragma unroll
    for (uint32_t r = 0; r < EPT; ++r) {
      // |zh|, zl < 2^30: each product's quotient estimate is off by at most 0.5 + 2^-22, so every
      // term is below 0.6 q_i in magnitude and the sum of 2K terms stays far below 2^53
      double acc = 0.0;
#pragma unroll
      for (uint32_t kk = 0; kk < KP; ++kk)
        acc += ar.mulc((double)(int32_t)opaque((uint32_t)zh[kk][r]), c1[kk], c1q[kk]) +
               ar.mulc((double)(int32_t)opaque((uint32_t)zl[kk][r]), c0[kk], c0q[kk]);
      work[cs.lds(r)] = ar.st(ar.red(acc));
    }
    wave_sync();
    ntt_rounds<false, 1, FpArith, EPT, NT, true, Lay>(work, ar, twf + (uint64_t)i * 4 * N, k1, logC, 0, 0);
    uint64_t* o = conv + ((uint64_t)bc * nl + i) * N;
    cs.store(o, work, [](uint64_t x) { return x; });  // internal FP64 form, read by the combine
    wave_sync();
  }
}

// tmp[bc] = the last limb of in[b] component c; with galois != NULL, multiplied by the one-hot mask
// tau_(galois[b])(base mask) on the fly (the mask multiply fused into rescale).
__global__ __launch_bounds__(kThreads) void k_copy_last(uint32_t B, uint32_t ncomp, uint32_t nl, uint32_t logN,
                                                       const ModInfo* __restrict__ mods,
                                                       const uint64_t* __restrict__ maskm,
                                                       const uint32_t* __restrict__ galois,
                                                       const uint64_t* const* __restrict__ in,
                                                       uint64_t* __restrict__ tmp) {
  const uint32_t N = 1u << logN;
  const uint64_t total = (uint64_t)B * ncomp << logN;
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < total; t += (uint64_t)gridDim.x * kThreads) {
    const uint32_t k = (uint32_t)t & (N - 1);
    const uint32_t bc = (uint32_t)(t >> logN), b = bc / ncomp, c = bc - b * ncomp;
    uint64_t v = gmem(in[b])[((uint64_t)c * nl + nl - 1) * N + k];
    if (galois) {
      const ModInfo m = mods[nl - 1];
      v = mont_mul(v, maskm[((uint64_t)(nl - 1) << logN) + automorph_src(k, galois[b], logN)], m.q, m.qinv);
    }
    tmp[t] = v;
  }
}

// w[bc][i] = centred(v) mod q_i, v = dropped limb in the coefficient domain; q_(nl-1) < q_i (descending chain).
__global__ __launch_bounds__(kThreads) void k_rescale_bcast(uint32_t BC, uint32_t nl, uint32_t logN,
                                                           const ModInfo* __restrict__ mods,
                                                           const uint64_t* __restrict__ tmp,
                                                           uint64_t* __restrict__ w) {
  const uint32_t N = 1u << logN, no = nl - 1;
  const uint64_t ql = mods[nl - 1].q;
  const uint64_t total = (uint64_t)BC * no << logN;
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < total; t += (uint64_t)gridDim.x * kThreads) {
    const uint32_t k = (uint32_t)t & (N - 1);
    const uint64_t r = t >> logN;
    const uint32_t i = (uint32_t)(r % no), bc = (uint32_t)(r / no);
    const uint64_t v = tmp[((uint64_t)bc << logN) + k];
    w[t] = v > (ql - 1) / 2 ? v + mods[i].q - ql : v;
  }
}

__global__ __launch_bounds__(kThreads) void k_rescale_combine(uint32_t B, uint32_t ncomp, uint32_t nl, uint32_t nq,
                                                             uint32_t logN, const ModInfo* __restrict__ mods,
                                                             const uint64_t* __restrict__ tab,
                                                             const uint64_t* const* __restrict__ in,
                                                             const uint64_t* __restrict__ w,
                                                             uint64_t* const* __restrict__ out) {
  const uint32_t N = 1u << logN, no = nl - 1;
  const uint64_t* inv = tab + 2 * (uint64_t)(nl - 1) * nq;
  const uint64_t total = (uint64_t)B * ncomp * no << logN;
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < total; t += (uint64_t)gridDim.x * kThreads) {
    const uint32_t k = (uint32_t)t & (N - 1);
    const uint64_t r = t >> logN;
    const uint32_t i = (uint32_t)(r % no);
    const uint32_t bc = (uint32_t)(r / no), b = bc / ncomp, c = bc - b * ncomp;
    const uint64_t q = mods[i].q;
    const uint64_t x = sub_mod(gmem(in[b])[((uint64_t)c * nl + i) * N + k], w[t], q);
    gmem(out[b])[((uint64_t)c * no + i) * N + k] = shoup_mul(x, inv[2 * i], inv[2 * i + 1], q);
  }
}

// Rescale, column part, per wavefront: per (polynomial bc, tile), the dropped limb (row phase of
// its INTT already applied, in tmp [BC][N]) goes through the inverse column phase mod q_l and N^-1
// and is centred (v' = v - q_l when v > (q_l - 1)/2), kept in registers; v' (|v'| < q_l/2 < q_i)
// then goes through the forward column phase of every remaining limb i; results in w [BC][nl-1][N].
template <int LOG_E, int NT, int K1>
__global__ __launch_bounds__(NT) void k_rescale_cols(uint32_t nl, uint32_t logN,
                                                    const ModInfo* __restrict__ mods, const double* __restrict__ twf,
                                                    const uint64_t* __restrict__ tmp, uint64_t* __restrict__ w) {
  constexpr uint32_t k1 = K1;  // column-phase stages (compile-time: round shapes and offsets fold)
  typedef ColSwz<K1> Lay;
  static_assert(LOG_E == 11 && NT == 256, "ColSwz assumes 2048-element tiles on 4 wavefronts");
  constexpr uint32_t E = 1u << LOG_E, EPT = E / NT;
  extern __shared__ uint64_t work[];
  const uint32_t N = 1u << logN, tiles = N >> LOG_E;
  const uint32_t tile = blockIdx.x % tiles, bc = blockIdx.x / tiles;
  const uint32_t no = nl - 1, k2 = logN - k1, logC = LOG_E - k1;
  const uint32_t wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const ColSlots<K1> cs(lane, wv, k2, tile);
  double vs[EPT];
  {
    const ModInfo m = mods[no];
    FpArith ar;
    ar.init(m);
    const uint64_t* src = tmp + ((uint64_t)bc << logN);
    cs.load(work, src);  // row-phase output in internal FP64 form
    wave_sync();
    ntt_rounds<true, 1, FpArith, EPT, NT, true, Lay>(work, ar, twf + (uint64_t)no * 4 * N + 2 * (uint64_t)N, k1, logC, 0,
                                                0);
    const double c = (double)m.n_inv, cq = c / ar.q;
#pragma unroll
    for (uint32_t r = 0; r < EPT; ++r) {
      double v = ar.mulc(ar.ld(work[cs.lds(r)]), c, cq);  // |v| <= 0.7 q_l
      v = v < 0.0 ? v + ar.q : v;                             // [0, q_l)
      vs[r] = v > 0.5 * (ar.q - 1.0) ? v - ar.q : v;          // centred
    }
    wave_sync();
  }
  for (uint32_t i = 0; i < no; ++i) {
    const ModInfo m = mods[i];
    FpArith ar;
    ar.init(m);
#pragma unroll
    for (uint32_t r = 0; r < EPT; ++r) {
      work[cs.lds(r)] = ar.st(vs[r]);
    }
    wave_sync();
    ntt_rounds<false, 1, FpArith, EPT, NT, true, Lay>(work, ar, twf + (uint64_t)i * 4 * N, k1, logC, 0, 0);
    uint64_t* o = w + ((uint64_t)bc * no + i) * N;
    cs.store(o, work, [](uint64_t x) { return x; });  // internal FP64 form, read by k_rescale_rows
    wave_sync();
  }
}

// Rescale, row part: per (polynomial bc = b * ncomp + c, remaining limb i, tile), the forward row
// phase of w in LDS fused with out = (in - w) q_l^-1 mod q_i (NTT domain), per wavefront.
template <int NT, int KR = 0>  // KR as in k_ntt
__global__ __launch_bounds__(NT) void k_rescale_rows(uint32_t ncomp, uint32_t nl, uint32_t nq, uint32_t logN,
                                                          uint32_t k1, const ModInfo* __restrict__ mods,
                                                          const double* __restrict__ twf,
                                                          const uint64_t* __restrict__ tab,
                                                          const uint64_t* __restrict__ maskm,
                                                          const uint32_t* __restrict__ galois,
                                                          const uint64_t* const* __restrict__ in,
                                                          const uint64_t* __restrict__ w,
                                                          uint64_t* const* __restrict__ out) {
  extern __shared__ uint64_t lds[];
  constexpr uint32_t kPer = kNttE / NT;
  const uint32_t N = 1u << logN, tiles = N >> kNttLogE, no = nl - 1;
  uint32_t bc, rest;
  xcd_split(gridDim.x / (no * tiles), bc, rest);  // polynomials innermost per XCD
  const uint32_t tile = rest % tiles, i = rest / tiles, b = bc / ncomp, c = bc - b * ncomp;
  const ModInfo m = mods[i];
  FpArith ar;
  ar.init(m);
  const uint32_t j0 = tile * kNttE, k = KR ? KR : logN - k1, logC = kNttLogE - k;
  const uint32_t wb = (threadIdx.x >> 6) * (kNttE / (NT / 64)), lane = threadIdx.x & 63;
  const uint64_t* src = w + ((uint64_t)bc * no + i) * N + j0;
#pragma unroll
  for (uint32_t r_ = 0; r_ < kPer; ++r_) {
    const uint32_t idx = wb + lane + r_ * 64;
    lds[pad_idx(idx)] = src[idx];  // internal FP64 form
  }
  wave_sync();
  ntt_rounds<false, 2, FpArith, kPer, NT, true>(lds, ar, twf + (uint64_t)i * 4 * N, k, logC, k1, j0);
  const uint64_t* inv = tab + 2 * ((uint64_t)no * nq + i);
  const auto x = gmem(in[b] + ((uint64_t)c * nl + i) * N + j0);
  const auto o = gmem(out[b] + ((uint64_t)c * no + i) * N + j0);
  const uint32_t ln = opaque(lane);
  const double iv = (double)inv[0], ivq = iv * ar.qinv;  // exact FP64 as in k_ntt_p2_combine
  // all loads first (as in k_ntt_p2_combine: `o` may alias the input as far as the compiler knows)
  uint64_t xv[kPer], mk[kPer];
#pragma unroll
  for (uint32_t r_ = 0; r_ < kPer; ++r_) {
    const uint32_t idx = wb + ln + r_ * 64;
    xv[r_] = x[idx];
    mk[r_] = galois ? maskm[((uint64_t)i << logN) + automorph_src(j0 + idx, galois[b], logN)] : 0;
  }
#pragma unroll
  for (uint32_t r_ = 0; r_ < kPer; ++r_) {
    const uint32_t idx = wb + ln + r_ * 64;
    // one-hot mask multiply fused in (mask in Montgomery form)
    const uint64_t xm = galois ? mont_mul(xv[r_], mk[r_], m.q, m.qinv) : xv[r_];
    const double v = ar.red(ar.mulc(u52_to_f64(xm) - ar.ld(lds[pad_idx(idx)]), iv, ivq));
    o[idx] = f64_to_u52(v < 0.0 ? v + ar.q : v);
  }
}

__global__ __launch_bounds__(kThreads) void k_mask_mul(uint32_t B, uint32_t nl, uint32_t logN,
                                                      const ModInfo* __restrict__ mods,
                                                      const uint64_t* __restrict__ maskm,
                                                      const uint64_t* const* __restrict__ in,
                                                      const uint32_t* __restrict__ galois,
                                                      uint64_t* const* __restrict__ out) {
  const uint32_t N = 1u << logN;
  const uint64_t total = (uint64_t)B << logN;
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < total; t += (uint64_t)gridDim.x * kThreads) {
    const uint32_t b = (uint32_t)(t >> logN), k = (uint32_t)t & (N - 1);
    const uint32_t ks = automorph_src(k, galois[b], logN);
    const auto s = gmem(in[b]);
    const auto d = gmem(out[b]);
    for (uint32_t i = 0; i < nl; ++i) {
      const ModInfo m = mods[i];
      const uint64_t mk = maskm[((uint64_t)i << logN) + ks];
      d[(uint64_t)i * N + k] = mont_mul(s[(uint64_t)i * N + k], mk, m.q, m.qinv);
      d[(uint64_t)(nl + i) * N + k] = mont_mul(s[(uint64_t)(nl + i) * N + k], mk, m.q, m.qinv);
    }
  }
}

// Grouped masked sums. Segment s: accumulator seg[4s] (at acc + seg[4s] * 2 nl N), entries
// [seg[4s+1], seg[4s+2]), and seg[4s+3] = 1 to overwrite the accumulator (first products of its
// group), 0 to add to it. acc[c][i][k] (+)= sum over the entries e of in[e][c][i][k] times the one-hot
// mask tau_(galois[e])(base mask) at limb i, coefficient k (NTT domain). All limbs are Q limbs
// (q < 2^50): the products are exact FP64 (FpArith::kacc, the mask as doubles, every term below
// 0.875 q) and the sums are reduced every four entries; the stored result is the residue in [0, q).
// One thread per (segment, limb, coefficient): both components share the mask word.
__global__ __launch_bounds__(kThreads) void k_mask_sum(uint32_t nseg, uint32_t nl, uint32_t logN,
                                                      const ModInfo* __restrict__ mods,
                                                      const uint64_t* __restrict__ maskf,
                                                      const uint32_t* __restrict__ seg,
                                                      const uint64_t* const* __restrict__ in,
                                                      const uint32_t* __restrict__ galois,
                                                      uint64_t* __restrict__ acc) {
  const uint32_t N = 1u << logN;
  const uint64_t per = (uint64_t)nl << logN;  // (limb, coefficient) positions per segment
  const uint64_t total = (uint64_t)nseg * per;
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < total; t += (uint64_t)gridDim.x * kThreads) {
    const uint32_t s = (uint32_t)(t / per);
    const uint64_t off = t - (uint64_t)s * per;
    const uint32_t i = (uint32_t)(off >> logN), k = (uint32_t)off & (N - 1);
    FpArith ar;
    ar.init(mods[i]);
    const uint32_t e0 = seg[4 * s + 1], e1 = seg[4 * s + 2];
    uint64_t* a = acc + (uint64_t)seg[4 * s] * 2 * per + off;
    double v0 = 0.0, v1 = 0.0;
    if (!seg[4 * s + 3]) {
      v0 = u52_to_f64(a[0]);
      v1 = u52_to_f64(a[per]);
    }
    const uint64_t* mrow = maskf + ((uint64_t)i << logN);
    uint32_t e = e0;
    // four entries per round (|sum| stays below q + 4 * 0.875 q < 2^53), loads issued first
    for (; e + 4 <= e1; e += 4) {
      uint64_t mk[4], x0[4], x1[4];
#pragma unroll
      for (uint32_t j = 0; j < 4; ++j) {
        const auto x = gmem(in[e + j] + off);
        mk[j] = mrow[automorph_src(k, galois[e + j], logN)];
        x0[j] = x[0];
        x1[j] = x[per];
      }
#pragma unroll
      for (uint32_t j = 0; j < 4; ++j) {
        v0 = ar.kacc(v0, u52_to_f64(x0[j]), mk[j]);
        v1 = ar.kacc(v1, u52_to_f64(x1[j]), mk[j]);
      }
      ar.kred(v0);
      ar.kred(v1);
    }
    for (; e < e1; ++e) {
      const uint64_t mk = mrow[automorph_src(k, galois[e], logN)];
      const auto x = gmem(in[e] + off);
      v0 = ar.kacc(v0, u52_to_f64(x[0]), mk);
      v1 = ar.kacc(v1, u52_to_f64(x[per]), mk);
    }
    a[0] = ar.kfinal(v0);
    a[per] = ar.kfinal(v1);
  }
}

// results[seg[3s]] += sum of contrib[b] for b in [seg[3s+1], seg[3s+2]), contributions given by
// pointer ([2][nl][N] each).
__global__ __launch_bounds__(kThreads) void k_accumulate_ptr(uint32_t nseg, uint32_t nl, uint32_t logN,
                                                            const ModInfo* __restrict__ mods,
                                                            const uint32_t* __restrict__ seg,
                                                            const uint64_t* const* __restrict__ contrib,
                                                            uint64_t* const* __restrict__ results) {
  const uint64_t per = (uint64_t)2 * nl << logN;
  const uint64_t total = (uint64_t)nseg * per;
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < total; t += (uint64_t)gridDim.x * kThreads) {
    const uint32_t s = (uint32_t)(t / per);
    const uint64_t off = t - (uint64_t)s * per;
    const uint64_t q = mods[(uint32_t)((off >> logN) % nl)].q;
    const uint32_t b0 = seg[3 * s + 1], b1 = seg[3 * s + 2];
    const auto res = gmem(results[seg[3 * s]]);
    uint64_t acc = res[off];
    for (uint32_t b = b0; b < b1; ++b) acc = add_mod(acc, gmem(contrib[b])[off], q);
    res[off] = acc;
  }
}

// x[i] = 0 for i < n (a kernel, so that it can be recorded in a graph).
__global__ __launch_bounds__(kThreads) void k_fill_zero(uint64_t n, uint64_t* __restrict__ x) {
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < n; t += (uint64_t)gridDim.x * kThreads) x[t] = 0;
}

// out[i] = the bits of (double)in[i] (residues below 2^53), i < n.
__global__ __launch_bounds__(kThreads) void k_to_f64_bits(uint64_t n, const uint64_t* __restrict__ in,
                                                         uint64_t* __restrict__ out) {
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < n; t += (uint64_t)gridDim.x * kThreads)
    out[t] = (uint64_t)__double_as_longlong((double)in[t]);
}

__global__ __launch_bounds__(kThreads) void k_accumulate(uint32_t nseg, uint32_t nl, uint32_t logN,
                                                        const ModInfo* __restrict__ mods,
                                                        const uint32_t* __restrict__ seg,
                                                        const uint64_t* __restrict__ contrib,
                                                        uint64_t* const* __restrict__ results) {
  const uint64_t per = (uint64_t)2 * nl << logN;
  const uint64_t total = (uint64_t)nseg * per;
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < total; t += (uint64_t)gridDim.x * kThreads) {
    const uint32_t s = (uint32_t)(t / per);
    const uint64_t off = t - (uint64_t)s * per;
    const uint32_t i = (uint32_t)((off >> logN) % nl);
    const uint64_t q = mods[i].q;
    const uint32_t b0 = seg[3 * s + 1], b1 = seg[3 * s + 2];
    const auto res = gmem(results[seg[3 * s]]);
    uint64_t acc = res[off];
    for (uint32_t b = b0; b < b1; ++b) acc = add_mod(acc, contrib[(uint64_t)b * per + off], q);
    res[off] = acc;
  }
}

__global__ __launch_bounds__(kThreads) void k_signed_to_limbs(const int64_t* __restrict__ v, uint32_t nlimbs,
                                                             uint32_t n_first, uint32_t p_base, uint32_t logN,
                                                             const ModInfo* __restrict__ mods,
                                                             uint64_t* __restrict__ out) {
  const uint64_t total = (uint64_t)nlimbs << logN;
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < total; t += (uint64_t)gridDim.x * kThreads) {
    const uint32_t e = (uint32_t)(t >> logN), k = (uint32_t)t & ((1u << logN) - 1);
    const uint64_t q = mods[e < n_first ? e : p_base + (e - n_first)].q;
    const int64_t x = v[k];
    const uint64_t ax = x < 0 ? (uint64_t)(-x) : (uint64_t)x;
    const uint64_t r = ax % q;
    out[t] = (x < 0 && r) ? q - r : r;
  }
}

__global__ __launch_bounds__(kThreads) void k_to_mont(uint64_t* __restrict__ x, uint32_t nlimbs, uint32_t n_first,
                                                     uint32_t p_base, uint32_t logN,
                                                     const ModInfo* __restrict__ mods) {
  const uint64_t total = (uint64_t)nlimbs << logN;
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < total; t += (uint64_t)gridDim.x * kThreads) {
    const uint32_t e = (uint32_t)(t >> logN);
    const ModInfo m = mods[e < n_first ? e : p_base + (e - n_first)];
    x[t] = mont_mul(x[t], m.r2, m.q, m.qinv);
  }
}

__global__ __launch_bounds__(kThreads) void k_keygen_digit(uint32_t nall, uint32_t nq, uint32_t logN,
                                                          const ModInfo* __restrict__ mods,
                                                          const uint64_t* __restrict__ a,
                                                          const uint64_t* __restrict__ s,
                                                          const uint64_t* __restrict__ e,
                                                          const uint64_t* __restrict__ sp,
                                                          const uint64_t* __restrict__ pfac,
                                                          uint64_t* __restrict__ bout, uint64_t* __restrict__ aout) {
  const uint64_t total = (uint64_t)nall << logN;
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < total; t += (uint64_t)gridDim.x * kThreads) {
    const uint32_t li = (uint32_t)(t >> logN);
    const ModInfo m = mods[li];
    const uint64_t as = mont_mul(mont_mul(a[t], s[t], m.q, m.qinv), m.r2, m.q, m.qinv);
    uint64_t b = sub_mod(e[t], as, m.q);
    const uint64_t f = pfac[li];
    if (f) b = add_mod(b, mont_mul(mont_mul(f, sp[t], m.q, m.qinv), m.r2, m.q, m.qinv), m.q);
    if (li < nq) {  // Q primes: the doubles' bits of the plain residues (FP64 key product)
      bout[t] = (uint64_t)__double_as_longlong((double)b);
      aout[t] = (uint64_t)__double_as_longlong((double)a[t]);
    } else {  // special primes: Montgomery form (integer key product)
      bout[t] = mont_mul(b, m.r2, m.q, m.qinv);
      aout[t] = mont_mul(a[t], m.r2, m.q, m.qinv);
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_square(uint32_t nall, uint32_t logN, const ModInfo* __restrict__ mods,
                                                    const uint64_t* __restrict__ s, uint64_t* __restrict__ s2) {
  const uint64_t total = (uint64_t)nall << logN;
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < total; t += (uint64_t)gridDim.x * kThreads) {
    const ModInfo m = mods[t >> logN];
    s2[t] = mont_mul(mont_mul(s[t], s[t], m.q, m.qinv), m.r2, m.q, m.qinv);
  }
}

__global__ __launch_bounds__(kThreads) void k_encrypt_combine(uint32_t nl, uint32_t logN,
                                                             const ModInfo* __restrict__ mods,
                                                             const uint64_t* __restrict__ a,
                                                             const uint64_t* __restrict__ em,
                                                             const uint64_t* __restrict__ s,
                                                             uint64_t* __restrict__ ct) {
  const uint64_t total = (uint64_t)nl << logN;
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < total; t += (uint64_t)gridDim.x * kThreads) {
    const ModInfo m = mods[t >> logN];
    const uint64_t as = mont_mul(mont_mul(a[t], s[t], m.q, m.qinv), m.r2, m.q, m.qinv);
    ct[t] = sub_mod(em[t], as, m.q);
    ct[total + t] = a[t];
  }
}

__global__ __launch_bounds__(kThreads) void k_decrypt_combine(uint32_t nl, uint32_t nlim, uint32_t logN,
                                                             const ModInfo* __restrict__ mods,
                                                             const uint64_t* __restrict__ ct,
                                                             const uint64_t* __restrict__ s,
                                                             uint64_t* __restrict__ mout) {
  const uint64_t total = (uint64_t)nlim << logN;
  const uint64_t c1off = (uint64_t)nl << logN;
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < total; t += (uint64_t)gridDim.x * kThreads) {
    const ModInfo m = mods[t >> logN];
    const uint64_t cs = mont_mul(mont_mul(ct[c1off + t], s[t], m.q, m.qinv), m.r2, m.q, m.qinv);
    mout[t] = add_mod(ct[t], cs, m.q);
  }
}

__global__ __launch_bounds__(kThreads) void k_add(uint32_t ncomp, uint32_t nl, uint32_t logN,
                                                 const ModInfo* __restrict__ mods, const uint64_t* __restrict__ a,
                                                 const uint64_t* __restrict__ b, uint64_t* __restrict__ out) {
  const uint64_t total = (uint64_t)ncomp * nl << logN;
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < total; t += (uint64_t)gridDim.x * kThreads) {
    const uint64_t q = mods[(t >> logN) % nl].q;
    out[t] = add_mod(a[t], b[t], q);
  }
}

// Throughput probe of the modular-product forms (a measurement hook, not a step of the method): every
// thread runs 8 independent chains of `iters` dependent products x <- x w mod q. kKind 0: the FP64
// product of the Q primes (FpArith::mulc), 1: the lazy Shoup product of the special primes, 2: the
// Montgomery product of the special primes' key words. The chains' ends are stored so that no
// product is dead code.
template <int kKind>
__global__ __launch_bounds__(kThreads) void k_bench_mulmod(uint32_t iters, uint64_t q, uint64_t qinv, uint64_t w,
                                                         uint64_t wx, uint64_t* __restrict__ out) {
  const uint64_t gid = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
  if (kKind == 0) {
    FpArith ar;
    ar.q = (double)q;
    ar.qinv = 1.0 / ar.q;
    const double wd = (double)w, wq = wd / ar.q;
    double x[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = (double)((gid * 8 + c) % q);
    for (uint32_t i = 0; i < iters; ++i)
#pragma unroll
      for (int c = 0; c < 8; ++c) x[c] = ar.mulc(x[c], wd, wq);
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) acc += x[c];
    out[gid] = (uint64_t)__double_as_longlong(acc);
  } else {
    uint64_t x[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = (gid * 8 + c) % q;
    for (uint32_t i = 0; i < iters; ++i)
#pragma unroll
      for (int c = 0; c < 8; ++c) x[c] = kKind == 1 ? shoup_mul_lazy(x[c], w, wx, q) : mont_mul(x[c], w, q, qinv);
    uint64_t acc = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) acc ^= x[c];
    out[gid] = acc;
  }
}

}  // namespace

// ------------------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------------------

static const ModInfo* mods_of(const fhe_ctx* ctx) { return (const ModInfo*)ctx->t.mods.get(); }

static void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) fail(FHE_EDEVICE, std::string("kernel launch failed (") + what + "): " + hipGetErrorString(e));
}

// Launch with optional event timing; `bytes` is the kernel's algorithmic HBM traffic for this launch.
// `ops` is the launch's count of modular products (see prof_end), 0 where it is not counted.
#define FHE_LAUNCH_TO(name, bytes, ops, kern, grid, threads, lds, st, ...)      \
  do {                                                                           \
    const int tok_ = prof_begin(name, st);                                       \
    hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), lds, st, __VA_ARGS__);  \
    prof_end(tok_, st, (double)(bytes), (double)(ops));                          \
    check_launch(name);                                                          \
  } while (0)
#define FHE_LAUNCH_T(name, bytes, kern, grid, threads, lds, st, ...) \
  FHE_LAUNCH_TO(name, bytes, 0.0, kern, grid, threads, lds, st, __VA_ARGS__)
#define FHE_LAUNCH(name, bytes, kern, grid, lds, st, ...) \
  FHE_LAUNCH_T(name, bytes, kern, grid, kThreads, lds, st, __VA_ARGS__)

static void check_batch(const fhe_ctx* ctx, const LimbBatch& lb) {
  const Params& p = ctx->p;
  uint32_t last = lb.limbs - 1;
  uint32_t mi = last < lb.n_first ? last : lb.p_base + (last - lb.n_first);
  uint32_t mi0 = 0 < lb.n_first ? 0 : lb.p_base;
  if (mi >= (uint32_t)p.nmod() || mi0 >= (uint32_t)p.nmod()) fail(FHE_EINVAL, "NTT batch modulus index out of range");
}

static uint32_t ntt_blocks(const fhe_ctx* ctx, const LimbBatch& lb) {
  const uint64_t blocks = (uint64_t)(ctx->p.N >> kNttLogE) * lb.limbs * lb.npoly;
  if (blocks >= (1ull << 31)) fail(FHE_EINVAL, "NTT batch too large");
  return (uint32_t)blocks;
}

// Launches one phase of the transform over a batch. Limbs [0, n_first) use moduli 0.., the others
// p_base..; each part runs the kernel for its moduli class (FP64 for Q primes, integer for P primes).
// Launches one phase of the transform over a batch, split into runs of limbs whose moduli are all Q
// primes (FP64 kernel) or all special primes (integer kernel):
//   rows [0, qa)             -> moduli 0.. (with the digit hole, if any), Q primes;
//   rows [qa, min(n_first))  -> moduli qa.., special primes (batches that index the whole chain);
//   rows [n_first, limbs)    -> moduli p_base.., Q or special primes.
template <bool kInv, int kPhase>
static void ntt_phase(const fhe_ctx* ctx, const LimbBatch& lb, const char* name_q, const char* name_p, bool from_src,
                      hipStream_t st) {
  const Params& p = ctx->p;
  const size_t lds = kNttLdsElems * sizeof(uint64_t);
  const uint32_t nq = (uint32_t)p.nq;
  const double* twf = (const double*)ctx->t.twf.get();
  const uint32_t nf = std::min(lb.n_first, lb.limbs);
  const uint32_t qa = lb.hole_items ? nf : std::min(nf, nq);
  struct Run {
    uint32_t lo, hi;
    bool q;
  };
  Run runs[3] = {{0, qa, true}, {qa, nf, false}, {nf, lb.limbs, lb.p_base + (lb.limbs - nf) <= nq}};
  if (nf < lb.limbs && !runs[2].q && lb.p_base < nq) fail(FHE_EINVAL, "NTT batch mixes Q and P moduli in its tail");
  for (int part = 0; part < 3; ++part) {
    const Run& r = runs[part];
    if (r.hi <= r.lo) continue;
    LimbBatch sub = lb;
    sub.base = lb.base + (uint64_t)r.lo * p.N;
    if (sub.src) sub.src = lb.src + (uint64_t)r.lo * p.N;
    if (sub.src_ptr) sub.src_ptr_limb0 = lb.src_ptr_limb0 + r.lo;
    sub.limbs = r.hi - r.lo;
    if (part == 0) {
      sub.n_first = sub.limbs;
    } else {
      sub.n_first = 0;
      sub.hole_items = 0;
      sub.p_base = part == 1 ? r.lo : lb.p_base;
    }
    const uint32_t blocks = ntt_blocks(ctx, sub);
    const double bytes = 16.0 * p.N * sub.limbs * sub.npoly;
    // butterflies of the phase's stages (plus the N^-1 scaling of the inverse column phase)
    const double ops = (double)sub.limbs * sub.npoly * p.N *
                       (0.5 * (kPhase == 1 ? p.k1 : p.logN - p.k1) + (kInv && kPhase == 1 ? 1.0 : 0.0));
    // row phase: 512 threads x 8 elements (3-stage rounds; about 66 VGPRs, three workgroups per CU)
    // or 256 x 16 (p.rows_nt); column phase: 256 threads x 16 elements
    // the usual row length (2^9): compile-time rounds (fewer VGPRs, a fourth workgroup per CU; the
    // forward gather instance is left out, it would need more)
    const bool r9 = p.logN - p.k1 == 9;
    if (kPhase == 2 && from_src && sub.src_ptr) {
      if (r.q && r9 && kInv)
        FHE_LAUNCH_TO(name_q, bytes, ops, (k_ntt<kInv, kPhase, FpArith, 512, true, 9>), blocks, 512, lds, st, sub,
                     mods_of(ctx), twf, p.logN, p.k1, from_src);
      else if (r.q)
        FHE_LAUNCH_TO(name_q, bytes, ops, (k_ntt<kInv, kPhase, FpArith, 512, true>), blocks, 512, lds, st, sub, mods_of(ctx),
                     twf, p.logN, p.k1, from_src);
      else
        FHE_LAUNCH_TO(name_p, bytes, ops, (k_ntt<kInv, kPhase, IntArith, 512, true>), blocks, 512, lds, st, sub,
                     mods_of(ctx), ctx->t.tw.u64(), p.logN, p.k1, from_src);
    } else if (kPhase == 2 && p.rows_nt == 512) {
      if (r.q && r9)
        FHE_LAUNCH_TO(name_q, bytes, ops, (k_ntt<kInv, kPhase, FpArith, 512, false, 9>), blocks, 512, lds, st, sub,
                     mods_of(ctx), twf, p.logN, p.k1, from_src);
      else if (r.q)
        FHE_LAUNCH_TO(name_q, bytes, ops, (k_ntt<kInv, kPhase, FpArith, 512>), blocks, 512, lds, st, sub, mods_of(ctx), twf,
                     p.logN, p.k1, from_src);
      else if (r9)
        FHE_LAUNCH_TO(name_p, bytes, ops, (k_ntt<kInv, kPhase, IntArith, 512, false, 9>), blocks, 512, lds, st, sub,
                     mods_of(ctx), ctx->t.tw.u64(), p.logN, p.k1, from_src);
      else
        FHE_LAUNCH_TO(name_p, bytes, ops, (k_ntt<kInv, kPhase, IntArith, 512>), blocks, 512, lds, st, sub, mods_of(ctx),
                     ctx->t.tw.u64(), p.logN, p.k1, from_src);
    } else {
      if (r.q)
        FHE_LAUNCH_TO(name_q, bytes, ops, (k_ntt<kInv, kPhase, FpArith, kThreads>), blocks, kThreads, lds, st, sub,
                      mods_of(ctx), twf,
                   p.logN, p.k1, from_src);
      else
        FHE_LAUNCH_TO(name_p, bytes, ops, (k_ntt<kInv, kPhase, IntArith, kThreads>), blocks, kThreads, lds, st, sub,
                      mods_of(ctx),
                   ctx->t.tw.u64(), p.logN, p.k1, from_src);
    }
  }
}

static void check_holes(const fhe_ctx* ctx, const LimbBatch& lb) {
  if (lb.hole_items && lb.n_first + lb.hole_len > (uint32_t)ctx->p.nq)
    fail(FHE_EINVAL, "NTT batch digit rows exceed the Q chain");
}

static void ntt_forward_cols(const fhe_ctx* ctx, const LimbBatch& lb, hipStream_t st) {
  if (lb.limbs == 0 || lb.npoly == 0) return;
  if (lb.src_ptr) fail(FHE_EINVAL, "automorphism reads are only for row phases");
  check_batch(ctx, lb);
  check_holes(ctx, lb);
  ntt_phase<false, 1>(ctx, lb, "ntt_fwd_p1_q", "ntt_fwd_p1_p", lb.src != nullptr, st);
}

void ntt_forward(const fhe_ctx* ctx, const LimbBatch& lb, hipStream_t st) {
  if (lb.limbs == 0 || lb.npoly == 0) return;
  if (lb.src_ptr) fail(FHE_EINVAL, "automorphism reads are only for row phases");
  check_batch(ctx, lb);
  check_holes(ctx, lb);
  ntt_phase<false, 1>(ctx, lb, "ntt_fwd_p1_q", "ntt_fwd_p1_p", lb.src != nullptr, st);
  ntt_phase<false, 2>(ctx, lb, "ntt_fwd_p2_q", "ntt_fwd_p2_p", false, st);
}

// Row phase of the inverse transform only (the column phase is fused into a consumer). The timer
// names default to the key switch's; the rescale passes its own.
static void ntt_inverse_rows(const fhe_ctx* ctx, const LimbBatch& lb, hipStream_t st, const char* name_q = "ntt_inv_p2_q",
                             const char* name_p = "ntt_inv_p2_p") {
  if (lb.limbs == 0 || lb.npoly == 0) return;
  check_batch(ctx, lb);
  check_holes(ctx, lb);
  ntt_phase<true, 2>(ctx, lb, name_q, name_p, lb.src != nullptr || lb.src_ptr != nullptr, st);
}

void ntt_inverse(const fhe_ctx* ctx, const LimbBatch& lb, hipStream_t st) {
  if (lb.limbs == 0 || lb.npoly == 0) return;
  if (lb.raw_out) fail(FHE_EINVAL, "internal-form output is only for row phases of inverse transforms");
  check_batch(ctx, lb);
  check_holes(ctx, lb);
  ntt_phase<true, 2>(ctx, lb, "ntt_inv_p2_q", "ntt_inv_p2_p", lb.src != nullptr || lb.src_ptr != nullptr, st);
  LimbBatch cols = lb;  // the column phase works in place on the row phase's output
  cols.src_ptr = nullptr;
  ntt_phase<true, 1>(ctx, cols, "ntt_inv_p1_q", "ntt_inv_p1_p", false, st);
}

void automorph(const fhe_ctx* ctx, uint32_t B, uint32_t ncomp, uint32_t nl, const uint64_t* const* src,
               const uint32_t* galois, uint64_t* dst, hipStream_t st) {
  if (!B) return;
  const double bytes = 16.0 * B * ncomp * nl * ctx->p.N;
  FHE_LAUNCH("automorph", bytes, k_automorph, grid_for((uint64_t)B << ctx->p.logN), 0, st, B, ncomp, nl, ctx->p.logN,
             src, galois, dst);
}

void tensor(const fhe_ctx* ctx, uint32_t B, uint32_t nl, const uint64_t* const* a, const uint64_t* const* b,
            uint64_t* out, hipStream_t st) {
  if (!B) return;
  const double bytes = 8.0 * 7 * B * nl * ctx->p.N;
  FHE_LAUNCH("tensor", bytes, k_tensor, grid_for((uint64_t)B * nl << ctx->p.logN), 0, st, B, nl, ctx->p.logN,
             mods_of(ctx), a, b, out);
}

// Rows per digit in the compacted ModUp buffer: next - (size of the last, possibly truncated, digit).
static uint32_t modup_rows(const Params& p, uint32_t nl) {
  const uint32_t beta = p.beta(nl), cnt_last = nl - (beta - 1) * p.alpha;
  return nl + p.np - cnt_last;
}

// Fused column-phase kernels (ModUp, ModDown, rescale): 2048-element tiles on 256 threads (8
// elements per thread), instantiated for column phases of k1 = 6, 7, 8 stages.
static uint32_t cols_log_e(const Params&) { return 11; }

static size_t cols_lds_bytes(uint32_t log_e) {
  const size_t E = (size_t)1 << log_e;
  return (E + (E >> 4)) * sizeof(uint64_t);
}

static size_t max_lds_per_block(int device) {
  static size_t cached[64] = {0};
  if (device < 0 || device >= 64) return 65536;
  if (!cached[device]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess || v <= 0) v = 65536;
    cached[device] = (size_t)v;
  }
  return cached[device];
}

// The fused column kernels keep at most 4 digit limbs / special primes in registers and are
// compiled for k1 in [6, 8]; other parameter sets take the unfused sequence.
static bool cols_fusable(const fhe_ctx* ctx, uint32_t regs_needed) {
  const Params& p = ctx->p;
  if (regs_needed > 4 || p.k1 < 6 || p.k1 > 8) return false;
  return cols_lds_bytes(cols_log_e(p)) <= max_lds_per_block(ctx->device);
}

static void keyswitch_moddown(const fhe_ctx* ctx, uint32_t B, uint32_t nl, uint64_t* u, uint64_t* conv,
                              const uint64_t* const* add, const uint32_t* galois, uint64_t* const* out,
                              hipStream_t st);

// Steps 1-3 of the key switch for B inputs (contiguous `in` with in_stride, or in_ptrs read through
// galois): INTT into dcoef, ModUp of every digit, column phase of the extended rows into ext
// ([beta][B][R][N], raw form).
static void keyswitch_modup(const fhe_ctx* ctx, uint32_t B, uint32_t nl, const uint64_t* in, uint64_t in_stride,
                            const uint64_t* const* in_ptrs, const uint32_t* galois, uint64_t* dcoef, uint64_t* ext,
                            hipStream_t st) {
  const Params& p = ctx->p;
  const uint32_t N = p.N, K = p.np, next = nl + K, beta = p.beta(nl), alpha = p.alpha;
  const uint32_t R = modup_rows(p, nl), cnt_last = nl - (beta - 1) * alpha;
  const uint32_t beta_full = cnt_last == alpha ? beta : beta - 1;
  const double e8 = 8.0 * N * B;
  // 1. INTT of the input into dcoef (the NTT-domain input is kept for the digits' own limbs).
  LimbBatch lb_in{dcoef, nl, B, (uint64_t)nl * N, nl, 0};
  lb_in.src = in;
  lb_in.src_stride = in_stride;
  if (in_ptrs) {
    lb_in.src_ptr = in_ptrs;
    lb_in.src_gal = galois;
  }
  if (cols_fusable(ctx, alpha)) {
    // 1-3 fused: row phase of the INTT here, then one kernel for the column phases and ModUp.
    LimbBatch lb_rows = lb_in;
    lb_rows.raw_out = 1;
    ntt_inverse_rows(ctx, lb_rows, st);
    const uint32_t le = cols_log_e(p);
    const size_t lds_mu = cols_lds_bytes(le);
    const uint64_t grid = (uint64_t)B * beta * (N >> le);
    if (grid >= (1ull << 31)) fail(FHE_EINVAL, "key-switch batch too large");
    const double bytes = e8 * beta * (double)next;  // nl digit rows read, beta * next - nl rows written
    // per digit: inverse column phase and scaling of its limbs, conversion to and forward column
    // phase of every other limb
    double ops = 0.0;
    for (uint32_t j = 0; j < beta; ++j) {
      const double cnt = (double)std::min(alpha, nl - j * alpha), h = 0.5 * N * p.k1;
      ops += cnt * (h + N) + ((double)next - cnt) * (cnt * N + h);
    }
    ops *= B;
    const uint64_t* mtab = ctx->t.modup.u64() + ctx->t.modup_offset[nl];
    const double* twf0 = (const double*)ctx->t.twf.get();
#define FHE_MODUP_COLS(AL, K1)                                                                                  \
  FHE_LAUNCH_TO("modup_cols", bytes, ops, (k_modup_cols<11, 256, AL, K1>), grid, 256, lds_mu, st, B, nl, K,      \
               (uint32_t)p.nq, alpha, R, p.logN, mods_of(ctx), twf0, ctx->t.tw.u64(), mtab, dcoef, ext)
#define FHE_MODUP_COLS_K(AL)          \
  switch (p.k1) {                     \
    case 6: FHE_MODUP_COLS(AL, 6); break; \
    case 7: FHE_MODUP_COLS(AL, 7); break; \
    default: FHE_MODUP_COLS(AL, 8); break; \
  }
    switch (alpha) {
      case 1: FHE_MODUP_COLS_K(1); break;
      case 2: FHE_MODUP_COLS_K(2); break;
      case 3: FHE_MODUP_COLS_K(3); break;
      default: FHE_MODUP_COLS_K(4); break;
    }
#undef FHE_MODUP_COLS_K
#undef FHE_MODUP_COLS
  } else {
    ntt_inverse(ctx, lb_in, st);
    // 2. ModUp: the limbs outside each digit.
    FHE_LAUNCH("modup", e8 * (nl + beta * (next - alpha)), k_modup, grid_for((uint64_t)B * beta * N), 0, st, B, nl,
               K, (uint32_t)p.nq, alpha, R, p.logN, mods_of(ctx), ctx->t.modup.u64() + ctx->t.modup_offset[nl],
               dcoef, ext);
    // 3. Column phase of the NTT of the extended rows (full digits, then a truncated last digit).
    if (beta_full) {
      LimbBatch lb{ext, next - alpha, beta_full * B, (uint64_t)R * N, nl - alpha, (uint32_t)p.nq};
      lb.hole_items = B;
      lb.hole_alpha = alpha;
      lb.hole_len = alpha;
      lb.hole_j0 = 0;
      lb.raw_out = 1;
      ntt_forward_cols(ctx, lb, st);
    }
    if (beta_full < beta) {
      LimbBatch lb{ext + (size_t)beta_full * B * R * N, next - cnt_last, B, (uint64_t)R * N, nl - cnt_last,
                   (uint32_t)p.nq};
      lb.hole_items = B;
      lb.hole_alpha = alpha;
      lb.hole_len = cnt_last;
      lb.hole_j0 = beta_full;
      lb.raw_out = 1;
      ntt_forward_cols(ctx, lb, st);
    }
  }
}

size_t keyswitch_ws_elems(const fhe_ctx* ctx, uint32_t B, uint32_t nl) {
  const Params& p = ctx->p;
  const size_t N = p.N, next = nl + p.np, beta = p.beta(nl), R = modup_rows(p, nl);
  return (size_t)B * N * (nl + beta * R + 2 * next + 2 * nl);
}

void keyswitch(const fhe_ctx* ctx, uint32_t B, uint32_t nl, const uint64_t* in, uint64_t in_stride,
               const uint64_t* const* keys, const uint64_t* const* add, uint64_t* const* out, uint64_t* ws,
               hipStream_t st, const uint32_t* galois, const uint64_t* const* in_ptrs) {
  if (!B) return;
  if (in_ptrs && !galois) fail(FHE_EINVAL, "key switch input pointers need their Galois elements");
  const Params& p = ctx->p;
  if (p.alpha > kMaxAlpha || p.np > kMaxK) fail(FHE_EINVAL, "alpha or n_p above kernel limits");
  if (nl < 1 || nl > (uint32_t)p.nq) fail(FHE_ESHAPE, "key switch level out of range");
  prof_count("keyswitch", B);
  prof_count(("keyswitch_nl" + std::to_string(nl)).c_str(), B);
  const uint32_t N = p.N, K = p.np, next = nl + K, beta = p.beta(nl), alpha = p.alpha;
  const uint32_t R = modup_rows(p, nl);
  uint64_t* dcoef = ws;                                 // [B][nl][N]
  uint64_t* ext = dcoef + (size_t)B * nl * N;           // [beta][B][R][N]
  uint64_t* u = ext + (size_t)beta * B * R * N;         // [B][2][next][N]
  uint64_t* conv = u + (size_t)B * 2 * next * N;        // [B][2][nl][N]
  keyswitch_modup(ctx, B, nl, in, in_stride, in_ptrs, galois, dcoef, ext, st);
  // 4. Row phase fused with the key inner product (Q limbs on the FP64 path, P limbs on the integer path).
  const size_t lds = kNttLdsElems * sizeof(uint64_t);
  const uint32_t tiles = N >> kNttLogE;
  if ((uint64_t)B * next * tiles >= (1ull << 31)) fail(FHE_EINVAL, "key-switch batch too large");
  const double* twf = (const double*)ctx->t.twf.get();
  // per extended limb: beta digit words (input or ModUp row), 2 beta key words, 2 output words
  const double ib = 8.0 * N * (double)B * (3.0 * beta + 2.0);
  const uint32_t* in_gal = in_ptrs ? galois : nullptr;
  // per Q limb: two key products per digit and the row phase of every digit's row but its own; per
  // special-prime limb: both for every digit
  const double hrow = 0.5 * N * (p.logN - p.k1);
  const double ops_q = (double)B * nl * (2.0 * N * beta + hrow * (beta - 1));
  const double ops_p = (double)B * K * beta * (2.0 * N + hrow);
  if (in_ptrs)
    FHE_LAUNCH_TO("ntt_p2_inner_q", ib * nl, ops_q, (k_ntt_p2_inner<FpArith, true>), (uint64_t)B * nl * tiles,
                  kInnerThreads,
                 lds, st, B, nl, K, (uint32_t)p.nq, alpha, R, 0u, nl, p.logN, p.k1, mods_of(ctx), twf, in, in_stride,
                 in_ptrs, in_gal, ext, keys, u);
  else
    FHE_LAUNCH_TO("ntt_p2_inner_q", ib * nl, ops_q, (k_ntt_p2_inner<FpArith, false>), (uint64_t)B * nl * tiles,
                  kInnerThreads,
                 lds, st, B, nl, K, (uint32_t)p.nq, alpha, R, 0u, nl, p.logN, p.k1, mods_of(ctx), twf, in, in_stride,
                 in_ptrs, in_gal, ext, keys, u);
  FHE_LAUNCH_TO("ntt_p2_inner_p", ib * K, ops_p, (k_ntt_p2_inner<IntArith, false>), (uint64_t)B * K * tiles,
                kInnerThreads, lds,
               st, B, nl, K, (uint32_t)p.nq, alpha, R, nl, K, p.logN, p.k1, mods_of(ctx), ctx->t.tw.u64(), in,
               in_stride, nullptr, nullptr, ext, keys, u);
  keyswitch_moddown(ctx, B, nl, u, conv, add, galois, out, st);
}

void keyswitch_hoisted(const fhe_ctx* ctx, uint32_t S, uint32_t B, uint32_t nl, const uint64_t* const* state_c1,
                       const uint32_t* ident, const uint32_t* state_of, const uint64_t* const* in_ptrs,
                       const uint32_t* galois, const uint64_t* const* keys, const uint64_t* const* add,
                       uint64_t* const* out, uint64_t* ws, hipStream_t st) {
  if (!B) return;
  const Params& p = ctx->p;
  if (S < 1 || S > B) fail(FHE_EINVAL, "hoisted key switch needs 1 <= S <= B polynomials");
  if (p.alpha > kMaxAlpha || p.np > kMaxK) fail(FHE_EINVAL, "alpha or n_p above kernel limits");
  if (nl < 1 || nl > (uint32_t)p.nq) fail(FHE_ESHAPE, "key switch level out of range");
  prof_count("keyswitch", B);
  prof_count(("keyswitch_nl" + std::to_string(nl)).c_str(), B);
  const uint32_t N = p.N, K = p.np, next = nl + K, beta = p.beta(nl), alpha = p.alpha;
  const uint32_t R = modup_rows(p, nl), cnt_last = nl - (beta - 1) * alpha;
  uint64_t* dcoef = ws;                                 // [S][nl][N] within the B-item layout
  uint64_t* ext = dcoef + (size_t)B * nl * N;           // [beta][S][R][N]
  uint64_t* u = ext + (size_t)beta * B * R * N;         // [B][2][next][N]
  uint64_t* conv = u + (size_t)B * 2 * next * N;        // [B][2][nl][N]
  // ModUp of every polynomial once (no automorphism), then the row phase of its digits in place
  keyswitch_modup(ctx, S, nl, nullptr, 0, state_c1, ident, dcoef, ext, st);
  const size_t lds = kNttLdsElems * sizeof(uint64_t);
  const uint32_t tiles = N >> kNttLogE, qrows = nl - cnt_last;
  const double* twf = (const double*)ctx->t.twf.get();
  const double e8s = 8.0 * N * S;
  if (qrows)
    FHE_LAUNCH_T("ext_rows_q", 16.0 * N * S * beta * qrows, (k_ext_rows<FpArith, true>),
                 (uint64_t)beta * S * qrows * tiles, kInnerThreads, lds, st, S, nl, K, (uint32_t)p.nq, alpha, R, qrows,
                 p.logN, p.k1, mods_of(ctx), twf, ext);
  FHE_LAUNCH_T("ext_rows_p", 2.0 * e8s * beta * K, (k_ext_rows<IntArith, false>), (uint64_t)beta * S * K * tiles,
               kInnerThreads, lds, st, S, nl, K, (uint32_t)p.nq, alpha, R, K, p.logN, p.k1, mods_of(ctx),
               ctx->t.tw.u64(), ext);
  // every rotation: the inner product through its automorphism, then ModDown as usual
  const uint32_t htiles = N / (kThreads * 8);
  const double ib = 8.0 * N * (double)B * (3.0 * beta + 2.0);
  FHE_LAUNCH("hoisted_inner_q", ib * nl, k_hoisted_inner<FpArith>, (uint64_t)B * nl * htiles, 0, st, B, S, nl, K,
             (uint32_t)p.nq, alpha, R, 0u, nl, p.logN, mods_of(ctx), state_of, galois, in_ptrs, ext, keys, u);
  FHE_LAUNCH("hoisted_inner_p", ib * K, k_hoisted_inner<IntArith>, (uint64_t)B * K * htiles, 0, st, B, S, nl, K,
             (uint32_t)p.nq, alpha, R, nl, K, p.logN, mods_of(ctx), state_of, galois, in_ptrs, ext, keys, u);
  keyswitch_moddown(ctx, B, nl, u, conv, add, galois, out, st);
}

// ModDown of the inner products u ([B][2][next][N]) into out, plus the addends (see keyswitch).
static void keyswitch_moddown(const fhe_ctx* ctx, uint32_t B, uint32_t nl, uint64_t* u, uint64_t* conv,
                              const uint64_t* const* add, const uint32_t* galois, uint64_t* const* out,
                              hipStream_t st) {
  const Params& p = ctx->p;
  const uint32_t N = p.N, K = p.np, next = nl + K;
  const double e8 = 8.0 * N * B;
  const size_t lds = kNttLdsElems * sizeof(uint64_t);
  const uint32_t tiles = N >> kNttLogE;
  const double* twf = (const double*)ctx->t.twf.get();
  // 5. ModDown: INTT of the P limbs, conversion to Q_l, column phase, row phase fused with the combine.
  const LimbBatch lb_up{u + (size_t)nl * N, K, 2 * B, (uint64_t)next * N, 0, (uint32_t)p.nq};
  if (cols_fusable(ctx, K)) {
    ntt_inverse_rows(ctx, lb_up, st);
    const uint32_t le = cols_log_e(p);
    const size_t lds_md = cols_lds_bytes(le);
    const uint64_t grid = (uint64_t)2 * B * (N >> le);
    const double bytes = e8 * 2 * (K + nl);
    // per component: inverse column phase and scaling of the K special-prime limbs, the two-part
    // conversion into and the forward column phase of every Q limb
    const double h1 = 0.5 * N * p.k1;
    const double ops = 2.0 * B * (K * (h1 + N) + (double)nl * (2.0 * K * N + h1));
    const double* twf0 = (const double*)ctx->t.twf.get();
#define FHE_MODDOWN_COLS(KP, K1)                                                                            \
  FHE_LAUNCH_TO("moddown_cols", bytes, ops, (k_moddown_cols<11, 256, KP, K1>), grid, 256, lds_md, st, nl, K, \
               (uint32_t)p.nq, p.logN, mods_of(ctx), twf0, ctx->t.tw.u64(), ctx->t.moddown.u64(),                 \
               (const double*)ctx->t.moddown_f.get(), u, conv)
#define FHE_MODDOWN_COLS_K(KP)             \
  switch (p.k1) {                          \
    case 6: FHE_MODDOWN_COLS(KP, 6); break; \
    case 7: FHE_MODDOWN_COLS(KP, 7); break; \
    default: FHE_MODDOWN_COLS(KP, 8); break; \
  }
    switch (K) {
      case 1: FHE_MODDOWN_COLS_K(1); break;
      case 2: FHE_MODDOWN_COLS_K(2); break;
      case 3: FHE_MODDOWN_COLS_K(3); break;
      default: FHE_MODDOWN_COLS_K(4); break;
    }
#undef FHE_MODDOWN_COLS_K
#undef FHE_MODDOWN_COLS
  } else {
    ntt_inverse(ctx, lb_up, st);
    FHE_LAUNCH("moddown_conv", e8 * 2 * (K + nl), k_moddown_conv, grid_for((uint64_t)B * 2 * N), 0, st, B, nl, K,
               (uint32_t)p.nq, p.logN, mods_of(ctx), ctx->t.moddown.u64(), u, conv);
    LimbBatch lb_conv{conv, nl, 2 * B, (uint64_t)nl * N, nl, 0};
    lb_conv.raw_out = 1;
    ntt_forward_cols(ctx, lb_conv, st);
  }
  // row phase of every converted Q limb and its product by P^-1
  const double ops_c = 2.0 * B * nl * (0.5 * N * (p.logN - p.k1) + N);
  if (p.rows_nt == 512 && p.logN - p.k1 == 9)
    FHE_LAUNCH_TO("ntt_p2_combine", e8 * 2 * nl * 3.5, ops_c, (k_ntt_p2_combine<FpArith, 512, 9>),
                 (uint64_t)2 * B * nl * tiles, 512, lds, st, nl, K, (uint32_t)p.nq, p.logN, p.k1, mods_of(ctx), twf,
                 ctx->t.moddown.u64(), u, conv, add, galois, out);
  else if (p.rows_nt == 512)
    FHE_LAUNCH_TO("ntt_p2_combine", e8 * 2 * nl * 3.5, ops_c, (k_ntt_p2_combine<FpArith, 512>),
                  (uint64_t)2 * B * nl * tiles,
                 512, lds, st, nl, K, (uint32_t)p.nq, p.logN, p.k1, mods_of(ctx), twf, ctx->t.moddown.u64(), u, conv,
                 add, galois, out);
  else
    FHE_LAUNCH_TO("ntt_p2_combine", e8 * 2 * nl * 3.5, ops_c, (k_ntt_p2_combine<FpArith, 256>),
                  (uint64_t)2 * B * nl * tiles,
                 256, lds, st, nl, K, (uint32_t)p.nq, p.logN, p.k1, mods_of(ctx), twf, ctx->t.moddown.u64(), u, conv,
                 add, galois, out);
}

size_t rescale_ws_elems(const fhe_ctx* ctx, uint32_t B, uint32_t ncomp, uint32_t nl) {
  return (size_t)B * ncomp * ctx->p.N * nl;
}

bool rescale_fuses_mask(const fhe_ctx* ctx) { return cols_fusable(ctx, 1); }

void rescale(const fhe_ctx* ctx, uint32_t B, uint32_t ncomp, uint32_t nl, const uint64_t* const* in,
             uint64_t* const* out, uint64_t* ws, hipStream_t st, const uint32_t* mask_galois) {
  if (!B) return;
  const Params& p = ctx->p;
  if (nl < 2 || nl > (uint32_t)p.nq) fail(FHE_ELEVEL, "rescale needs at least two limbs");
  prof_count("rescale", B);
  if (mask_galois && (!rescale_fuses_mask(ctx) || nl > (uint32_t)p.nq - 1))
    fail(FHE_EINVAL, "mask-fused rescale needs the fused column kernels and a level below the top");
  const uint32_t N = p.N, BC = B * ncomp;
  const double e8 = 8.0 * N * BC;
  uint64_t* tmp = ws;                       // [BC][N]
  uint64_t* w = ws + (size_t)BC * N;        // [BC][nl-1][N]
  FHE_LAUNCH("copy_last", e8 * 2, k_copy_last, grid_for((uint64_t)BC * N), 0, st, B, ncomp, nl, p.logN, mods_of(ctx),
             ctx->t.mask.u64(), mask_galois, in, tmp);
  if (cols_fusable(ctx, 1)) {
    // row phase of the dropped limb's INTT; column phases and the broadcast in one kernel; row
    // phase of the broadcast fused with the combine
    LimbBatch lb_last{tmp, 1, BC, N, 0, nl - 1};
    lb_last.raw_out = 1;
    ntt_inverse_rows(ctx, lb_last, st, "rescale_inv_p2");
    const uint32_t le = cols_log_e(p);
    const size_t lds_rs = cols_lds_bytes(le);
    const uint64_t grid = (uint64_t)BC * (N >> le);
    const double* twf = (const double*)ctx->t.twf.get();
    if (grid >= (1ull << 31)) fail(FHE_EINVAL, "rescale batch too large");
    // column phases: inverse of the dropped limb, forward of its broadcast into every other limb;
    // rows: forward row phase of the broadcast and the (x - w) q_l^-1 product (and the mask product)
    const double h1 = 0.5 * N * p.k1, h2 = 0.5 * N * (p.logN - p.k1);
    const double ops_cols = (double)BC * (h1 + N + (nl - 1) * h1);
    const double ops_rows = (double)BC * (nl - 1) * (h2 + (mask_galois ? 2.0 : 1.0) * N);
    switch (p.k1) {
      case 6:
        FHE_LAUNCH_TO("rescale_cols", e8 * nl, ops_cols, (k_rescale_cols<11, 256, 6>), grid, 256, lds_rs, st, nl, p.logN,
                     mods_of(ctx), twf, tmp, w);
        break;
      case 7:
        FHE_LAUNCH_TO("rescale_cols", e8 * nl, ops_cols, (k_rescale_cols<11, 256, 7>), grid, 256, lds_rs, st, nl, p.logN,
                     mods_of(ctx), twf, tmp, w);
        break;
      default:
        FHE_LAUNCH_TO("rescale_cols", e8 * nl, ops_cols, (k_rescale_cols<11, 256, 8>), grid, 256, lds_rs, st, nl, p.logN,
                     mods_of(ctx), twf, tmp, w);
        break;
    }
    const size_t lds = kNttLdsElems * sizeof(uint64_t);
    if (p.rows_nt == 512 && p.logN - p.k1 == 9)
      FHE_LAUNCH_TO("rescale_rows", e8 * 3 * (nl - 1), ops_rows, (k_rescale_rows<512, 9>),
                   (uint64_t)BC * (nl - 1) * (N >> kNttLogE), 512, lds, st, ncomp, nl, (uint32_t)p.nq, p.logN, p.k1,
                   mods_of(ctx), twf, ctx->t.rescale.u64(), ctx->t.mask.u64(), mask_galois, in, w, out);
    else if (p.rows_nt == 512)
      FHE_LAUNCH_TO("rescale_rows", e8 * 3 * (nl - 1), ops_rows, k_rescale_rows<512>, (uint64_t)BC * (nl - 1) * (N >> kNttLogE),
                   512, lds, st, ncomp, nl, (uint32_t)p.nq, p.logN, p.k1, mods_of(ctx), twf, ctx->t.rescale.u64(),
                   ctx->t.mask.u64(), mask_galois, in, w, out);
    else
      FHE_LAUNCH_TO("rescale_rows", e8 * 3 * (nl - 1), ops_rows, k_rescale_rows<256>, (uint64_t)BC * (nl - 1) * (N >> kNttLogE),
                   256, lds, st, ncomp, nl, (uint32_t)p.nq, p.logN, p.k1, mods_of(ctx), twf, ctx->t.rescale.u64(),
                   ctx->t.mask.u64(), mask_galois, in, w, out);
    return;
  }
  ntt_inverse(ctx, LimbBatch{tmp, 1, BC, N, 0, nl - 1}, st);
  FHE_LAUNCH("rescale_bcast", e8 * nl, k_rescale_bcast, grid_for((uint64_t)BC * (nl - 1) * N), 0, st, BC, nl, p.logN,
             mods_of(ctx), tmp, w);
  ntt_forward(ctx, LimbBatch{w, nl - 1, BC, (uint64_t)(nl - 1) * N, nl - 1, 0}, st);
  FHE_LAUNCH("rescale_combine", e8 * 3 * (nl - 1), k_rescale_combine, grid_for((uint64_t)BC * (nl - 1) * N), 0, st, B,
             ncomp, nl, (uint32_t)p.nq, p.logN, mods_of(ctx), ctx->t.rescale.u64(), in, w, out);
}

void mask_mul(const fhe_ctx* ctx, uint32_t B, uint32_t nl, const uint64_t* const* in, const uint32_t* galois,
              uint64_t* const* out, hipStream_t st) {
  if (!B) return;
  if (nl > (uint32_t)ctx->p.nq - 1) fail(FHE_ESHAPE, "mask multiply above level top-1");
  const double bytes = 8.0 * ctx->p.N * nl * (4.0 * B + 1);
  FHE_LAUNCH("mask_mul", bytes, k_mask_mul, grid_for((uint64_t)B << ctx->p.logN), 0, st, B, nl, ctx->p.logN,
             mods_of(ctx), ctx->t.mask.u64(), in, galois, out);
}

void mask_sum(const fhe_ctx* ctx, uint32_t nseg, uint32_t nentries, uint32_t nl, const uint32_t* seg,
              const uint64_t* const* in, const uint32_t* galois, uint64_t* acc, hipStream_t st) {
  if (!nseg) return;
  if (nl > (uint32_t)ctx->p.nq - 1) fail(FHE_ESHAPE, "mask multiply above level top-1");
  // every entry's two components and one mask row read, every accumulator written (read once more
  // when it already holds a partial sum; counted as written only)
  const double bytes = 8.0 * nl * ctx->p.N * (3.0 * nentries + 2.0 * nseg);
  FHE_LAUNCH("mask_sum", bytes, k_mask_sum, grid_for((uint64_t)nseg * nl << ctx->p.logN), 0, st, nseg, nl,
             ctx->p.logN, mods_of(ctx), ctx->t.mask_f.u64(), seg, in, galois, acc);
}

void accumulate_ptr(const fhe_ctx* ctx, uint32_t nseg, uint32_t ncontrib, uint32_t nl, const uint32_t* seg,
                    const uint64_t* const* contrib, uint64_t* const* results, hipStream_t st) {
  if (!nseg) return;
  const double bytes = 8.0 * 2 * nl * ctx->p.N * ((double)ncontrib + 2.0 * nseg);
  FHE_LAUNCH("accumulate", bytes, k_accumulate_ptr, grid_for((uint64_t)nseg * 2 * nl << ctx->p.logN), 0, st, nseg,
             nl, ctx->p.logN, mods_of(ctx), seg, contrib, results);
}

void fill_zero(const fhe_ctx* ctx, uint64_t n, uint64_t* x, hipStream_t st) {
  if (!n) return;
  FHE_LAUNCH("fill_zero", 8.0 * n, k_fill_zero, grid_for(n), 0, st, n, x);
}

void to_f64_bits(const fhe_ctx* ctx, uint64_t n, const uint64_t* in, uint64_t* out, hipStream_t st) {
  FHE_LAUNCH("to_f64_bits", 16.0 * n, k_to_f64_bits, grid_for(n), 0, st, n, in, out);
}

void accumulate(const fhe_ctx* ctx, uint32_t nseg, uint32_t ncontrib, uint32_t nl, const uint32_t* seg,
                const uint64_t* contrib, uint64_t* const* results, hipStream_t st) {
  if (!nseg) return;
  // every contribution read once, every touched result chunk read and written once
  const double bytes = 8.0 * 2 * nl * ctx->p.N * ((double)ncontrib + 2.0 * nseg);
  FHE_LAUNCH("accumulate", bytes, k_accumulate, grid_for((uint64_t)nseg * 2 * nl << ctx->p.logN), 0, st, nseg, nl,
             ctx->p.logN, mods_of(ctx), seg, contrib, results);
}

void signed_to_limbs(const fhe_ctx* ctx, const int64_t* v, uint32_t nlimbs, uint32_t n_first, uint32_t p_base,
                     uint64_t* out, hipStream_t st) {
  FHE_LAUNCH("signed_to_limbs", 0.0, k_signed_to_limbs, grid_for((uint64_t)nlimbs << ctx->p.logN), 0, st, v, nlimbs,
             n_first, p_base, ctx->p.logN, mods_of(ctx), out);
}

void to_montgomery(const fhe_ctx* ctx, uint64_t* x, uint32_t nlimbs, uint32_t n_first, uint32_t p_base,
                   hipStream_t st) {
  FHE_LAUNCH("to_montgomery", 0.0, k_to_mont, grid_for((uint64_t)nlimbs << ctx->p.logN), 0, st, x, nlimbs, n_first,
             p_base, ctx->p.logN, mods_of(ctx));
}

void keygen_digit(const fhe_ctx* ctx, uint32_t nall, const uint64_t* a, const uint64_t* s, const uint64_t* e,
                  const uint64_t* sp, const uint64_t* pfac, uint64_t* bout, uint64_t* aout, hipStream_t st) {
  FHE_LAUNCH("keygen_digit", 0.0, k_keygen_digit, grid_for((uint64_t)nall << ctx->p.logN), 0, st, nall, (uint32_t)ctx->p.nq,
             ctx->p.logN,
             mods_of(ctx), a, s, e, sp, pfac, bout, aout);
}

void square(const fhe_ctx* ctx, uint32_t nall, const uint64_t* s, uint64_t* s2, hipStream_t st) {
  FHE_LAUNCH("square", 0.0, k_square, grid_for((uint64_t)nall << ctx->p.logN), 0, st, nall, ctx->p.logN, mods_of(ctx),
             s, s2);
}

void encrypt_combine(const fhe_ctx* ctx, uint32_t nl, const uint64_t* a, const uint64_t* em, const uint64_t* s,
                     uint64_t* ct, hipStream_t st) {
  FHE_LAUNCH("encrypt_combine", 0.0, k_encrypt_combine, grid_for((uint64_t)nl << ctx->p.logN), 0, st, nl, ctx->p.logN,
             mods_of(ctx), a, em, s, ct);
}

void decrypt_combine(const fhe_ctx* ctx, uint32_t nl, uint32_t nlim, const uint64_t* ct, const uint64_t* s,
                     uint64_t* m, hipStream_t st) {
  FHE_LAUNCH("decrypt_combine", 0.0, k_decrypt_combine, grid_for((uint64_t)nlim << ctx->p.logN), 0, st, nl, nlim,
             ctx->p.logN, mods_of(ctx), ct, s, m);
}

void add_ct(const fhe_ctx* ctx, uint32_t ncomp, uint32_t nl, const uint64_t* a, const uint64_t* b, uint64_t* out,
            hipStream_t st) {
  FHE_LAUNCH("add", 24.0 * ncomp * nl * ctx->p.N, k_add, grid_for((uint64_t)ncomp * nl << ctx->p.logN), 0, st, ncomp,
             nl, ctx->p.logN, mods_of(ctx), a, b, out);
}

double bench_mulmod(int kind, uint32_t iters, hipStream_t st) {
  if (kind < 0 || kind > 2) fail(FHE_EINVAL, "kind must be 0 (FP64), 1 (Shoup) or 2 (Montgomery)");
  if (iters < 1 || iters > (1u << 20)) fail(FHE_EINVAL, "iters must be in [1, 2^20]");
  // any odd modulus of the right size times the same instruction sequence as a prime
  const uint64_t q = kind == 0 ? (1ull << 49) + 12345 : (1ull << 59) + 54321;
  const uint64_t w = q / 3 + 7, wx = shoup_prep(w, q), qinv = mont_qinv(q);
  const uint32_t blocks = 256 * 16;
  DevBuf out((size_t)blocks * kThreads * 8, st);
  hipEvent_t a, b;
  HIPCHECK(hipEventCreate(&a));
  HIPCHECK(hipEventCreate(&b));
  float ms = 0.f;
  for (int rep = 0; rep < 2; ++rep) {  // the first launch loads the code object
    HIPCHECK(hipEventRecord(a, st));
    if (kind == 0)
      hipLaunchKernelGGL(k_bench_mulmod<0>, dim3(blocks), dim3(kThreads), 0, st, iters, q, qinv, w, wx, out.u64());
    else if (kind == 1)
      hipLaunchKernelGGL(k_bench_mulmod<1>, dim3(blocks), dim3(kThreads), 0, st, iters, q, qinv, w, wx, out.u64());
    else
      hipLaunchKernelGGL(k_bench_mulmod<2>, dim3(blocks), dim3(kThreads), 0, st, iters, q, qinv, w, wx, out.u64());
    check_launch("bench_mulmod");
    HIPCHECK(hipEventRecord(b, st));
    HIPCHECK(hipEventSynchronize(b));
    HIPCHECK(hipEventElapsedTime(&ms, a, b));
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return (double)blocks * kThreads * 8.0 * iters / (ms * 1e-3);
}

}  // namespace fhe
