// gfx950 kernels for RNS-CKKS: negacyclic NTT, automorphism, tensor product, hybrid key switching
// (ModUp fast base conversion, key inner product, ModDown), rescale, one-hot mask multiply and
// accumulation. Residues are uint64 in [0, q), limb-major ([..][limb][coefficient]) so that a
// wavefront reads 64 consecutive coefficients of one limb (512 contiguous bytes).
#include "kernels.h"

namespace fhe {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxAlpha = 8;
constexpr int kMaxK = 8;

__device__ __forceinline__ uint32_t brev_bits(uint32_t x, uint32_t bits) { return __brev(x) >> (32 - bits); }

__device__ __forceinline__ uint32_t mod_index(const LimbBatch& lb, uint32_t e) {
  return e < lb.n_first ? e : lb.p_base + (e - lb.n_first);
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
// twiddles: stage s uses w = psi_rev[2^s + floor(j / 2t)], t = N / 2^(s+1). Stages 0..k1-1 (t >= N2)
// pair elements in the same column of the N1 x N2 view (stride N2); phase 1 loads 2^logC adjacent
// columns per workgroup into LDS. Stages k1..logN-1 act inside contiguous rows; phase 2 loads a
// contiguous tile of rows. Each workgroup moves one 2^logE-element tile through LDS per phase.
// ------------------------------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_ntt_fwd_p1(LimbBatch lb, const ModInfo* __restrict__ mods,
                                                        const uint64_t* __restrict__ tw, uint32_t logN,
                                                        uint32_t k1, uint32_t logE) {
  extern __shared__ uint64_t lds[];
  const uint32_t N = 1u << logN, k2 = logN - k1, E = 1u << logE, logC = logE - k1, C = 1u << logC;
  const uint32_t tiles = N >> logE;
  const uint32_t limb = blockIdx.x / tiles, tile = blockIdx.x - limb * tiles;
  const uint32_t poly = limb / lb.limbs, e = limb - poly * lb.limbs;
  uint64_t* a = lb.base + (uint64_t)poly * lb.poly_stride + (uint64_t)e * N;
  const uint32_t mi = mod_index(lb, e);
  const uint64_t q = mods[mi].q;
  const uint64_t* w = tw + (uint64_t)mi * 4 * N;
  const uint64_t* wp = w + N;
  const uint32_t y0 = tile << logC;
  for (uint32_t idx = threadIdx.x; idx < E; idx += kThreads)
    lds[idx] = a[((uint64_t)(idx >> logC) << k2) + y0 + (idx & (C - 1))];
  __syncthreads();
  for (uint32_t s = 0; s < k1; ++s) {
    const uint32_t logt = k1 - 1 - s;  // column distance 2^logt
    for (uint32_t b = threadIdx.x; b < E / 2; b += kThreads) {
      const uint32_t c = b & (C - 1), h = b >> logC;
      const uint32_t x = ((h >> logt) << (logt + 1)) + (h & ((1u << logt) - 1));
      const uint32_t wi = (1u << s) + (x >> (logt + 1));
      const uint32_t i0 = (x << logC) + c, i1 = i0 + (1u << (logt + logC));
      const uint64_t U = lds[i0];
      const uint64_t V = shoup_mul(lds[i1], w[wi], wp[wi], q);
      lds[i0] = add_mod(U, V, q);
      lds[i1] = sub_mod(U, V, q);
    }
    __syncthreads();
  }
  for (uint32_t idx = threadIdx.x; idx < E; idx += kThreads)
    a[((uint64_t)(idx >> logC) << k2) + y0 + (idx & (C - 1))] = lds[idx];
}

__global__ __launch_bounds__(kThreads) void k_ntt_fwd_p2(LimbBatch lb, const ModInfo* __restrict__ mods,
                                                        const uint64_t* __restrict__ tw, uint32_t logN,
                                                        uint32_t k1, uint32_t logE) {
  extern __shared__ uint64_t lds[];
  const uint32_t N = 1u << logN, E = 1u << logE;
  const uint32_t tiles = N >> logE;
  const uint32_t limb = blockIdx.x / tiles, tile = blockIdx.x - limb * tiles;
  const uint32_t poly = limb / lb.limbs, e = limb - poly * lb.limbs;
  uint64_t* a = lb.base + (uint64_t)poly * lb.poly_stride + (uint64_t)e * N + (uint64_t)tile * E;
  const uint32_t mi = mod_index(lb, e);
  const uint64_t q = mods[mi].q;
  const uint64_t* w = tw + (uint64_t)mi * 4 * N;
  const uint64_t* wp = w + N;
  const uint32_t j0 = tile * E;
  for (uint32_t idx = threadIdx.x; idx < E; idx += kThreads) lds[idx] = a[idx];
  __syncthreads();
  for (uint32_t s = k1; s < logN; ++s) {
    const uint32_t logt = logN - 1 - s;
    for (uint32_t b = threadIdx.x; b < E / 2; b += kThreads) {
      const uint32_t j = ((b >> logt) << (logt + 1)) + (b & ((1u << logt) - 1));
      const uint32_t wi = (1u << s) + ((j0 + j) >> (logt + 1));
      const uint64_t U = lds[j];
      const uint64_t V = shoup_mul(lds[j + (1u << logt)], w[wi], wp[wi], q);
      lds[j] = add_mod(U, V, q);
      lds[j + (1u << logt)] = sub_mod(U, V, q);
    }
    __syncthreads();
  }
  for (uint32_t idx = threadIdx.x; idx < E; idx += kThreads) a[idx] = lds[idx];
}

__global__ __launch_bounds__(kThreads) void k_ntt_inv_p2(LimbBatch lb, const ModInfo* __restrict__ mods,
                                                        const uint64_t* __restrict__ tw, uint32_t logN,
                                                        uint32_t k1, uint32_t logE) {
  extern __shared__ uint64_t lds[];
  const uint32_t N = 1u << logN, E = 1u << logE;
  const uint32_t tiles = N >> logE;
  const uint32_t limb = blockIdx.x / tiles, tile = blockIdx.x - limb * tiles;
  const uint32_t poly = limb / lb.limbs, e = limb - poly * lb.limbs;
  uint64_t* a = lb.base + (uint64_t)poly * lb.poly_stride + (uint64_t)e * N + (uint64_t)tile * E;
  const uint32_t mi = mod_index(lb, e);
  const uint64_t q = mods[mi].q;
  const uint64_t* w = tw + (uint64_t)mi * 4 * N + 2 * (uint64_t)N;
  const uint64_t* wp = w + N;
  const uint32_t j0 = tile * E;
  for (uint32_t idx = threadIdx.x; idx < E; idx += kThreads) lds[idx] = a[idx];
  __syncthreads();
  for (int s = (int)logN - 1; s >= (int)k1; --s) {
    const uint32_t logt = logN - 1 - s;
    for (uint32_t b = threadIdx.x; b < E / 2; b += kThreads) {
      const uint32_t j = ((b >> logt) << (logt + 1)) + (b & ((1u << logt) - 1));
      const uint32_t wi = (1u << s) + ((j0 + j) >> (logt + 1));
      const uint64_t U = lds[j], V = lds[j + (1u << logt)];
      lds[j] = add_mod(U, V, q);
      lds[j + (1u << logt)] = shoup_mul(sub_mod(U, V, q), w[wi], wp[wi], q);
    }
    __syncthreads();
  }
  for (uint32_t idx = threadIdx.x; idx < E; idx += kThreads) a[idx] = lds[idx];
}

__global__ __launch_bounds__(kThreads) void k_ntt_inv_p1(LimbBatch lb, const ModInfo* __restrict__ mods,
                                                        const uint64_t* __restrict__ tw, uint32_t logN,
                                                        uint32_t k1, uint32_t logE) {
  extern __shared__ uint64_t lds[];
  const uint32_t N = 1u << logN, k2 = logN - k1, E = 1u << logE, logC = logE - k1, C = 1u << logC;
  const uint32_t tiles = N >> logE;
  const uint32_t limb = blockIdx.x / tiles, tile = blockIdx.x - limb * tiles;
  const uint32_t poly = limb / lb.limbs, e = limb - poly * lb.limbs;
  uint64_t* a = lb.base + (uint64_t)poly * lb.poly_stride + (uint64_t)e * N;
  const uint32_t mi = mod_index(lb, e);
  const uint64_t q = mods[mi].q;
  const uint64_t ninv = mods[mi].n_inv, ninvp = mods[mi].n_inv_shoup;
  const uint64_t* w = tw + (uint64_t)mi * 4 * N + 2 * (uint64_t)N;
  const uint64_t* wp = w + N;
  const uint32_t y0 = tile << logC;
  for (uint32_t idx = threadIdx.x; idx < E; idx += kThreads)
    lds[idx] = a[((uint64_t)(idx >> logC) << k2) + y0 + (idx & (C - 1))];
  __syncthreads();
  for (int s = (int)k1 - 1; s >= 0; --s) {
    const uint32_t logt = k1 - 1 - s;
    for (uint32_t b = threadIdx.x; b < E / 2; b += kThreads) {
      const uint32_t c = b & (C - 1), h = b >> logC;
      const uint32_t x = ((h >> logt) << (logt + 1)) + (h & ((1u << logt) - 1));
      const uint32_t wi = (1u << s) + (x >> (logt + 1));
      const uint32_t i0 = (x << logC) + c, i1 = i0 + (1u << (logt + logC));
      const uint64_t U = lds[i0], V = lds[i1];
      lds[i0] = add_mod(U, V, q);
      lds[i1] = shoup_mul(sub_mod(U, V, q), w[wi], wp[wi], q);
    }
    __syncthreads();
  }
  for (uint32_t idx = threadIdx.x; idx < E; idx += kThreads)
    a[((uint64_t)(idx >> logC) << k2) + y0 + (idx & (C - 1))] = shoup_mul(lds[idx], ninv, ninvp, q);
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
    const uint64_t* s = src[b];
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
    const uint64_t* a = A[b];
    const uint64_t* bb = Bc[b];
    const uint64_t a0 = a[(uint64_t)i * N + k], a1 = a[(uint64_t)(nl + i) * N + k];
    const uint64_t b0 = bb[(uint64_t)i * N + k], b1 = bb[(uint64_t)(nl + i) * N + k];
    uint64_t* o = out + (uint64_t)b * 3 * nl * N;
    o[(uint64_t)i * N + k] = mont_mul(mont_mul(a0, b0, m.q, m.qinv), m.r2, m.q, m.qinv);
    const uint64_t x = add_mod(mont_mul(a0, b1, m.q, m.qinv), mont_mul(a1, b0, m.q, m.qinv), m.q);
    o[(uint64_t)(nl + i) * N + k] = mont_mul(x, m.r2, m.q, m.qinv);
    o[(uint64_t)(2 * nl + i) * N + k] = mont_mul(mont_mul(a1, b1, m.q, m.qinv), m.r2, m.q, m.qinv);
  }
}

// ModUp (coefficient domain): for item b, digit j, coefficient k.
// tab block of digit j: [alpha][2] (Dhat_i^-1 mod q_i, shoup) then [alpha][next][2] (Dhat_i mod t_e, shoup).
__global__ __launch_bounds__(kThreads) void k_modup(uint32_t B, uint32_t nl, uint32_t K, uint32_t nq, uint32_t alpha,
                                                   uint32_t logN, const ModInfo* __restrict__ mods,
                                                   const uint64_t* __restrict__ tab, const uint64_t* __restrict__ din,
                                                   uint64_t in_stride, uint64_t* __restrict__ ext) {
  const uint32_t N = 1u << logN;
  const uint32_t beta = (nl + alpha - 1) / alpha, next = nl + K;
  const uint64_t total = (uint64_t)B * beta << logN;
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < total; t += (uint64_t)gridDim.x * kThreads) {
    const uint32_t k = (uint32_t)t & (N - 1);
    const uint64_t r = t >> logN;
    const uint32_t j = (uint32_t)(r % beta), b = (uint32_t)(r / beta);
    const uint32_t lo = j * alpha, cnt = min(alpha, nl - lo);
    const uint64_t* blk = tab + (uint64_t)j * (2 * alpha + 2 * alpha * next);
    const uint64_t* d = din + (uint64_t)b * in_stride;
    uint64_t dv[kMaxAlpha], y[kMaxAlpha];
    for (uint32_t i = 0; i < cnt; ++i) {
      dv[i] = d[(uint64_t)(lo + i) * N + k];
      y[i] = shoup_mul(dv[i], blk[2 * i], blk[2 * i + 1], mods[lo + i].q);
    }
    uint64_t* o = ext + (uint64_t)(b * beta + j) * next * N + k;
    for (uint32_t e = 0; e < next; ++e) {
      uint64_t v;
      if (e >= lo && e < lo + cnt) {
        v = dv[e - lo];
      } else {
        const uint64_t tq = mods[e < nl ? e : nq + (e - nl)].q;
        const uint64_t* mrow = blk + 2 * alpha + 2 * (uint64_t)e;
        v = 0;
        for (uint32_t i = 0; i < cnt; ++i) {
          const uint64_t* c = mrow + (uint64_t)i * 2 * next;
          v = add_mod(v, shoup_mul(y[i], c[0], c[1], tq), tq);
        }
      }
      o[(uint64_t)e * N] = v;
    }
  }
}

// u[b][c][e] = sum_j ext[b][j][e] * key[b][j][c][limb(e)] (key in Montgomery form).
__global__ __launch_bounds__(kThreads) void k_ks_inner(uint32_t B, uint32_t nl, uint32_t K, uint32_t nq,
                                                      uint32_t alpha, uint32_t logN, const ModInfo* __restrict__ mods,
                                                      const uint64_t* __restrict__ ext,
                                                      const uint64_t* const* __restrict__ keys,
                                                      uint64_t* __restrict__ u) {
  const uint32_t N = 1u << logN;
  const uint32_t beta = (nl + alpha - 1) / alpha, next = nl + K, nall = nq + K;
  const uint64_t total = (uint64_t)B * next << logN;
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < total; t += (uint64_t)gridDim.x * kThreads) {
    const uint32_t k = (uint32_t)t & (N - 1);
    const uint64_t r = t >> logN;
    const uint32_t e = (uint32_t)(r % next), b = (uint32_t)(r / next);
    const uint32_t mi = e < nl ? e : nq + (e - nl);
    const ModInfo m = mods[mi];
    const uint64_t* key = keys[b];
    uint64_t acc0 = 0, acc1 = 0;
    for (uint32_t j = 0; j < beta; ++j) {
      const uint64_t x = ext[((uint64_t)(b * beta + j) * next + e) * N + k];
      const uint64_t k0 = key[((uint64_t)(j * 2 + 0) * nall + mi) * N + k];
      const uint64_t k1 = key[((uint64_t)(j * 2 + 1) * nall + mi) * N + k];
      acc0 = add_mod(acc0, mont_mul(x, k0, m.q, m.qinv), m.q);
      acc1 = add_mod(acc1, mont_mul(x, k1, m.q, m.qinv), m.q);
    }
    u[((uint64_t)(b * 2 + 0) * next + e) * N + k] = acc0;
    u[((uint64_t)(b * 2 + 1) * next + e) * N + k] = acc1;
  }
}

// ModDown base conversion P -> Q_l (coefficient domain). tab: [K][2] ((P/p_k)^-1 mod p_k),
// [K][nq][2] ((P/p_k) mod q_i), [nq][2] (P^-1 mod q_i).
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
    for (uint32_t kk = 0; kk < K; ++kk)
      z[kk] = shoup_mul(u[((uint64_t)bc * next + nl + kk) * N + k], tab[2 * kk], tab[2 * kk + 1], mods[nq + kk].q);
    const uint64_t* pq = tab + 2 * K;
    for (uint32_t i = 0; i < nl; ++i) {
      const uint64_t q = mods[i].q;
      uint64_t acc = 0;
      for (uint32_t kk = 0; kk < K; ++kk) {
        const uint64_t* c = pq + 2 * ((uint64_t)kk * nq + i);
        acc = add_mod(acc, shoup_mul(z[kk], c[0], c[1], q), q);
      }
      conv[((uint64_t)bc * nl + i) * N + k] = acc;
    }
  }
}

// out[b][c][i] = add[2b+c][i] + (u[b][c][i] - conv[b][c][i]) P^-1 (NTT domain).
__global__ __launch_bounds__(kThreads) void k_ks_combine(uint32_t B, uint32_t nl, uint32_t K, uint32_t nq,
                                                        uint32_t logN, const ModInfo* __restrict__ mods,
                                                        const uint64_t* __restrict__ tab,
                                                        const uint64_t* __restrict__ u,
                                                        const uint64_t* __restrict__ conv,
                                                        const uint64_t* const* __restrict__ add,
                                                        uint64_t* const* __restrict__ out) {
  const uint32_t N = 1u << logN, next = nl + K;
  const uint64_t* pinv = tab + 2 * K + 2 * (uint64_t)K * nq;
  const uint64_t total = (uint64_t)B * 2 * nl << logN;
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < total; t += (uint64_t)gridDim.x * kThreads) {
    const uint32_t k = (uint32_t)t & (N - 1);
    const uint64_t r = t >> logN;
    const uint32_t i = (uint32_t)(r % nl);
    const uint32_t bc = (uint32_t)(r / nl), b = bc >> 1, c = bc & 1;
    const uint64_t q = mods[i].q;
    uint64_t v = sub_mod(u[((uint64_t)bc * next + i) * N + k], conv[((uint64_t)bc * nl + i) * N + k], q);
    v = shoup_mul(v, pinv[2 * i], pinv[2 * i + 1], q);
    const uint64_t* ad = add[bc];
    if (ad) v = add_mod(v, ad[(uint64_t)i * N + k], q);
    out[b][((uint64_t)c * nl + i) * N + k] = v;
  }
}

__global__ __launch_bounds__(kThreads) void k_copy_last(uint32_t B, uint32_t ncomp, uint32_t nl, uint32_t logN,
                                                       const uint64_t* const* __restrict__ in,
                                                       uint64_t* __restrict__ tmp) {
  const uint32_t N = 1u << logN;
  const uint64_t total = (uint64_t)B * ncomp << logN;
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < total; t += (uint64_t)gridDim.x * kThreads) {
    const uint32_t k = (uint32_t)t & (N - 1);
    const uint32_t bc = (uint32_t)(t >> logN), b = bc / ncomp, c = bc - b * ncomp;
    tmp[t] = in[b][((uint64_t)c * nl + nl - 1) * N + k];
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
    const uint64_t x = sub_mod(in[b][((uint64_t)c * nl + i) * N + k], w[t], q);
    out[b][((uint64_t)c * no + i) * N + k] = shoup_mul(x, inv[2 * i], inv[2 * i + 1], q);
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
    const uint64_t* s = in[b];
    uint64_t* d = out[b];
    for (uint32_t i = 0; i < nl; ++i) {
      const ModInfo m = mods[i];
      const uint64_t mk = maskm[((uint64_t)i << logN) + ks];
      d[(uint64_t)i * N + k] = mont_mul(s[(uint64_t)i * N + k], mk, m.q, m.qinv);
      d[(uint64_t)(nl + i) * N + k] = mont_mul(s[(uint64_t)(nl + i) * N + k], mk, m.q, m.qinv);
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_accumulate(uint32_t nseg, uint32_t nl, uint32_t logN,
                                                        const ModInfo* __restrict__ mods,
                                                        const uint32_t* __restrict__ seg,
                                                        const uint64_t* __restrict__ contrib,
                                                        uint64_t* __restrict__ result) {
  const uint32_t N = 1u << logN;
  const uint64_t per = (uint64_t)2 * nl << logN;
  const uint64_t total = (uint64_t)nseg * per;
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < total; t += (uint64_t)gridDim.x * kThreads) {
    const uint32_t s = (uint32_t)(t / per);
    const uint64_t off = t - (uint64_t)s * per;
    const uint32_t i = (uint32_t)((off >> logN) % nl);
    const uint64_t q = mods[i].q;
    const uint32_t chunk = seg[3 * s], b0 = seg[3 * s + 1], b1 = seg[3 * s + 2];
    uint64_t acc = result[(uint64_t)chunk * per + off];
    for (uint32_t b = b0; b < b1; ++b) acc = add_mod(acc, contrib[(uint64_t)b * per + off], q);
    result[(uint64_t)chunk * per + off] = acc;
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

__global__ __launch_bounds__(kThreads) void k_keygen_digit(uint32_t nall, uint32_t logN,
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
    bout[t] = mont_mul(b, m.r2, m.q, m.qinv);
    aout[t] = mont_mul(a[t], m.r2, m.q, m.qinv);
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

}  // namespace

// ------------------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------------------

static const ModInfo* mods_of(const fhe_ctx* ctx) { return (const ModInfo*)ctx->t.mods.get(); }

static void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) fail(FHE_EDEVICE, std::string("kernel launch failed (") + what + "): " + hipGetErrorString(e));
}

static void check_batch(const fhe_ctx* ctx, const LimbBatch& lb) {
  const Params& p = ctx->p;
  if (lb.limbs == 0 || lb.npoly == 0) return;
  uint32_t last = lb.limbs - 1;
  uint32_t mi = last < lb.n_first ? last : lb.p_base + (last - lb.n_first);
  uint32_t mi0 = 0 < lb.n_first ? 0 : lb.p_base;
  if (mi >= (uint32_t)p.nmod() || mi0 >= (uint32_t)p.nmod()) fail(FHE_EINVAL, "NTT batch modulus index out of range");
}

void ntt_forward(const fhe_ctx* ctx, const LimbBatch& lb, hipStream_t st) {
  if (lb.limbs == 0 || lb.npoly == 0) return;
  check_batch(ctx, lb);
  const Params& p = ctx->p;
  const uint32_t tiles = p.N >> p.logE;
  const uint64_t blocks = (uint64_t)tiles * lb.limbs * lb.npoly;
  if (blocks >= (1ull << 31)) fail(FHE_EINVAL, "NTT batch too large");
  const size_t lds = ((size_t)1 << p.logE) * sizeof(uint64_t);
  hipLaunchKernelGGL(k_ntt_fwd_p1, dim3((uint32_t)blocks), dim3(kThreads), lds, st, lb, mods_of(ctx), ctx->t.tw.u64(),
                     p.logN, p.k1, p.logE);
  hipLaunchKernelGGL(k_ntt_fwd_p2, dim3((uint32_t)blocks), dim3(kThreads), lds, st, lb, mods_of(ctx), ctx->t.tw.u64(),
                     p.logN, p.k1, p.logE);
  check_launch("ntt_forward");
}

void ntt_inverse(const fhe_ctx* ctx, const LimbBatch& lb, hipStream_t st) {
  if (lb.limbs == 0 || lb.npoly == 0) return;
  check_batch(ctx, lb);
  const Params& p = ctx->p;
  const uint32_t tiles = p.N >> p.logE;
  const uint64_t blocks = (uint64_t)tiles * lb.limbs * lb.npoly;
  if (blocks >= (1ull << 31)) fail(FHE_EINVAL, "NTT batch too large");
  const size_t lds = ((size_t)1 << p.logE) * sizeof(uint64_t);
  hipLaunchKernelGGL(k_ntt_inv_p2, dim3((uint32_t)blocks), dim3(kThreads), lds, st, lb, mods_of(ctx), ctx->t.tw.u64(),
                     p.logN, p.k1, p.logE);
  hipLaunchKernelGGL(k_ntt_inv_p1, dim3((uint32_t)blocks), dim3(kThreads), lds, st, lb, mods_of(ctx), ctx->t.tw.u64(),
                     p.logN, p.k1, p.logE);
  check_launch("ntt_inverse");
}

void automorph(const fhe_ctx* ctx, uint32_t B, uint32_t ncomp, uint32_t nl, const uint64_t* const* src,
               const uint32_t* galois, uint64_t* dst, hipStream_t st) {
  if (!B) return;
  hipLaunchKernelGGL(k_automorph, dim3(grid_for((uint64_t)B << ctx->p.logN)), dim3(kThreads), 0, st, B, ncomp, nl,
                     ctx->p.logN, src, galois, dst);
  check_launch("automorph");
}

void tensor(const fhe_ctx* ctx, uint32_t B, uint32_t nl, const uint64_t* const* a, const uint64_t* const* b,
            uint64_t* out, hipStream_t st) {
  if (!B) return;
  hipLaunchKernelGGL(k_tensor, dim3(grid_for((uint64_t)B * nl << ctx->p.logN)), dim3(kThreads), 0, st, B, nl,
                     ctx->p.logN, mods_of(ctx), a, b, out);
  check_launch("tensor");
}

size_t keyswitch_ws_elems(const fhe_ctx* ctx, uint32_t B, uint32_t nl) {
  const Params& p = ctx->p;
  const size_t N = p.N, next = nl + p.np, beta = p.beta(nl);
  return (size_t)B * N * (beta * next + 2 * next + 2 * nl);
}

void keyswitch(const fhe_ctx* ctx, uint32_t B, uint32_t nl, uint64_t* in, uint64_t in_stride,
               const uint64_t* const* keys, const uint64_t* const* add, uint64_t* const* out, uint64_t* ws,
               hipStream_t st) {
  if (!B) return;
  const Params& p = ctx->p;
  if (p.alpha > kMaxAlpha || p.np > kMaxK) fail(FHE_EINVAL, "alpha or n_p above kernel limits");
  if (nl < 1 || nl > (uint32_t)p.nq) fail(FHE_ESHAPE, "key switch level out of range");
  const uint32_t N = p.N, K = p.np, next = nl + K, beta = p.beta(nl);
  uint64_t* ext = ws;                                   // [B][beta][next][N]
  uint64_t* u = ext + (size_t)B * beta * next * N;      // [B][2][next][N]
  uint64_t* conv = u + (size_t)B * 2 * next * N;        // [B][2][nl][N]
  // 1. INTT of the input (in place).
  ntt_inverse(ctx, LimbBatch{in, nl, B, in_stride, nl, 0}, st);
  // 2. ModUp per digit, all limbs of the extended basis.
  hipLaunchKernelGGL(k_modup, dim3(grid_for((uint64_t)B * beta * N)), dim3(kThreads), 0, st, B, nl, K, (uint32_t)p.nq,
                     (uint32_t)p.alpha, p.logN, mods_of(ctx), ctx->t.modup.u64() + ctx->t.modup_offset[nl], in, in_stride,
                     ext);
  check_launch("modup");
  // 3. NTT of the extended digits.
  ntt_forward(ctx, LimbBatch{ext, next, B * beta, (uint64_t)next * N, nl, (uint32_t)p.nq}, st);
  // 4. Inner product with the key.
  hipLaunchKernelGGL(k_ks_inner, dim3(grid_for((uint64_t)B * next * N)), dim3(kThreads), 0, st, B, nl, K,
                     (uint32_t)p.nq, (uint32_t)p.alpha, p.logN, mods_of(ctx), ext, keys, u);
  check_launch("ks_inner");
  // 5. ModDown: INTT of the P limbs, conversion to Q_l, NTT, combine.
  ntt_inverse(ctx, LimbBatch{u + (size_t)nl * N, K, 2 * B, (uint64_t)next * N, 0, (uint32_t)p.nq}, st);
  hipLaunchKernelGGL(k_moddown_conv, dim3(grid_for((uint64_t)B * 2 * N)), dim3(kThreads), 0, st, B, nl, K,
                     (uint32_t)p.nq, p.logN, mods_of(ctx), ctx->t.moddown.u64(), u, conv);
  check_launch("moddown_conv");
  ntt_forward(ctx, LimbBatch{conv, nl, 2 * B, (uint64_t)nl * N, nl, 0}, st);
  hipLaunchKernelGGL(k_ks_combine, dim3(grid_for((uint64_t)B * 2 * nl * N)), dim3(kThreads), 0, st, B, nl, K,
                     (uint32_t)p.nq, p.logN, mods_of(ctx), ctx->t.moddown.u64(), u, conv, add, out);
  check_launch("ks_combine");
}

size_t rescale_ws_elems(const fhe_ctx* ctx, uint32_t B, uint32_t ncomp, uint32_t nl) {
  return (size_t)B * ncomp * ctx->p.N * nl;
}

void rescale(const fhe_ctx* ctx, uint32_t B, uint32_t ncomp, uint32_t nl, const uint64_t* const* in,
             uint64_t* const* out, uint64_t* ws, hipStream_t st) {
  if (!B) return;
  const Params& p = ctx->p;
  if (nl < 2 || nl > (uint32_t)p.nq) fail(FHE_ELEVEL, "rescale needs at least two limbs");
  const uint32_t N = p.N, BC = B * ncomp;
  uint64_t* tmp = ws;                       // [BC][N]
  uint64_t* w = ws + (size_t)BC * N;        // [BC][nl-1][N]
  hipLaunchKernelGGL(k_copy_last, dim3(grid_for((uint64_t)BC * N)), dim3(kThreads), 0, st, B, ncomp, nl, p.logN, in,
                     tmp);
  check_launch("copy_last");
  ntt_inverse(ctx, LimbBatch{tmp, 1, BC, N, 0, nl - 1}, st);
  hipLaunchKernelGGL(k_rescale_bcast, dim3(grid_for((uint64_t)BC * (nl - 1) * N)), dim3(kThreads), 0, st, BC, nl,
                     p.logN, mods_of(ctx), tmp, w);
  check_launch("rescale_bcast");
  ntt_forward(ctx, LimbBatch{w, nl - 1, BC, (uint64_t)(nl - 1) * N, nl - 1, 0}, st);
  hipLaunchKernelGGL(k_rescale_combine, dim3(grid_for((uint64_t)BC * (nl - 1) * N)), dim3(kThreads), 0, st, B, ncomp,
                     nl, (uint32_t)p.nq, p.logN, mods_of(ctx), ctx->t.rescale.u64(), in, w, out);
  check_launch("rescale_combine");
}

void mask_mul(const fhe_ctx* ctx, uint32_t B, uint32_t nl, const uint64_t* const* in, const uint32_t* galois,
              uint64_t* const* out, hipStream_t st) {
  if (!B) return;
  if (nl > (uint32_t)ctx->p.nq - 1) fail(FHE_ESHAPE, "mask multiply above level top-1");
  hipLaunchKernelGGL(k_mask_mul, dim3(grid_for((uint64_t)B << ctx->p.logN)), dim3(kThreads), 0, st, B, nl,
                     ctx->p.logN, mods_of(ctx), ctx->t.mask.u64(), in, galois, out);
  check_launch("mask_mul");
}

void accumulate(const fhe_ctx* ctx, uint32_t nseg, uint32_t nl, const uint32_t* seg, const uint64_t* contrib,
                uint64_t* result, hipStream_t st) {
  if (!nseg) return;
  hipLaunchKernelGGL(k_accumulate, dim3(grid_for((uint64_t)nseg * 2 * nl << ctx->p.logN)), dim3(kThreads), 0, st, nseg,
                     nl, ctx->p.logN, mods_of(ctx), seg, contrib, result);
  check_launch("accumulate");
}

void signed_to_limbs(const fhe_ctx* ctx, const int64_t* v, uint32_t nlimbs, uint32_t n_first, uint32_t p_base,
                     uint64_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_signed_to_limbs, dim3(grid_for((uint64_t)nlimbs << ctx->p.logN)), dim3(kThreads), 0, st, v,
                     nlimbs, n_first, p_base, ctx->p.logN, mods_of(ctx), out);
  check_launch("signed_to_limbs");
}

void to_montgomery(const fhe_ctx* ctx, uint64_t* x, uint32_t nlimbs, uint32_t n_first, uint32_t p_base,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_to_mont, dim3(grid_for((uint64_t)nlimbs << ctx->p.logN)), dim3(kThreads), 0, st, x, nlimbs,
                     n_first, p_base, ctx->p.logN, mods_of(ctx));
  check_launch("to_montgomery");
}

void keygen_digit(const fhe_ctx* ctx, uint32_t nall, const uint64_t* a, const uint64_t* s, const uint64_t* e,
                  const uint64_t* sp, const uint64_t* pfac, uint64_t* bout, uint64_t* aout, hipStream_t st) {
  hipLaunchKernelGGL(k_keygen_digit, dim3(grid_for((uint64_t)nall << ctx->p.logN)), dim3(kThreads), 0, st, nall,
                     ctx->p.logN, mods_of(ctx), a, s, e, sp, pfac, bout, aout);
  check_launch("keygen_digit");
}

void square(const fhe_ctx* ctx, uint32_t nall, const uint64_t* s, uint64_t* s2, hipStream_t st) {
  hipLaunchKernelGGL(k_square, dim3(grid_for((uint64_t)nall << ctx->p.logN)), dim3(kThreads), 0, st, nall,
                     ctx->p.logN, mods_of(ctx), s, s2);
  check_launch("square");
}

void encrypt_combine(const fhe_ctx* ctx, uint32_t nl, const uint64_t* a, const uint64_t* em, const uint64_t* s,
                     uint64_t* ct, hipStream_t st) {
  hipLaunchKernelGGL(k_encrypt_combine, dim3(grid_for((uint64_t)nl << ctx->p.logN)), dim3(kThreads), 0, st, nl,
                     ctx->p.logN, mods_of(ctx), a, em, s, ct);
  check_launch("encrypt_combine");
}

void decrypt_combine(const fhe_ctx* ctx, uint32_t nl, uint32_t nlim, const uint64_t* ct, const uint64_t* s,
                     uint64_t* m, hipStream_t st) {
  hipLaunchKernelGGL(k_decrypt_combine, dim3(grid_for((uint64_t)nlim << ctx->p.logN)), dim3(kThreads), 0, st, nl, nlim,
                     ctx->p.logN, mods_of(ctx), ct, s, m);
  check_launch("decrypt_combine");
}

void add_ct(const fhe_ctx* ctx, uint32_t ncomp, uint32_t nl, const uint64_t* a, const uint64_t* b, uint64_t* out,
            hipStream_t st) {
  hipLaunchKernelGGL(k_add, dim3(grid_for((uint64_t)ncomp * nl << ctx->p.logN)), dim3(kThreads), 0, st, ncomp, nl,
                     ctx->p.logN, mods_of(ctx), a, b, out);
  check_launch("add");
}

}  // namespace fhe
