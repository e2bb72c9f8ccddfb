// Context tables, key generation, encryption/decryption and single-ciphertext operations.
#include <algorithm>
#include <cstdlib>

#include "ckks.h"

#include <cmath>
#include <cstring>
#include <thread>

#include "host_math.h"

namespace fhe {

namespace {

uint32_t bitrev(uint32_t x, uint32_t bits) {
  uint32_t r = 0;
  for (uint32_t i = 0; i < bits; ++i) {
    r = (r << 1) | (x & 1);
    x >>= 1;
  }
  return r;
}

// Runs f(i) for i in [0, n) on up to 16 host threads.
template <class F>
void par_items(uint32_t n, F f) {
  unsigned w = std::thread::hardware_concurrency();
  if (w == 0) w = 1;
  if (w > 16) w = 16;
  if (w > n) w = n;
  if (w <= 1) {
    for (uint32_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::vector<std::thread> th;
  for (unsigned t = 0; t < w; ++t)
    th.emplace_back([=] {
      for (uint32_t i = t; i < n; i += w) f(i);
    });
  for (auto& x : th) x.join();
}

void sync(hipStream_t st) { HIPCHECK(hipStreamSynchronize(st)); }

}  // namespace

void ctx_init(fhe_ctx* ctx, const fhe_params_desc* d) {
  Params& p = ctx->p;
  p.d = *d;
  if (d->log_n < 12 || d->log_n > 17) fail(FHE_EINVAL, "log_n must be in [12, 17]");
  if (d->n_q < 3) fail(FHE_ELEVEL, "the method needs at least 3 Q primes (two rescales)");
  if (d->n_q > 64) fail(FHE_EINVAL, "n_q must be <= 64");
  if (d->q_bits < 30 || d->q_bits > 50) fail(FHE_EINVAL, "q_bits must be in [30, 50]");
  if (d->n_p < 1 || d->n_p > 8) fail(FHE_EINVAL, "n_p must be in [1, 8]");
  if (d->p_bits <= d->q_bits || d->p_bits > 61) fail(FHE_EINVAL, "p_bits must be in (q_bits, 61]");
  if (d->alpha < 1 || d->alpha > 8 || d->alpha > d->n_q) fail(FHE_EINVAL, "alpha must be in [1, min(8, n_q)]");
  if (d->rot_digits < 1 || d->rot_digits > d->log_n - 1) fail(FHE_EINVAL, "rot_digits must be in [1, log_n - 1]");
  if (d->log_delta < 1 || d->log_delta > 60 || d->mask_bits < 0 || d->mask_bits > 20)
    fail(FHE_EINVAL, "log_delta / mask_bits out of range");
  ctx->device = d->device;
  ctx->al = current_allocator();
  {  // released results kept for reuse: FHE_RESULT_POOL_MB (default 4096 MiB, 0 keeps none)
    const char* e = std::getenv("FHE_RESULT_POOL_MB");
    const long long mb = e ? std::max(0LL, std::atoll(e)) : 4096;
    ctx->results->clear((size_t)mb << 20);
  }
  HIPCHECK(hipSetDevice(d->device));
  noalloc_setup(d->device);
  p.logN = d->log_n;
  p.N = 1u << p.logN;
  p.S = p.N / 2;
  p.nq = d->n_q;
  p.np = d->n_p;
  p.alpha = d->alpha;
  p.rot_digits = d->rot_digits;
  p.rot_bits = (int)((p.logN - 1 + p.rot_digits - 1) / p.rot_digits);
  // NTT split: rows of 2^9 once N >= 2^15 (the column phase then has whole 3-stage rounds and
  // wider row segments), halves below. FHE_NTT_K1 overrides it (any split gives the same
  // transform; it only changes how the stages are grouped).
  p.k1 = p.logN >= 15 ? p.logN - 9 : p.logN / 2;
  if (const char* e = std::getenv("FHE_NTT_K1")) {
    const int v = std::atoi(e);
    if (v >= (int)p.logN - 9 && v <= 9 && v >= 1 && v < (int)p.logN) p.k1 = (uint32_t)v;
  }
  // row-phase workgroup shape (same results either way): FHE_ROWS_NT=256 or the autotuner
  if (const char* e = std::getenv("FHE_ROWS_NT")) p.rows_nt = std::atoi(e) == 256 ? 256 : 512;
  const uint64_t m = 2ull * p.N;
  std::vector<uint64_t> qs = primes_below(d->q_bits, p.nq, m);
  if ((int)qs.size() != p.nq) fail(FHE_EINVAL, "not enough Q primes of the requested size");
  std::vector<uint64_t> ps = primes_below(d->p_bits, p.np, m);
  if ((int)ps.size() != p.np) fail(FHE_EINVAL, "not enough P primes of the requested size");
  p.moduli = qs;
  p.moduli.insert(p.moduli.end(), ps.begin(), ps.end());
  const int nmod = p.nmod();
  const uint32_t N = p.N;
  hipStream_t st = nullptr;

  // Per-modulus constants and NTT twiddles.
  std::vector<ModInfo> mi(nmod);
  std::vector<uint64_t> tw((size_t)nmod * 4 * N);
  std::vector<double> twf((size_t)nmod * 4 * N);
  for (int i = 0; i < nmod; ++i) {
    const uint64_t q = p.moduli[i];
    ModInfo& x = mi[i];
    memset(&x, 0, sizeof(x));
    x.q = q;
    x.qinv = mont_qinv(q);
    const uint64_t r = (uint64_t)(((u128)1 << 64) % q);
    x.r2 = mulmod_host(r, r, q);
    x.n_inv = invmod_host(N % q, q);
    x.n_inv_shoup = shoup_prep(x.n_inv, q);
    const uint64_t psi = root_2n(N, q), psi_inv = invmod_host(psi, q);
    uint64_t* f = tw.data() + (size_t)i * 4 * N;
    // psi^k and psi^-k for k < N, then bit-reversed placement.
    std::vector<uint64_t> pp(N), pi(N);
    pp[0] = pi[0] = 1;
    for (uint32_t k = 1; k < N; ++k) {
      pp[k] = mulmod_host(pp[k - 1], psi, q);
      pi[k] = mulmod_host(pi[k - 1], psi_inv, q);
    }
    for (uint32_t k = 0; k < N; ++k) {
      const uint32_t rk = bitrev(k, p.logN);
      // (twiddle, companion) pairs interleaved so one 16-byte load fetches both
      f[2 * k] = pp[rk];
      f[2 * k + 1] = shoup_prep(pp[rk], q);
      f[2 * N + 2 * k] = pi[rk];
      f[2 * N + 2 * k + 1] = shoup_prep(pi[rk], q);
      // FP64 twiddles (used for q < 2^50): w and fl(w / q).
      double* ff = twf.data() + (size_t)i * 4 * N;
      ff[2 * k] = (double)pp[rk];
      ff[2 * k + 1] = (double)pp[rk] / (double)q;
      ff[2 * N + 2 * k] = (double)pi[rk];
      ff[2 * N + 2 * k + 1] = (double)pi[rk] / (double)q;
    }
  }
  ctx->t.mods = upload(mi, st);
  ctx->t.tw = upload(tw, st);
  ctx->t.twf = upload(twf, st);

  // ModUp constants per level.
  const int K = p.np;
  std::vector<uint64_t> mu;
  ctx->t.modup_offset.assign(p.nq + 1, 0);
  for (int nl = 1; nl <= p.nq; ++nl) {
    ctx->t.modup_offset[nl] = mu.size();
    const int beta = p.beta(nl), next = nl + K, a = p.alpha;
    for (int j = 0; j < beta; ++j) {
      const int lo = j * a, cnt = std::min(a, nl - lo);
      std::vector<uint64_t> blk(2 * a + 2 * (size_t)a * next, 0);
      for (int i = 0; i < cnt; ++i) {
        const uint64_t qi = p.moduli[lo + i];
        uint64_t dh = 1;
        for (int i2 = 0; i2 < cnt; ++i2)
          if (i2 != i) dh = mulmod_host(dh, p.moduli[lo + i2] % qi, qi);
        const uint64_t inv = invmod_host(dh, qi);
        blk[2 * i] = inv;
        blk[2 * i + 1] = shoup_prep(inv, qi);
        for (int e = 0; e < next; ++e) {
          const uint64_t t = p.moduli[e < nl ? e : p.nq + (e - nl)];
          uint64_t v = 1;
          for (int i2 = 0; i2 < cnt; ++i2)
            if (i2 != i) v = mulmod_host(v, p.moduli[lo + i2] % t, t);
          blk[2 * a + 2 * ((size_t)i * next + e)] = v;
          blk[2 * a + 2 * ((size_t)i * next + e) + 1] = shoup_prep(v, t);
        }
      }
      mu.insert(mu.end(), blk.begin(), blk.end());
    }
  }
  ctx->t.modup = upload(mu, st);

  // ModDown constants.
  std::vector<uint64_t> md(4 * K + 2 * (size_t)K * p.nq + 3 * (size_t)p.nq, 0);
  for (int kk = 0; kk < K; ++kk) {
    const uint64_t pk = p.moduli[p.nq + kk];
    uint64_t ph = 1;
    for (int k2 = 0; k2 < K; ++k2)
      if (k2 != kk) ph = mulmod_host(ph, p.moduli[p.nq + k2] % pk, pk);
    const uint64_t inv = invmod_host(ph, pk);
    md[2 * kk] = inv;
    md[2 * kk + 1] = shoup_prep(inv, pk);
    // the same factor times N^-1 (the fused kernel applies both after the inverse column phase)
    const uint64_t inv_n = mulmod_host(inv, invmod_host((uint64_t)p.N % pk, pk), pk);
    const size_t tail = 2 * K + 2 * (size_t)K * p.nq + 3 * (size_t)p.nq;
    md[tail + 2 * kk] = inv_n;
    md[tail + 2 * kk + 1] = shoup_prep(inv_n, pk);
    for (int i = 0; i < p.nq; ++i) {
      const uint64_t qi = p.moduli[i];
      uint64_t v = 1;
      for (int k2 = 0; k2 < K; ++k2)
        if (k2 != kk) v = mulmod_host(v, p.moduli[p.nq + k2] % qi, qi);
      md[2 * K + 2 * ((size_t)kk * p.nq + i)] = v;
      md[2 * K + 2 * ((size_t)kk * p.nq + i) + 1] = shoup_prep(v, qi);
    }
  }
  for (int i = 0; i < p.nq; ++i) {
    const uint64_t qi = p.moduli[i];
    uint64_t P = 1;
    for (int kk = 0; kk < K; ++kk) P = mulmod_host(P, p.moduli[p.nq + kk] % qi, qi);
    const uint64_t inv = invmod_host(P, qi);
    md[2 * K + 2 * (size_t)K * p.nq + 2 * i] = inv;
    md[2 * K + 2 * (size_t)K * p.nq + 2 * i + 1] = shoup_prep(inv, qi);
    md[2 * K + 2 * (size_t)K * p.nq + 2 * (size_t)p.nq + i] = P;
  }
  ctx->t.moddown = upload(md, st);
  // FP64 form of the conversion constants for the fused kernel: per (k, i) the pair
  // c0 = (P/p_k) mod q_i and c1 = c0 2^30 mod q_i, each with fl(c / q_i).
  std::vector<double> mdf(4 * (size_t)K * p.nq, 0.0);
  for (int kk = 0; kk < K; ++kk)
    for (int i = 0; i < p.nq; ++i) {
      const uint64_t qi = p.moduli[i];
      const uint64_t c0 = md[2 * K + 2 * ((size_t)kk * p.nq + i)];
      const uint64_t c1 = mulmod_host(c0, ((uint64_t)1 << 30) % qi, qi);
      double* f = mdf.data() + 4 * ((size_t)kk * p.nq + i);
      f[0] = (double)c0;
      f[1] = (double)c0 / (double)qi;
      f[2] = (double)c1;
      f[3] = (double)c1 / (double)qi;
    }
  ctx->t.moddown_f = upload(mdf, st);

  // Rescale constants: q_l^-1 mod q_i for i < l.
  std::vector<uint64_t> rs(2 * (size_t)p.nq * p.nq, 0);
  for (int l = 1; l < p.nq; ++l)
    for (int i = 0; i < l; ++i) {
      const uint64_t qi = p.moduli[i];
      const uint64_t inv = invmod_host(p.moduli[l] % qi, qi);
      rs[2 * ((size_t)l * p.nq + i)] = inv;
      rs[2 * ((size_t)l * p.nq + i) + 1] = shoup_prep(inv, qi);
    }
  ctx->t.rescale = upload(rs, st);

  // Base mask: the encoding of the one-hot vector e_0 at scale 2^mask_bits * q_(nq-2).
  const double one = 1.0;
  const double dm = std::ldexp((double)p.moduli[p.nq - 2], d->mask_bits);
  ctx->t.base_mask.assign(N, 0);
  encode_real(&one, 1, dm, N, ctx->t.base_mask.data());
  DevBuf mint = upload(ctx->t.base_mask, st);
  const uint32_t nml = p.nq - 1;
  ctx->t.mask = DevBuf((size_t)nml * N * 8, st);
  signed_to_limbs(ctx, (const int64_t*)mint.get(), nml, nml, 0, ctx->t.mask.u64(), st);
  ntt_forward(ctx, LimbBatch{ctx->t.mask.u64(), nml, 1, (uint64_t)nml * N, nml, 0}, st);
  ctx->t.mask_f = DevBuf((size_t)nml * N * 8, st);
  to_f64_bits(ctx, (uint64_t)nml * N, ctx->t.mask.u64(), ctx->t.mask_f.u64(), st);
  to_montgomery(ctx, ctx->t.mask.u64(), nml, nml, 0, st);
  sync(st);
}

size_t ctx_key_bytes(const fhe_ctx* ctx) {
  size_t b = ctx->relin ? ctx->relin->buf.bytes() : 0;
  for (const auto& kv : ctx->rot) b += kv.second->buf.bytes();
  return b;
}

size_t ctx_resident_bytes(const fhe_ctx* ctx) {
  const Tables& t = ctx->t;
  return ctx_key_bytes(ctx) + t.mods.bytes() + t.tw.bytes() + t.twf.bytes() + t.modup.bytes() + t.moddown.bytes() +
         t.moddown_f.bytes() + t.rescale.bytes() + t.mask.bytes() + t.mask_f.bytes();
}

std::vector<uint32_t> rotation_steps(const Params& p, int64_t r) {
  std::vector<uint32_t> out;
  int64_t rr = r % (int64_t)p.S;
  if (rr < 0) rr += p.S;
  if (rr == 0) return out;
  const uint32_t b = (uint32_t)p.rot_bits, mask = (1u << b) - 1;
  for (int t = 0; t < p.rot_digits; ++t) {
    const uint32_t rt = ((uint32_t)rr >> (b * t)) & mask;
    if (rt) out.push_back(rt << (b * t));
  }
  return out;
}

uint32_t galois_of_step(const Params& p, uint32_t step) {
  const uint64_t m = 2ull * p.N;
  uint64_t g = 1, base = 5;
  for (uint32_t e = step; e; e >>= 1) {
    if (e & 1) g = g * base % m;
    base = base * base % m;
  }
  return (uint32_t)g;
}

uint32_t mask_galois(const Params& p, int slot) { return galois_of_step(p, (p.S - (uint32_t)slot) % p.S); }

const SwitchKey* rotation_key(const fhe_ctx* ctx, uint32_t step) {
  auto it = ctx->rot.find(galois_of_step(ctx->p, step));
  if (it == ctx->rot.end()) fail(FHE_EKEY, "rotation key for step " + std::to_string(step) + " not generated");
  return it->second.get();
}

namespace {

// One switching key for target secret s' (NTT domain on all limbs, device).
std::unique_ptr<SwitchKey> make_switch_key(fhe_ctx* ctx, const fhe_sk* sk, uint64_t key_id, uint64_t kind_a,
                                           uint64_t kind_e, const uint64_t* sp, hipStream_t st) {
  const Params& p = ctx->p;
  const uint32_t N = p.N, nall = p.nmod(), beta = p.beta(p.nq);
  auto key = std::make_unique<SwitchKey>();
  key->buf = DevBuf((size_t)beta * 2 * nall * N * 8, st);
  std::vector<uint64_t> ah((size_t)nall * N);
  std::vector<int64_t> eh(N);
  DevBuf da((size_t)nall * N * 8, st), de((size_t)nall * N * 8, st), dei(N * 8, st), dpf(nall * 8, st);
  // P mod q_i for the digit term.
  std::vector<uint64_t> pmod(nall, 0);
  for (int i = 0; i < p.nq; ++i) {
    uint64_t v = 1;
    for (int kk = 0; kk < p.np; ++kk) v = mulmod_host(v, p.moduli[p.nq + kk] % p.moduli[i], p.moduli[i]);
    pmod[i] = v;
  }
  for (uint32_t j = 0; j < beta; ++j) {
    par_items(nall + 1, [&](uint32_t i) {
      if (i < nall) sample_uniform(sk->seed, stream_tag(kind_a, key_id, j, i), p.moduli[i], N, ah.data() + (size_t)i * N);
      else sample_gauss(sk->seed, stream_tag(kind_e, key_id, j, 0), N, eh.data());
    });
    std::vector<uint64_t> pf(nall, 0);
    for (int i = 0; i < p.nq; ++i)
      if (i / p.alpha == (int)j) pf[i] = pmod[i];
    HIPCHECK(hipMemcpyAsync(da.get(), ah.data(), ah.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHECK(hipMemcpyAsync(dei.get(), eh.data(), eh.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHECK(hipMemcpyAsync(dpf.get(), pf.data(), pf.size() * 8, hipMemcpyHostToDevice, st));
    signed_to_limbs(ctx, (const int64_t*)dei.get(), nall, nall, 0, de.u64(), st);
    ntt_forward(ctx, LimbBatch{da.u64(), nall, 1, (uint64_t)nall * N, nall, 0}, st);
    ntt_forward(ctx, LimbBatch{de.u64(), nall, 1, (uint64_t)nall * N, nall, 0}, st);
    uint64_t* bout = key->buf.u64() + ((size_t)j * 2 + 0) * nall * N;
    uint64_t* aout = key->buf.u64() + ((size_t)j * 2 + 1) * nall * N;
    keygen_digit(ctx, nall, da.u64(), sk->s_ntt.u64(), de.u64(), sp, dpf.u64(), bout, aout, st);
    sync(st);  // host buffers are reused for the next digit
  }
  return key;
}

}  // namespace

void keygen(fhe_ctx* ctx, uint64_t seed, hipStream_t st, fhe_sk* sk) {
  const Params& p = ctx->p;
  const uint32_t N = p.N, nall = p.nmod();
  sk->seed = seed;
  sk->s.assign(N, 0);
  sample_ternary(seed, stream_tag(kTagSecret, 0, 0, 0), N, sk->s.data());
  DevBuf si = upload(sk->s, st);
  sk->s_ntt = DevBuf((size_t)nall * N * 8, st);
  signed_to_limbs(ctx, (const int64_t*)si.get(), nall, nall, 0, sk->s_ntt.u64(), st);
  ntt_forward(ctx, LimbBatch{sk->s_ntt.u64(), nall, 1, (uint64_t)nall * N, nall, 0}, st);
  DevBuf s2((size_t)nall * N * 8, st);
  square(ctx, nall, sk->s_ntt.u64(), s2.u64(), st);
  ctx->relin = make_switch_key(ctx, sk, 0, kTagRelinA, kTagRelinE, s2.u64(), st);
  ctx->rot.clear();
  if (p.rot_digits >= 2) {
    std::vector<uint32_t> steps;
    const uint32_t b = p.rot_bits;
    for (int t = 0; t < p.rot_digits; ++t)
      for (uint32_t r = 1; r < (1u << b); ++r) {
        const uint64_t amount = (uint64_t)r << (b * t);
        if (amount < p.S) steps.push_back((uint32_t)amount);
      }
    keygen_rotation_steps(ctx, sk, steps, st);
  }
  sync(st);
}

void keygen_rotation_steps(fhe_ctx* ctx, const fhe_sk* sk, const std::vector<uint32_t>& steps, hipStream_t st) {
  const Params& p = ctx->p;
  const uint32_t N = p.N, nall = p.nmod();
  DevBuf sp((size_t)nall * N * 8, st);
  for (uint32_t step : steps) {
    if (step == 0 || step >= p.S) fail(FHE_EINVAL, "rotation step out of range");
    const uint32_t g = galois_of_step(p, step);
    if (ctx->rot.count(g)) continue;
    ArgPack ap;
    size_t o_src = ap.push(std::vector<const uint64_t*>{sk->s_ntt.u64()});
    size_t o_g = ap.push(std::vector<uint32_t>{g});
    ap.upload(st);
    automorph(ctx, 1, 1, nall, ap.at<const uint64_t*>(o_src), ap.at<uint32_t>(o_g), sp.u64(), st);
    ctx->rot[g] = make_switch_key(ctx, sk, g, kTagRotA, kTagRotE, sp.u64(), st);
  }
}

void encrypt_values(fhe_ctx* ctx, const fhe_sk* sk, const double* values, int64_t nnz, double delta, uint64_t seed,
                    hipStream_t st, fhe_mat* out) {
  const Params& p = ctx->p;
  const uint32_t N = p.N, S = p.S, nq = p.nq;
  const int nch = nnz == 0 ? 1 : (int)((nnz + S - 1) / S);
  out->nl = nq;
  out->nchunks = nch;
  out->scale = delta;
  out->data = DevBuf((size_t)nch * 2 * nq * N * 8, st);
  std::vector<int64_t> m(N), e(N);
  std::vector<uint64_t> ah((size_t)nq * N);
  DevBuf dem(N * 8, st), demq((size_t)nq * N * 8, st), da((size_t)nq * N * 8, st);
  for (int c = 0; c < nch; ++c) {
    const int64_t lo = (int64_t)c * S;
    const uint32_t cnt = (uint32_t)std::max<int64_t>(0, std::min<int64_t>(S, nnz - lo));
    encode_real(values + lo, cnt, delta, N, m.data());
    par_items(nq + 1, [&](uint32_t i) {
      if (i < nq) sample_uniform(seed, stream_tag(kTagEncA, c, 0, i), p.moduli[i], N, ah.data() + (size_t)i * N);
      else sample_gauss(seed, stream_tag(kTagEncE, c, 0, 0), N, e.data());
    });
    for (uint32_t k = 0; k < N; ++k) e[k] += m[k];
    HIPCHECK(hipMemcpyAsync(dem.get(), e.data(), N * 8, hipMemcpyHostToDevice, st));
    HIPCHECK(hipMemcpyAsync(da.get(), ah.data(), ah.size() * 8, hipMemcpyHostToDevice, st));
    signed_to_limbs(ctx, (const int64_t*)dem.get(), nq, nq, 0, demq.u64(), st);
    ntt_forward(ctx, LimbBatch{demq.u64(), nq, 1, (uint64_t)nq * N, nq, 0}, st);
    ntt_forward(ctx, LimbBatch{da.u64(), nq, 1, (uint64_t)nq * N, nq, 0}, st);
    encrypt_combine(ctx, nq, da.u64(), demq.u64(), sk->s_ntt.u64(), out->chunk(c, N), st);
    sync(st);
  }
}

void decrypt_decode_chunk(fhe_ctx* ctx, const fhe_sk* sk, const uint64_t* chunk, int nl, double scale, hipStream_t st,
                          std::vector<double>& slots) {
  const Params& p = ctx->p;
  const uint32_t N = p.N;
  if (nl < 2) fail(FHE_ELEVEL, "decryption needs at least two limbs");
  DevBuf dm((size_t)2 * N * 8, st);
  decrypt_combine(ctx, nl, 2, chunk, sk->s_ntt.u64(), dm.u64(), st);
  ntt_inverse(ctx, LimbBatch{dm.u64(), 2, 1, (uint64_t)2 * N, 2, 0}, st);
  std::vector<uint64_t> h((size_t)2 * N);
  HIPCHECK(hipMemcpyAsync(h.data(), dm.get(), h.size() * 8, hipMemcpyDeviceToHost, st));
  sync(st);
  const uint64_t q0 = p.moduli[0], q1 = p.moduli[1];
  const u128 Q = (u128)q0 * q1;
  const uint64_t q0inv = invmod_host(q0 % q1, q1);
  std::vector<double> mm(N);
  for (uint32_t k = 0; k < N; ++k) {
    const uint64_t r0 = h[k], r1 = h[N + k];
    const uint64_t t = mulmod_host((r1 + q1 - r0 % q1) % q1, q0inv, q1);
    const u128 x = (u128)r0 + (u128)q0 * t;
    mm[k] = x > Q / 2 ? -(double)(Q - x) : (double)x;
  }
  slots.assign(p.S, 0.0);
  decode_all(mm.data(), N, scale, slots.data());
}

void export_coeffs(fhe_ctx* ctx, const uint64_t* data, int ncomp, int nl, hipStream_t st, uint64_t* host_out) {
  const uint32_t N = ctx->p.N;
  const size_t n = (size_t)ncomp * nl * N;
  DevBuf tmp(n * 8, st);
  HIPCHECK(hipMemcpyAsync(tmp.get(), data, n * 8, hipMemcpyDeviceToDevice, st));
  ntt_inverse(ctx, LimbBatch{tmp.u64(), (uint32_t)nl, (uint32_t)ncomp, (uint64_t)nl * N, (uint32_t)nl, 0}, st);
  HIPCHECK(hipMemcpyAsync(host_out, tmp.get(), n * 8, hipMemcpyDeviceToHost, st));
  sync(st);
}

void ct_rotate(fhe_ctx* ctx, const uint64_t* src, int nl, int64_t r, uint64_t* dst, hipStream_t st) {
  const Params& p = ctx->p;
  const uint32_t N = p.N;
  std::vector<uint32_t> steps = rotation_steps(p, r);
  if (steps.empty()) {
    HIPCHECK(hipMemcpyAsync(dst, src, (size_t)2 * nl * N * 8, hipMemcpyDeviceToDevice, st));
    return;
  }
  DevBuf tmp((size_t)2 * nl * N * 8, st);
  DevBuf ws(keyswitch_ws_elems(ctx, 1, nl) * 8, st);
  const uint64_t* cur = src;
  for (uint32_t step : steps) {
    const SwitchKey* key = rotation_key(ctx, step);
    ArgPack ap;
    size_t o_src = ap.push(std::vector<const uint64_t*>{cur});
    size_t o_g = ap.push(std::vector<uint32_t>{galois_of_step(p, step)});
    size_t o_key = ap.push(std::vector<const uint64_t*>{key->buf.u64()});
    size_t o_add = ap.push(std::vector<const uint64_t*>{tmp.u64(), nullptr});
    size_t o_out = ap.push(std::vector<uint64_t*>{dst});
    ap.upload(st);
    automorph(ctx, 1, 2, nl, ap.at<const uint64_t*>(o_src), ap.at<uint32_t>(o_g), tmp.u64(), st);
    keyswitch(ctx, 1, nl, tmp.u64() + (size_t)nl * N, 0, ap.at<const uint64_t*>(o_key), ap.at<const uint64_t*>(o_add),
              ap.at<uint64_t*>(o_out), ws.u64(), st);
    sync(st);
    cur = dst;
  }
}

void ct_mult_relin(fhe_ctx* ctx, const uint64_t* a, const uint64_t* b, int nl, uint64_t* dst, hipStream_t st) {
  const uint32_t N = ctx->p.N;
  if (!ctx->relin) fail(FHE_EKEY, "relinearisation key not generated");
  DevBuf d((size_t)3 * nl * N * 8, st);
  DevBuf ws(keyswitch_ws_elems(ctx, 1, nl) * 8, st);
  ArgPack ap;
  size_t o_a = ap.push(std::vector<const uint64_t*>{a});
  size_t o_b = ap.push(std::vector<const uint64_t*>{b});
  size_t o_key = ap.push(std::vector<const uint64_t*>{ctx->relin->buf.u64()});
  size_t o_add = ap.push(std::vector<const uint64_t*>{d.u64(), d.u64() + (size_t)nl * N});
  size_t o_out = ap.push(std::vector<uint64_t*>{dst});
  ap.upload(st);
  tensor(ctx, 1, nl, ap.at<const uint64_t*>(o_a), ap.at<const uint64_t*>(o_b), d.u64(), st);
  keyswitch(ctx, 1, nl, d.u64() + (size_t)2 * nl * N, 0, ap.at<const uint64_t*>(o_key), ap.at<const uint64_t*>(o_add),
            ap.at<uint64_t*>(o_out), ws.u64(), st);
  sync(st);
}

void ct_rescale(fhe_ctx* ctx, const uint64_t* src, int ncomp, int nl, uint64_t* dst, hipStream_t st) {
  DevBuf ws(rescale_ws_elems(ctx, 1, ncomp, nl) * 8, st);
  ArgPack ap;
  size_t o_in = ap.push(std::vector<const uint64_t*>{src});
  size_t o_out = ap.push(std::vector<uint64_t*>{dst});
  ap.upload(st);
  rescale(ctx, 1, ncomp, nl, ap.at<const uint64_t*>(o_in), ap.at<uint64_t*>(o_out), ws.u64(), st);
  sync(st);
}

void ct_mask(fhe_ctx* ctx, const uint64_t* src, int nl, int slot, uint64_t* dst, hipStream_t st) {
  ArgPack ap;
  size_t o_in = ap.push(std::vector<const uint64_t*>{src});
  size_t o_g = ap.push(std::vector<uint32_t>{mask_galois(ctx->p, slot)});
  size_t o_out = ap.push(std::vector<uint64_t*>{dst});
  ap.upload(st);
  mask_mul(ctx, 1, nl, ap.at<const uint64_t*>(o_in), ap.at<uint32_t>(o_g), ap.at<uint64_t*>(o_out), st);
  sync(st);
}

}  // namespace fhe
