// Launchers of the gfx950 kernels. All pointers are device pointers; arrays of per-item pointers
// (`const uint64_t* const*` etc.) live in device memory. Every launcher enqueues on `st`.
#pragma once
#include "common.h"

namespace fhe {

// A batch of limbs to transform: poly p, limb e is at base + p * poly_stride + e * N and uses
// modulus index e (e < n_first) or p_base + (e - n_first) (e >= n_first).
// Optional: `src` (with src_stride per poly) is where the first phase reads from (out of place);
// a "hole" skips a key-switch digit's own limbs in compacted ModUp rows: with hole_items > 0, poly p
// belongs to digit j = hole_j0 + p / hole_items and rows e >= j * hole_alpha (and < n_first) map to
// modulus e + hole_len.
struct LimbBatch {
  uint64_t* base;
  uint32_t limbs;
  uint32_t npoly;
  uint64_t poly_stride;
  uint32_t n_first;
  uint32_t p_base;
  const uint64_t* src = nullptr;
  uint64_t src_stride = 0;
  uint32_t hole_items = 0, hole_alpha = 0, hole_len = 0, hole_j0 = 0;
  // Nonzero: Q-prime limbs are written in the FP64 kernels' internal form (the bits of a double
  // holding a representative in [-q/2 - 2, q/2 + 2]) instead of [0, q) integers; special-prime
  // limbs are unaffected. Only for forward transforms and the row phase of inverse ones, whose
  // consumers are the fused key-switch / rescale kernels.
  uint32_t raw_out = 0;
  // Optional, for the phase that reads `src` in a row-phase (phase 2) launch: poly p is read from
  // src_ptr[p] ([limbs][N]) through the automorphism tau_(src_gal[p]) (device arrays).
  const uint64_t* const* src_ptr = nullptr;
  const uint32_t* src_gal = nullptr;
  uint32_t src_ptr_limb0 = 0;  // limb of src_ptr[p] that this batch's limb 0 reads
};

// Negacyclic NTT, in place. Forward: coefficients -> evaluations at psi^(2 brv(i) + 1) (bit-reversed
// order); inverse: back to coefficients (N^-1 included).
void ntt_forward(const fhe_ctx* ctx, const LimbBatch& lb, hipStream_t st);
void ntt_inverse(const fhe_ctx* ctx, const LimbBatch& lb, hipStream_t st);

// dst[b] = tau_(galois[b]) (src[b]) in the NTT domain; src[b] is [ncomp][nl][N]; dst contiguous
// [B][ncomp][nl][N].
void automorph(const fhe_ctx* ctx, uint32_t B, uint32_t ncomp, uint32_t nl, const uint64_t* const* src,
               const uint32_t* galois, uint64_t* dst, hipStream_t st);

// out (contiguous [B][3][nl][N]) = (a0 b0, a0 b1 + a1 b0, a1 b1) per item, NTT domain.
void tensor(const fhe_ctx* ctx, uint32_t B, uint32_t nl, const uint64_t* const* a, const uint64_t* const* b,
            uint64_t* out, hipStream_t st);

// Hybrid key switch of B polynomials at nl limbs (NTT domain). Input item b is `in + b * in_stride`
// ([nl][N]); it is read, not modified. keys[b]: switching key. add[2b + c] (may be NULL): [nl][N] added to
// output component c. out[b]: [2][nl][N]. ws: keyswitch_ws_elems(ctx, B, nl) uint64 of workspace.
// With galois (device array of B Galois elements), add[2b] (component 0) is read through the
// automorphism tau_(galois[b]) (NTT domain): a rotation then needs tau of component 1 only; out[b]
// must not overlap add[2b] in that case. With galois and in_ptrs (device array of B pointers to
// [nl][N]), input item b is tau_(galois[b])(in_ptrs[b]), read through the automorphism by the
// kernels themselves (`in` and in_stride are unused): a rotation then runs no separate
// automorphism launch at all.
size_t keyswitch_ws_elems(const fhe_ctx* ctx, uint32_t B, uint32_t nl);
void keyswitch(const fhe_ctx* ctx, uint32_t B, uint32_t nl, const uint64_t* in, uint64_t in_stride,
               const uint64_t* const* keys, const uint64_t* const* add, uint64_t* const* out, uint64_t* ws,
               hipStream_t st, const uint32_t* galois = nullptr, const uint64_t* const* in_ptrs = nullptr);

// Hoisted key switches of B rotations of S polynomials (S <= B): state_c1[s] ([nl][N], NTT domain;
// `ident`: S Galois elements equal to 1) gets ModUp and the forward transform of its digits once;
// item b then switches tau_(galois[b])(state_c1[state_of[b]]) with keys[b], reading those digits through
// the automorphism (in_ptrs[b] = state_c1[state_of[b]]). add/out as in keyswitch (with galois). ws:
// keyswitch_ws_elems(ctx, B, nl). The digits of tau(x) are tau(ModUp(x)) here, not ModUp(tau(x)): the
// same rotation up to noise, other limbs.
void keyswitch_hoisted(const fhe_ctx* ctx, uint32_t S, uint32_t B, uint32_t nl, const uint64_t* const* state_c1,
                       const uint32_t* ident, const uint32_t* state_of, const uint64_t* const* in_ptrs,
                       const uint32_t* galois, const uint64_t* const* keys, const uint64_t* const* add,
                       uint64_t* const* out, uint64_t* ws, hipStream_t st);

// Rescale of B ciphertexts [ncomp][nl][N] -> [ncomp][nl-1][N] (nearest rounding of the dropped limb).
// With mask_galois (device array of B Galois elements, needs rescale_fuses_mask and nl <= nq - 1),
// every input is first multiplied by its one-hot mask tau_(galois[b])(base mask), on the fly: the
// result equals mask_mul followed by rescale.
size_t rescale_ws_elems(const fhe_ctx* ctx, uint32_t B, uint32_t ncomp, uint32_t nl);
bool rescale_fuses_mask(const fhe_ctx* ctx);
void rescale(const fhe_ctx* ctx, uint32_t B, uint32_t ncomp, uint32_t nl, const uint64_t* const* in,
             uint64_t* const* out, uint64_t* ws, hipStream_t st, const uint32_t* mask_galois = nullptr);

// out[b] = in[b] * tau_(galois[b])(base mask) (one-hot mask), [2][nl][N], nl <= nq - 1.
void mask_mul(const fhe_ctx* ctx, uint32_t B, uint32_t nl, const uint64_t* const* in, const uint32_t* galois,
              uint64_t* const* out, hipStream_t st);

// Grouped masked sums (nl <= nq - 1): for segment s, accumulator seg[4s] (acc + seg[4s] * 2 nl N,
// [2][nl][N]) is set (seg[4s+3] = 1) or incremented (0) by the sum over entries e in
// [seg[4s+1], seg[4s+2]) of in[e] * tau_(galois[e])(base mask). `seg` (4 nseg words), `in` and
// `galois` (nentries each) are device arrays.
void mask_sum(const fhe_ctx* ctx, uint32_t nseg, uint32_t nentries, uint32_t nl, const uint32_t* seg,
              const uint64_t* const* in, const uint32_t* galois, uint64_t* acc, hipStream_t st);

// As accumulate, with the contributions given by a device array of pointers.
void accumulate_ptr(const fhe_ctx* ctx, uint32_t nseg, uint32_t ncontrib, uint32_t nl, const uint32_t* seg,
                    const uint64_t* const* contrib, uint64_t* const* results, hipStream_t st);

// x[i] = 0 for i < n (a kernel launch: usable inside a recorded graph).
void fill_zero(const fhe_ctx* ctx, uint64_t n, uint64_t* x, hipStream_t st);

// out[i] = the bits of in[i] as a double (values below 2^53), i < n.
void to_f64_bits(const fhe_ctx* ctx, uint64_t n, const uint64_t* in, uint64_t* out, hipStream_t st);

// results[seg[3s]] += sum of contrib[b] for b in [seg[3s+1], seg[3s+2]); [2][nl][N] each; `results` is
// a device array of result-chunk pointers. ncontrib (the number of contributions the segments cover)
// only sizes the launch's traffic figure for the kernel timer.
void accumulate(const fhe_ctx* ctx, uint32_t nseg, uint32_t ncontrib, uint32_t nl, const uint32_t* seg,
                const uint64_t* contrib,
                uint64_t* const* results, hipStream_t st);

// out[e][k] = v[k] mod modulus(e) for e < nlimbs (modulus index rule as in LimbBatch).
void signed_to_limbs(const fhe_ctx* ctx, const int64_t* v, uint32_t nlimbs, uint32_t n_first, uint32_t p_base,
                     uint64_t* out, hipStream_t st);

// x -> x R mod q (Montgomery form) on [nlimbs][N], modulus index rule as above.
void to_montgomery(const fhe_ctx* ctx, uint64_t* x, uint32_t nlimbs, uint32_t n_first, uint32_t p_base,
                   hipStream_t st);

// Switching-key digit on all nall limbs (NTT domain): b = e - a s + pfac_i s' (pfac_i = 0 outside the
// digit). Writes b and a as the doubles' bits of the residues on Q primes (FP64 key product) and in
// Montgomery form on special primes. pfac: [nall] (device).
void keygen_digit(const fhe_ctx* ctx, uint32_t nall, const uint64_t* a, const uint64_t* s, const uint64_t* e,
                  const uint64_t* sp, const uint64_t* pfac, uint64_t* bout, uint64_t* aout, hipStream_t st);

// s2 = s * s pointwise on [nall][N] (NTT domain).
void square(const fhe_ctx* ctx, uint32_t nall, const uint64_t* s, uint64_t* s2, hipStream_t st);

// Encryption: c0 = em - a s, c1 = a on [nl][N] (NTT domain); ct = [2][nl][N].
void encrypt_combine(const fhe_ctx* ctx, uint32_t nl, const uint64_t* a, const uint64_t* em, const uint64_t* s,
                     uint64_t* ct, hipStream_t st);

// m = c0 + c1 s on limbs [0, nlim) of ct [2][nl][N] (NTT domain) -> m [nlim][N].
void decrypt_combine(const fhe_ctx* ctx, uint32_t nl, uint32_t nlim, const uint64_t* ct, const uint64_t* s,
                     uint64_t* m, hipStream_t st);

// out = a + b, elementwise mod q on [ncomp][nl][N].
void add_ct(const fhe_ctx* ctx, uint32_t ncomp, uint32_t nl, const uint64_t* a, const uint64_t* b, uint64_t* out,
            hipStream_t st);

// Measurement hook: modular products per second of one form (0: FP64 product for q < 2^50, 1: lazy
// Shoup product, 2: Montgomery product, both for p < 2^61) over 8 independent chains of `iters`
// dependent products per thread on a full grid (second of two timed launches).
double bench_mulmod(int kind, uint32_t iters, hipStream_t st);

}  // namespace fhe
