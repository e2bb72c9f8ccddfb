// Host orchestration of the CKKS operations (context tables, keys, encryption, single-ciphertext ops).
#pragma once
#include <cstring>

#include "common.h"
#include "kernels.h"

namespace fhe {

// Packs small host arrays (pointer lists, Galois elements, segment tables) into one device upload.
class ArgPack {
 public:
  template <class T>
  size_t push(const std::vector<T>& v) {
    static_assert(sizeof(T) == 8 || sizeof(T) == 4, "8- or 4-byte items");
    size_t off = words_.size();
    size_t nw = (v.size() * sizeof(T) + 7) / 8;
    words_.resize(off + nw + 1, 0);
    if (!v.empty()) memcpy(words_.data() + off, v.data(), v.size() * sizeof(T));
    return off;
  }
  // Enqueues the copy on `st` (stream-ordered); the host words stay owned by this object.
  void upload(hipStream_t st) {
    buf_ = DevBuf(words_.size() * 8 + 8, st);
    if (!words_.empty())
      HIPCHECK(hipMemcpyAsync(buf_.get(), words_.data(), words_.size() * 8, hipMemcpyHostToDevice, st));
  }
  template <class T>
  T* at(size_t off) const {
    return (T*)(buf_.u64() + off);
  }
  size_t words() const { return words_.size(); }

 private:
  std::vector<uint64_t> words_;
  DevBuf buf_;
};

void ctx_init(fhe_ctx* ctx, const fhe_params_desc* d);
// One autotuner candidate: NTT split k1, row-phase threads per workgroup, time (ms).
struct TuneTrial {
  int k1 = 0, rows = 0;
  double ms = 0.0;
};
// Times top-level key switches of B synthetic polynomials for every admissible NTT split and
// row-phase shape, keeps the fastest in ctx (results are identical for every choice).
void autotune_split(fhe_ctx* ctx, hipStream_t st, uint32_t B, std::vector<TuneTrial>& tried, TuneTrial& best);
// As autotune_split, timing the first `pairs` matched pairs of A B (the real per-pair sequence).
void autotune_plan(fhe_ctx* ctx, hipStream_t st, const fhe_mat* A, const fhe_mat* B, int64_t pairs,
                   std::vector<TuneTrial>& tried, TuneTrial& best);
// Device bytes a context holds for good: constant tables and every evaluation key.
size_t ctx_resident_bytes(const fhe_ctx* ctx);
size_t ctx_key_bytes(const fhe_ctx* ctx);
void keygen(fhe_ctx* ctx, uint64_t seed, hipStream_t st, fhe_sk* sk);
void keygen_rotation_steps(fhe_ctx* ctx, const fhe_sk* sk, const std::vector<uint32_t>& steps, hipStream_t st);

// Left-rotation amount r (mod S) -> key-switched steps r_t 2^(b t), t ascending, zeros skipped.
std::vector<uint32_t> rotation_steps(const Params& p, int64_t r);
uint32_t galois_of_step(const Params& p, uint32_t step);
const SwitchKey* rotation_key(const fhe_ctx* ctx, uint32_t step);

// Encrypts S-slot chunks of `values` (nnz) at scale `delta` with the stream seed; returns [nch][2][nq][N].
void encrypt_values(fhe_ctx* ctx, const fhe_sk* sk, const double* values, int64_t nnz, double delta, uint64_t seed,
                    hipStream_t st, fhe_mat* out);
// Decrypts chunk data [2][nl][N] (NTT domain) and decodes all S slots.
void decrypt_decode_chunk(fhe_ctx* ctx, const fhe_sk* sk, const uint64_t* chunk, int nl, double scale, hipStream_t st,
                          std::vector<double>& slots);
// Coefficient-domain export of [ncomp][nl][N] NTT-domain data.
void export_coeffs(fhe_ctx* ctx, const uint64_t* data, int ncomp, int nl, hipStream_t st, uint64_t* host_out);

// Single-ciphertext operations (batch of one).
void ct_rotate(fhe_ctx* ctx, const uint64_t* src, int nl, int64_t r, uint64_t* dst, hipStream_t st);
// The no-alloc rotation (noalloc.hip): noalloc_setup resolves the static scratch array's device
// address on `device` (current) once; ct_rotate_noalloc is ct_rotate with all of its scratch in that
// array (dst may equal src), failing with FHE_ENOMEM when noalloc_rotate_bytes exceeds it.
void noalloc_setup(int device);
size_t noalloc_rotate_bytes(const fhe_ctx* ctx, uint32_t nl);
void ct_rotate_noalloc(fhe_ctx* ctx, const uint64_t* src, uint32_t nl, int64_t r, uint64_t* dst, hipStream_t st);
void ct_mult_relin(fhe_ctx* ctx, const uint64_t* a, const uint64_t* b, int nl, uint64_t* dst, hipStream_t st);
void ct_rescale(fhe_ctx* ctx, const uint64_t* src, int ncomp, int nl, uint64_t* dst, hipStream_t st);
void ct_mask(fhe_ctx* ctx, const uint64_t* src, int nl, int slot, uint64_t* dst, hipStream_t st);
uint32_t mask_galois(const Params& p, int slot);


}  // namespace fhe
