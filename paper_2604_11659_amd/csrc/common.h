// Internal types of the library: errors, device buffers, parameter set, context and handles.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "arith.h"
#include "fhe_spmspm.h"

namespace fhe {

// Internal failures are thrown as Error and converted to return codes at the C boundary.
struct Error {
  int code;
  std::string msg;
};
[[noreturn]] void fail(int code, const std::string& msg);
// Records msg as the calling thread's fhe_last_error() and returns code (entry points that return
// codes directly instead of throwing).
int set_error(int code, const char* msg);
void hip_check(hipError_t e, const char* what, const char* file, int line);
#define HIPCHECK(x) ::fhe::hip_check((x), #x, __FILE__, __LINE__)

struct Allocator {
  fhe_alloc_fn alloc = nullptr;
  fhe_free_fn free_ = nullptr;
  void* user = nullptr;
};
Allocator current_allocator();

// Per-kernel device timing (HIP events around tracked launches); see runtime.cpp.
int prof_begin(const char* name, hipStream_t st);
// algorithmic_bytes: the HBM reads + writes the launch must do; mulmods: the modular products it
// performs (an NTT butterfly, a pointwise or a base-conversion product count one each).
void prof_end(int tok, hipStream_t st, double algorithmic_bytes, double mulmods = 0.0);
void prof_enable(bool on);
// Adds n to the work counter `name` while timing is on (reported as "count:<name>" with n launches).
void prof_count(const char* name, int64_t n);
// While alive, launches on this thread are not timed (they are being captured into a graph).
// prof_count adds to the scope's own counters instead.
struct CaptureScope {
  CaptureScope();
  ~CaptureScope();
  int64_t count(const char* name) const;
};
struct ProfRow {
  std::string name;
  int64_t launches = 0;
  double ms = 0.0, bytes = 0.0, mulmods = 0.0;
};
std::vector<ProfRow> prof_summary();

// Owning device buffer, allocated and released through the registered allocator.
class DevBuf {
 public:
  DevBuf() = default;
  DevBuf(size_t bytes, hipStream_t stream);
  ~DevBuf() { reset(); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept { *this = std::move(o); }
  DevBuf& operator=(DevBuf&& o) noexcept;
  void reset();
  uint64_t* u64() const { return (uint64_t*)ptr_; }
  void* get() const { return ptr_; }
  size_t bytes() const { return bytes_; }

 private:
  void* ptr_ = nullptr;
  size_t bytes_ = 0;
  hipStream_t stream_ = nullptr;
  Allocator al_;
};

// Copies a host vector into a new device buffer (synchronous with respect to the host).
template <class T>
DevBuf upload(const std::vector<T>& v, hipStream_t stream) {
  DevBuf b(v.size() * sizeof(T) + 8, stream);
  if (!v.empty()) HIPCHECK(hipMemcpyAsync(b.get(), v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, stream));
  HIPCHECK(hipStreamSynchronize(stream));
  return b;
}

struct Params {
  fhe_params_desc d;
  uint32_t N = 0, logN = 0, S = 0;
  int nq = 0, np = 0, alpha = 1, rot_digits = 1, rot_bits = 0;
  std::vector<uint64_t> moduli;  // q_0..q_{nq-1}, p_0..p_{np-1}
  int nmod() const { return nq + np; }
  int beta(int nl) const { return (nl + alpha - 1) / alpha; }
  // NTT split: phase 1 transforms columns of 2^k1 elements, phase 2 rows of 2^(logN-k1).
  uint32_t k1 = 0;
  uint32_t rows_nt = 512;  // row-phase workgroups: 512 threads x 8 elements, or 256 x 16
};

// Constant tables for one context (all in device memory).
struct Tables {
  DevBuf mods;     // ModInfo[nmod]
  DevBuf tw;       // per modulus: fwd[N][2] (w, shoup), inv[N][2] (w, shoup)
  DevBuf twf;      // per modulus (as double): fwd[N][2] (w, w / q), inv[N][2] (w, w / q)
  DevBuf modup;    // per (nl, digit): see modup_offset
  DevBuf moddown;  // phat_inv[K][2], phat_mod_q[K][nq][2], pinv_mod_q[nq][2], p_mod_q[nq], N^-1 phat_inv[K][2]
  DevBuf moddown_f;  // doubles [K][nq][4]: c0 = phat mod q_i, c0 / q_i, c1 = c0 2^30 mod q_i, c1 / q_i
  DevBuf rescale;  // ql_inv[l][i][2] = (q_l^-1 mod q_i, shoup), l < nq, i < l
  DevBuf mask;     // NTT of the base mask on limbs 0..nq-2, Montgomery form: [nq-1][N]
  DevBuf mask_f;   // the same residues in [0, q) as the bits of doubles (FP64 products)
  std::vector<size_t> modup_offset;  // index nl (1..nq): offset (uint64 units) of the nl block
  std::vector<int64_t> base_mask;    // coefficient-domain base mask (host copy)
};

struct SwitchKey {
  DevBuf buf;  // [beta_top][2][nq+np][N], NTT domain; Q limbs as doubles' bits, P limbs in Montgomery form
};

}  // namespace fhe

namespace fhe {
// Device blocks of released matmul results, kept by size and handed to the next results of the same
// size (a release and a fresh allocation per result cost more host time than a small call's
// planning). At most `cap` bytes are kept; a context's pool dies with the context.
struct ResultPool {
  std::mutex mu;
  std::map<size_t, std::vector<DevBuf>> blocks;
  size_t bytes = 0, cap = 0;
  DevBuf take(size_t size);  // a kept block of exactly `size` bytes, or an empty buffer
  void put(DevBuf& b);       // keeps b (moved from) if it fits under the cap, else leaves it
  void clear(size_t new_cap);
};
struct GraphEntry;  // a captured matmul launch stream (spmspm.cpp)
uint64_t next_handle_id();
// Stream created on first use (default priority), destroyed with its owner.
struct OwnedStream {
  hipStream_t s = nullptr;
  hipStream_t get();
  ~OwnedStream();
};
}  // namespace fhe

struct fhe_ctx {
  fhe::Params p;
  int device = 0;
  fhe::Allocator al;
  fhe::Tables t;
  std::unique_ptr<fhe::SwitchKey> relin;
  std::map<uint32_t, std::unique_ptr<fhe::SwitchKey>> rot;  // keyed by Galois element 5^r mod 2N
  std::recursive_mutex exec_mu;  // one matmul execution at a time per context (shared scratch); the
                                 // autotuner holds it across the matmuls it times
  fhe::DevBuf ws_cache;  // executor scratch, grown on demand
  fhe::DevBuf group_cache;  // grouped plans' resident products between direct calls, grown on demand
  std::shared_ptr<fhe::ResultPool> results = std::make_shared<fhe::ResultPool>();  // released result blocks
  fhe::OwnedStream capture_stream;  // stream the executor captures HIP graphs on
  std::vector<std::shared_ptr<fhe::GraphEntry>> graphs;  // captured matmuls, most recent last
};

struct fhe_sk {
  std::vector<int64_t> s;  // ternary secret, coefficient domain
  fhe::DevBuf s_ntt;       // [nq+np][N], NTT domain (normal form)
  uint64_t seed = 0;
};

struct fhe_ct {
  int ncomp = 2, nl = 0;
  double scale = 1.0;
  fhe::DevBuf data;  // [ncomp][nl][N], NTT domain
};

struct fhe_mat {
  uint64_t id = fhe::next_handle_id();  // unique per handle in the process (keys captured graphs)
  int kind = 0;  // 0 CSR operand, 1 CSC operand, 2 dense result
  int rows = 0, cols = 0;
  std::vector<int32_t> indptr, indices;  // public pattern (operands)
  int64_t nnz = 0;
  int nl = 0, nchunks = 0;
  double scale = 1.0;
  fhe::DevBuf data;  // [nchunks][2][nl][N], NTT domain
  std::weak_ptr<fhe::ResultPool> pool;  // results: where `data` goes back on release
  uint64_t* chunk(int c, uint32_t N) const { return data.u64() + (size_t)c * 2 * nl * N; }
  ~fhe_mat() {
    if (auto p = pool.lock()) p->put(data);
  }
};
