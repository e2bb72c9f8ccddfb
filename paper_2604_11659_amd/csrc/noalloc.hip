// Rotation of one ciphertext into a caller-owned output without any device allocation. The scratch
// it needs (the automorphism's copy of the input, the key-switch workspace and the launch argument
// words) is one static device array per GPU, resolved to a device address once per device when a
// context is created on it. Same kernels and the same sequence as the allocating rotation, so the
// results are identical.
#include <array>
#include <mutex>
#include <vector>

#include "ckks.h"
#include "kernels.h"

// Host code never uses this name as an address (on the host it is a stand-in symbol): it resolves
// the array's device address once per GPU and passes that pointer on.
static __device__ __align__(256) uint64_t scratch[FHE_NOALLOC_SCRATCH_BYTES / 8];

namespace fhe {

namespace {

constexpr size_t kScratchBytes = FHE_NOALLOC_SCRATCH_BYTES;
constexpr size_t kArgBytes = 4096;  // launch argument words at the start of the array
constexpr int kMaxDevices = 64;

std::mutex g_mu;
std::array<uint64_t*, kMaxDevices> g_scratch{};  // device address of `scratch` on each GPU

uint64_t* scratch_on(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  uint64_t* p = device >= 0 && device < kMaxDevices ? g_scratch[device] : nullptr;
  if (!p) fail(FHE_EINVAL, "no-alloc scratch not set up on device " + std::to_string(device));
  return p;
}

}  // namespace

void noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) fail(FHE_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return;
  int cur = -1;
  HIPCHECK(hipGetDevice(&cur));
  if (cur != device) fail(FHE_EINVAL, "no-alloc scratch set-up needs its device current");
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr)
    fail(FHE_EINVAL, std::string("device address of the no-alloc scratch array: ") + hipGetErrorString(e));
  g_scratch[device] = (uint64_t*)p;
}

size_t noalloc_rotate_bytes(const fhe_ctx* ctx, uint32_t nl) {
  return kArgBytes + ((size_t)2 * nl * ctx->p.N + keyswitch_ws_elems(ctx, 1, nl)) * 8;
}

void ct_rotate_noalloc(fhe_ctx* ctx, const uint64_t* src, uint32_t nl, int64_t r, uint64_t* dst, hipStream_t st) {
  const Params& p = ctx->p;
  const size_t N = p.N;
  const size_t need = noalloc_rotate_bytes(ctx, nl);
  if (need > kScratchBytes)
    fail(FHE_ENOMEM, "rotation at " + std::to_string(nl) + " limbs needs " + std::to_string(need) +
                         " bytes of scratch; the no-alloc entry point has " + std::to_string(kScratchBytes));
  // the digit steps of r (the rotation-key rule) and their keys, all checked before any work is queued
  int64_t rr = r % (int64_t)p.S;
  if (rr < 0) rr += p.S;
  std::array<uint32_t, 32> steps{};
  std::array<const SwitchKey*, 32> keys{};
  uint32_t ns = 0;
  const uint32_t b = (uint32_t)p.rot_bits, digit_mask = (1u << b) - 1;
  for (int t = 0; t < p.rot_digits; ++t) {
    const uint32_t rt = ((uint32_t)rr >> (b * t)) & digit_mask;
    if (rt) {
      steps[ns] = rt << (b * t);
      keys[ns] = rotation_key(ctx, steps[ns]);
      ++ns;
    }
  }
  uint64_t* base = scratch_on(ctx->device);
  if (ns == 0) {
    if (dst != src) HIPCHECK(hipMemcpyAsync(dst, src, (size_t)2 * nl * N * 8, hipMemcpyDeviceToDevice, st));
    HIPCHECK(hipStreamSynchronize(st));
    return;
  }
  // argument words, 8 per step: [0] input, [1] Galois element, [2] key, [3..4] addends, [5] output
  constexpr size_t kW = 8;
  static_assert(32 * kW * 8 <= kArgBytes, "argument words fit their region");
  uint64_t* args = base;
  uint64_t* tmp = base + kArgBytes / 8;  // tau(input), [2][nl][N]
  uint64_t* ws = tmp + (size_t)2 * nl * N;
  std::array<uint64_t, 32 * kW> words{};
  for (uint32_t i = 0; i < ns; ++i) {
    uint64_t* w = words.data() + i * kW;
    w[0] = (uint64_t)(uintptr_t)(i == 0 ? src : dst);
    w[1] = galois_of_step(p, steps[i]);
    w[2] = (uint64_t)(uintptr_t)keys[i]->buf.u64();
    w[3] = (uint64_t)(uintptr_t)tmp;  // component 0 of tau(input) is added to the switched component 0
    w[4] = 0;
    w[5] = (uint64_t)(uintptr_t)dst;
  }
  HIPCHECK(hipMemcpyAsync(args, words.data(), ns * kW * 8, hipMemcpyHostToDevice, st));
  for (uint32_t i = 0; i < ns; ++i) {
    uint64_t* w = args + i * kW;
    // step i reads the previous step's output (dst) as a whole into tmp before overwriting dst
    automorph(ctx, 1, 2, nl, (const uint64_t* const*)w, (const uint32_t*)(w + 1), tmp, st);
    keyswitch(ctx, 1, nl, tmp + (size_t)nl * N, 0, (const uint64_t* const*)(w + 2), (const uint64_t* const*)(w + 3),
              (uint64_t* const*)(w + 5), ws, st);
  }
  // `words` is host memory the queued copy reads: it must outlive the copy
  HIPCHECK(hipStreamSynchronize(st));
}

}  // namespace fhe
