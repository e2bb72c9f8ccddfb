// Errors, the device allocator hook and owning device buffers.
#include <mutex>

#include "common.h"

namespace fhe {

namespace {
std::mutex g_alloc_mu;
Allocator g_alloc;
}  // namespace

[[noreturn]] void fail(int code, const std::string& msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char* what, const char* file, int line) {
  if (e != hipSuccess) {
    fail(e == hipErrorOutOfMemory ? FHE_ENOMEM : FHE_EDEVICE,
         std::string(what) + " failed: " + hipGetErrorString(e) + " (" + file + ":" + std::to_string(line) + ")");
  }
}

Allocator current_allocator() {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  return g_alloc;
}

void set_allocator(fhe_alloc_fn a, fhe_free_fn f, void* user) {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc = Allocator{a, f, user};
}

DevBuf::DevBuf(size_t bytes, hipStream_t stream) : bytes_(bytes), stream_(stream), al_(current_allocator()) {
  if (bytes == 0) return;
  if (al_.alloc) {
    ptr_ = al_.alloc(bytes, (void*)stream, al_.user);
    if (!ptr_) fail(FHE_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  } else {
    hipError_t e = hipMalloc(&ptr_, bytes);
    if (e != hipSuccess) {
      ptr_ = nullptr;
      (void)hipGetLastError();
      fail(FHE_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    }
  }
}

DevBuf& DevBuf::operator=(DevBuf&& o) noexcept {
  if (this != &o) {
    reset();
    ptr_ = o.ptr_;
    bytes_ = o.bytes_;
    stream_ = o.stream_;
    al_ = o.al_;
    o.ptr_ = nullptr;
    o.bytes_ = 0;
  }
  return *this;
}

void DevBuf::reset() {
  if (ptr_) {
    if (al_.free_) al_.free_(ptr_, (void*)stream_, al_.user);
    else (void)hipFree(ptr_);
  }
  ptr_ = nullptr;
  bytes_ = 0;
}

}  // namespace fhe
