// Errors, the device allocator hook and owning device buffers.
#include <atomic>
#include <map>
#include <mutex>
#include <tuple>

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

DevBuf ResultPool::take(size_t size) {
  std::lock_guard<std::mutex> lk(mu);
  auto it = blocks.find(size);
  if (it == blocks.end() || it->second.empty()) return DevBuf();
  DevBuf b = std::move(it->second.back());
  it->second.pop_back();
  bytes -= size;
  return b;
}

void ResultPool::put(DevBuf& b) {
  if (!b.get()) return;
  std::lock_guard<std::mutex> lk(mu);
  if (bytes + b.bytes() > cap) return;
  bytes += b.bytes();
  blocks[b.bytes()].push_back(std::move(b));
}

void ResultPool::clear(size_t new_cap) {
  std::map<size_t, std::vector<DevBuf>> old;
  {
    std::lock_guard<std::mutex> lk(mu);
    old.swap(blocks);
    bytes = 0;
    cap = new_cap;
  }
}  // the blocks are released here, outside the lock

void DevBuf::reset() {
  if (ptr_) {
    if (al_.free_) al_.free_(ptr_, (void*)stream_, al_.user);
    else (void)hipFree(ptr_);
  }
  ptr_ = nullptr;
  bytes_ = 0;
}

}  // namespace fhe

// ------------------------------------------------------------------------------------------------
// Per-kernel timing with HIP events (off by default). Each tracked launch is bracketed by two events
// recorded on the launch stream, so a query reports device time per kernel, not host time.
// ------------------------------------------------------------------------------------------------
namespace fhe {

namespace {
struct TimerRec {
  const char* name;
  hipEvent_t a, b;
  double bytes;
  double mulmods;
};
struct KernelTimer {
  std::mutex mu;
  bool on = false;
  std::vector<TimerRec> recs;
  std::vector<hipEvent_t> pool;
  std::map<std::string, int64_t> counts;  // work counters (no timing), e.g. key switches issued
};
KernelTimer& timer() {
  static KernelTimer* t = new KernelTimer();
  return *t;
}
hipEvent_t take_event(KernelTimer& t) {
  if (!t.pool.empty()) {
    hipEvent_t e = t.pool.back();
    t.pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIPCHECK(hipEventCreate(&e));
  return e;
}
}  // namespace

namespace {
thread_local int g_capturing = 0;
thread_local std::map<std::string, int64_t>* g_capture_counts = nullptr;
std::atomic<uint64_t> g_handle_id{1};
}  // namespace

CaptureScope::CaptureScope() {
  if (!g_capturing++) g_capture_counts = new std::map<std::string, int64_t>();
}
CaptureScope::~CaptureScope() {
  if (!--g_capturing) {
    delete g_capture_counts;
    g_capture_counts = nullptr;
  }
}
int64_t CaptureScope::count(const char* name) const {
  auto it = g_capture_counts->find(name);
  return it == g_capture_counts->end() ? 0 : it->second;
}

uint64_t next_handle_id() { return g_handle_id.fetch_add(1); }

hipStream_t OwnedStream::get() {
  if (!s) HIPCHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  return s;
}
OwnedStream::~OwnedStream() {
  if (s) (void)hipStreamDestroy(s);
}

int prof_begin(const char* name, hipStream_t st) {
  if (g_capturing) return -1;
  KernelTimer& t = timer();
  std::lock_guard<std::mutex> lk(t.mu);
  if (!t.on) return -1;
  TimerRec r{name, take_event(t), take_event(t), 0.0, 0.0};
  HIPCHECK(hipEventRecord(r.a, st));
  t.recs.push_back(r);
  return (int)t.recs.size() - 1;
}

void prof_end(int tok, hipStream_t st, double bytes, double mulmods) {
  if (tok < 0) return;
  KernelTimer& t = timer();
  std::lock_guard<std::mutex> lk(t.mu);
  if (tok >= (int)t.recs.size()) return;
  t.recs[tok].bytes = bytes;
  t.recs[tok].mulmods = mulmods;
  HIPCHECK(hipEventRecord(t.recs[tok].b, st));
}

void prof_count(const char* name, int64_t n) {
  if (g_capturing) {
    (*g_capture_counts)[name] += n;
    return;
  }
  KernelTimer& t = timer();
  std::lock_guard<std::mutex> lk(t.mu);
  if (t.on) t.counts[name] += n;
}

void prof_enable(bool on) {
  KernelTimer& t = timer();
  std::lock_guard<std::mutex> lk(t.mu);
  if (on) {  // a new measurement starts: recycle the events of the previous one
    for (auto& r : t.recs) {
      (void)hipEventSynchronize(r.b);
      t.pool.push_back(r.a);
      t.pool.push_back(r.b);
    }
    t.recs.clear();
    t.counts.clear();
  }
  t.on = on;
}

// Aggregates the records per kernel name (launches, total ms, algorithmic bytes, modular products).
std::vector<ProfRow> prof_summary() {
  KernelTimer& t = timer();
  std::lock_guard<std::mutex> lk(t.mu);
  std::map<std::string, ProfRow> agg;
  for (auto& r : t.recs) {
    HIPCHECK(hipEventSynchronize(r.b));
    float ms = 0.f;
    HIPCHECK(hipEventElapsedTime(&ms, r.a, r.b));
    ProfRow& x = agg[r.name];
    x.name = r.name;
    x.launches += 1;
    x.ms += ms;
    x.bytes += r.bytes;
    x.mulmods += r.mulmods;
  }
  std::vector<ProfRow> out;
  for (auto& kv : agg) out.push_back(kv.second);
  for (auto& kv : t.counts) {
    ProfRow x;
    x.name = "count:" + kv.first;
    x.launches = kv.second;
    out.push_back(x);
  }
  return out;
}

}  // namespace fhe
