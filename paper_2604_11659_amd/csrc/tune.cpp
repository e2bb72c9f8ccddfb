// Autotuner for the schedule choices that leave every result bit unchanged.
//
// Two knobs change the schedule without changing a bit of the results. The NTT split: a limb is
// transformed as 2^k1 columns by 2^(logN - k1) rows, and k1 decides how the stages are grouped into
// LDS rounds, how wide the column segments are and which kernels (fused column kernels for k1 in
// [6, 8]) run. The row-phase workgroup shape: 512 threads with 8 elements each (3-stage rounds) or
// 256 threads with 16 (4-stage rounds, more registers per thread). The transform is the same for
// every choice, so the tuner may pick any of them. It times each candidate (a batch of synthetic
// key switches, or a prefix of the caller's own plan), keeps the fastest in the context and
// reports the timings.
#include <algorithm>
#include <random>

#include "ckks.h"
#include "kernels.h"
#include "spmspm.h"

using namespace fhe;

namespace {

// Median time of `reps` batched key switches of `B` synthetic polynomials at `nl` limbs.
double time_keyswitch(fhe_ctx* ctx, uint32_t B, uint32_t nl, const DevBuf& in, const ArgPack& ap, size_t o_key,
                      size_t o_add, size_t o_out, DevBuf& ws, int reps, hipStream_t st) {
  hipEvent_t a, b;
  HIPCHECK(hipEventCreate(&a));
  HIPCHECK(hipEventCreate(&b));
  const uint64_t stride = (uint64_t)nl * ctx->p.N;
  auto run = [&] {
    keyswitch(ctx, B, nl, in.u64(), stride, ap.at<const uint64_t*>(o_key), ap.at<const uint64_t*>(o_add),
              ap.at<uint64_t*>(o_out), ws.u64(), st);
  };
  run();  // warm-up (code objects, caches)
  std::vector<double> t;
  for (int r = 0; r < reps; ++r) {
    HIPCHECK(hipEventRecord(a, st));
    run();
    HIPCHECK(hipEventRecord(b, st));
    HIPCHECK(hipEventSynchronize(b));
    float ms = 0;
    HIPCHECK(hipEventElapsedTime(&ms, a, b));
    t.push_back(ms);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  std::sort(t.begin(), t.end());
  return t[t.size() / 2];
}

// Times every (k1 in [lo, hi], row shape) with `time_ms`, leaves the fastest in p and reports all.
// The current choice stays unless another is at least 2 % faster (about the timing noise).
template <class F>
void search(Params& p, int lo, int hi, std::vector<TuneTrial>& tried, TuneTrial& best, F&& time_ms) {
  const TuneTrial orig{(int)p.k1, (int)p.rows_nt, 0.0};
  tried.clear();
  best = orig;
  double orig_ms = 0, best_ms = 0;
  try {
    for (int nt : {512, 256}) {
      for (int k1 = lo; k1 <= hi; ++k1) {
        p.k1 = (uint32_t)k1;
        p.rows_nt = (uint32_t)nt;
        const double ms = time_ms();
        tried.push_back(TuneTrial{k1, nt, ms});
        if (k1 == orig.k1 && nt == orig.rows) orig_ms = ms;
        if (best_ms == 0 || ms < best_ms) {
          best_ms = ms;
          best = tried.back();
        }
      }
    }
  } catch (...) {
    p.k1 = (uint32_t)orig.k1;
    p.rows_nt = (uint32_t)orig.rows;
    throw;
  }
  if (orig_ms > 0 && best_ms > 0.98 * orig_ms) best = TuneTrial{orig.k1, orig.rows, orig_ms};
  p.k1 = (uint32_t)best.k1;
  p.rows_nt = (uint32_t)best.rows;
}

}  // namespace

void fhe::autotune_split(fhe_ctx* ctx, hipStream_t st, uint32_t B, std::vector<TuneTrial>& tried, TuneTrial& best) {
  if (B < 1 || B > 4096) fail(FHE_EINVAL, "autotune batch must be in [1, 4096]");
  if (!ctx->relin) fail(FHE_EKEY, "autotuning times key switches with the relinearisation key: run keygen first");
  std::lock_guard<std::recursive_mutex> lk(ctx->exec_mu);
  Params& p = ctx->p;
  const uint32_t N = p.N, nl = (uint32_t)p.nq;
  // synthetic input: residues in [0, q_i) on every limb (values do not matter for timing)
  std::vector<uint64_t> host((size_t)B * nl * N);
  std::mt19937_64 rng(12345);
  for (uint32_t b = 0; b < B; ++b)
    for (uint32_t i = 0; i < nl; ++i) {
      uint64_t* row = host.data() + ((size_t)b * nl + i) * N;
      for (uint32_t k = 0; k < N; ++k) row[k] = rng() % p.moduli[i];
    }
  DevBuf in = upload(host, st);
  DevBuf out((size_t)B * 2 * nl * N * 8, st);
  DevBuf ws(keyswitch_ws_elems(ctx, B, nl) * 8, st);
  ArgPack ap;
  std::vector<const uint64_t*> keys(B, ctx->relin->buf.u64());
  std::vector<uint64_t*> outs(B);
  for (uint32_t b = 0; b < B; ++b) outs[b] = out.u64() + (size_t)b * 2 * nl * N;
  const std::vector<const uint64_t*> adds(2 * (size_t)B, nullptr);  // no addend
  const size_t o_key = ap.push(keys), o_add = ap.push(adds), o_out = ap.push(outs);
  ap.upload(st);
  const int lo = std::max<int>(1, (int)p.logN - 9), hi = std::min<int>(9, (int)p.logN - 1);
  // the levels the matmul switches keys at: the top (alignment rotations, relinearisation) and two
  // below it (target rotations, the bulk); the same key serves both (lower levels index a prefix)
  const uint32_t nl_low = nl >= 3 ? nl - 2 : nl;
  search(p, lo, hi, tried, best, [&] {
    return time_keyswitch(ctx, B, nl, in, ap, o_key, o_add, o_out, ws, 5, st) +
           time_keyswitch(ctx, B, nl_low, in, ap, o_key, o_add, o_out, ws, 5, st);
  });
  HIPCHECK(hipStreamSynchronize(st));
}

void fhe::autotune_plan(fhe_ctx* ctx, hipStream_t st, const fhe_mat* A, const fhe_mat* B, int64_t pairs,
                        std::vector<TuneTrial>& tried, TuneTrial& best) {
  if (pairs < 1) fail(FHE_EINVAL, "autotune pair count must be positive");
  std::lock_guard<std::recursive_mutex> lk(ctx->exec_mu);
  Params& p = ctx->p;
  const int lo = std::max<int>(1, (int)p.logN - 9), hi = std::min<int>(9, (int)p.logN - 1);
  hipEvent_t a, b;
  HIPCHECK(hipEventCreate(&a));
  HIPCHECK(hipEventCreate(&b));
  // the first `pairs` matched pairs of the plan, each with its full sequence (alignment, product,
  // mask, rescales, target rotation, accumulation), timed as one matmul call
  auto run = [&]() -> double {
    fhe_mat C;
    std::vector<Job> jobs(1);
    jobs[0] = Job{A, B, build_plan(p, A, B, 0, pairs), &C};
    HIPCHECK(hipEventRecord(a, st));
    execute_jobs(ctx, jobs, st);
    HIPCHECK(hipEventRecord(b, st));
    HIPCHECK(hipEventSynchronize(b));
    float ms = 0;
    HIPCHECK(hipEventElapsedTime(&ms, a, b));
    return ms;
  };
  try {
    search(p, lo, hi, tried, best, [&] {
      run();  // warm-up
      std::vector<double> t{run(), run(), run()};
      std::sort(t.begin(), t.end());
      return t[1];
    });
  } catch (...) {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    throw;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
}
