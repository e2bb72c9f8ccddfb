// Planner and batched executor for the CSR x CSC ciphertext matmul.
//
// The planner walks Algorithm 1 (every row i of A against every column j of B, a two-pointer merge
// of A's column ids and B's row ids) and records, for each match, the operand chunks, the alignment
// rotation (only the operand holding the later slot is rotated, by the slot difference), the
// isolated slot min_pos and the target rotation of Algorithm 2. Matched pairs that share
// (chunk of A, chunk of B, alignment) share the aligned product EvalMult -> Relinearize -> Rescale
// bit for bit, so the executor computes each such product once.
//
// The executor runs the per-pair sequence for many pairs at a time: each step (automorphism, key
// switch, tensor, rescale, mask multiply, accumulation) is one batched launch over a group of
// ciphertexts, which is what keeps 256 CUs busy with N = 2^13..2^17 limbs.
#include "spmspm.h"

#include <algorithm>
#include <cstdlib>
#include <functional>
#include <unordered_map>

namespace fhe {

void check_pattern(int32_t outer, int32_t inner, const int32_t* indptr, const int32_t* indices) {
  if (outer < 0 || inner < 0) fail(FHE_EINVAL, "negative matrix dimension");
  if (!indptr) fail(FHE_EINVAL, "indptr is NULL");
  if (indptr[0] != 0) fail(FHE_EINVAL, "indptr[0] must be 0");
  for (int32_t r = 0; r < outer; ++r) {
    if (indptr[r + 1] < indptr[r]) fail(FHE_EINVAL, "indptr must be non-decreasing");
    for (int32_t k = indptr[r]; k < indptr[r + 1]; ++k) {
      if (!indices) fail(FHE_EINVAL, "indices is NULL");
      if (indices[k] < 0 || indices[k] >= inner) fail(FHE_EINVAL, "index out of range");
      if (k > indptr[r] && indices[k] <= indices[k - 1]) fail(FHE_EINVAL, "indices must be strictly ascending");
    }
  }
}

Plan build_plan(const Params& p, const fhe_mat* A, const fhe_mat* B, int64_t begin, int64_t end,
                const uint8_t* nonzero_a, const uint8_t* nonzero_b) {
  Plan plan;
  const int64_t S = p.S;
  const int m = A->rows, n = B->cols;
  plan.nres = (int)std::max<int64_t>(1, ((int64_t)m * n + S - 1) / S);
  std::unordered_map<uint64_t, int32_t> prod_id;
  int64_t idx = 0;
  // the traversal stops at the end of the range: pairs after it are not needed, and a prefix of a
  // large matmul would otherwise pay for the merge over every cell of C
  for (int i = 0; i < m && idx < end; ++i) {
    const int32_t a_end = A->indptr[i + 1];
    for (int j = 0; j < n && idx < end; ++j) {
      int32_t a_pos = A->indptr[i], b_pos = B->indptr[j];
      const int32_t b_end = B->indptr[j + 1];
      while (a_pos < a_end && b_pos < b_end) {
        const int32_t a_col = A->indices[a_pos], b_row = B->indices[b_pos];
        if (a_col == b_row) {
          if (nonzero_a && !nonzero_a[a_pos] && !nonzero_b[b_pos]) {  // both entries known zero: skipped
            ++a_pos;
            ++b_pos;
            continue;
          }
          if (idx >= begin && idx < end) {
            const int32_t ca = (int32_t)(a_pos / S), la = (int32_t)(a_pos % S);
            const int32_t cb = (int32_t)(b_pos / S), lb = (int32_t)(b_pos % S);
            const int32_t d = lb - la, mn = std::min(la, lb);
            const uint64_t key = ((uint64_t)ca << 42) | ((uint64_t)cb << 21) | (uint64_t)(d + S);
            auto it = prod_id.find(key);
            int32_t pid;
            if (it == prod_id.end()) {
              pid = (int32_t)plan.prods.size();
              prod_id.emplace(key, pid);
              plan.prods.push_back(PlanProduct{ca, cb, d});
            } else {
              pid = it->second;
            }
            const int64_t t = (int64_t)i * n + j;
            const int32_t cr = (int32_t)(t / S), lt = (int32_t)(t % S);
            const uint32_t rot = (uint32_t)(((int64_t)mn - lt) % S + S) % S;
            plan.pairs.push_back(PlanPair{pid, mn, cr, rot});
          }
          ++idx;
          ++a_pos;
          ++b_pos;
        } else if (a_col < b_row) {
          ++a_pos;
        } else {
          ++b_pos;
        }
      }
    }
  }
  plan.matched = idx;
  // Order the products by the ciphertext their alignment rotates and by its rotation digits, low
  // digit first: products whose rotations start with the same steps become neighbours, so a batch of
  // products computes each shared intermediate rotation once (the executor keys rotation states by
  // source and amount prefix). Bits are unaffected: every product still sees its own sequence.
  const uint32_t rb = (uint32_t)p.rot_bits, rm = (1u << rb) - 1;
  auto skey = [&](const PlanProduct& pr, int t) -> int64_t {
    const uint32_t a = (uint32_t)(pr.d > 0 ? pr.d : -pr.d);
    return (int64_t)((a >> (rb * t)) & rm);
  };
  std::vector<int32_t> order(plan.prods.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int32_t)i;
  std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    const PlanProduct &a = plan.prods[x], &b = plan.prods[y];
    const int ka = a.d > 0 ? 1 : (a.d < 0 ? 0 : 2), kb = b.d > 0 ? 1 : (b.d < 0 ? 0 : 2);
    if (ka != kb) return ka < kb;
    const int32_t ca = a.d > 0 ? a.cb : a.ca, cb = b.d > 0 ? b.cb : b.ca;
    if (ca != cb) return ca < cb;
    for (int t = 0; t < p.rot_digits; ++t) {
      const int64_t da = skey(a, t), db = skey(b, t);
      if (da != db) return da < db;
    }
    if (a.ca != b.ca) return a.ca < b.ca;
    return a.cb < b.cb;
  });
  std::vector<int32_t> rank(order.size());
  std::vector<PlanProduct> sorted(order.size());
  for (size_t r = 0; r < order.size(); ++r) {
    rank[order[r]] = (int32_t)r;
    sorted[r] = plan.prods[order[r]];
  }
  plan.prods.swap(sorted);
  for (auto& pa : plan.pairs) pa.prod = rank[pa.prod];
  return plan;
}

void plan_counts(const Params& p, const Plan& plan, int64_t out[6]) {
  int64_t align = 0, target = 0;
  for (const auto& pr : plan.prods) align += (int64_t)rotation_steps(p, pr.d > 0 ? pr.d : -pr.d).size();
  for (const auto& pa : plan.pairs) target += (int64_t)rotation_steps(p, pa.rot).size();
  out[0] = (int64_t)plan.pairs.size();
  out[1] = (int64_t)plan.prods.size();
  out[2] = align;
  out[3] = (int64_t)plan.prods.size();
  out[4] = target;
  out[5] = plan.nres;
}

void plan_group_counts(const Params& p, const Plan& plan, int64_t out[3]) {
  std::vector<uint64_t> keys;
  keys.reserve(plan.pairs.size());
  for (const auto& pa : plan.pairs) keys.push_back(((uint64_t)(uint32_t)pa.chunk << 32) | pa.rot);
  std::sort(keys.begin(), keys.end());
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  int64_t target = 0;
  for (uint64_t k : keys) target += (int64_t)rotation_steps(p, (uint32_t)k).size();
  out[0] = (int64_t)keys.size();
  out[1] = target;
  // digit tree: one key switch per distinct nonzero (chunk, digits from t up) with digit t nonzero
  const uint32_t rb = (uint32_t)p.rot_bits, rlow = (1u << rb) - 1;
  int64_t tree = 0;
  for (int t = 0; t < p.rot_digits; ++t) {
    std::vector<uint64_t> lk;
    for (uint64_t k : keys) {
      const uint32_t rest = (uint32_t)k >> (rb * t);
      if (rest & rlow) lk.push_back((k & ~0xffffffffull) | rest);
    }
    std::sort(lk.begin(), lk.end());
    tree += (int64_t)(std::unique(lk.begin(), lk.end()) - lk.begin());
  }
  out[2] = tree;
}

namespace {

struct Workspace {
  uint64_t *align = nullptr, *rtmp = nullptr, *tens = nullptr, *pfull = nullptr, *prod = nullptr;
  uint64_t *msk = nullptr, *cur = nullptr, *ksws = nullptr, *rsws = nullptr;
};

// Executor scratch budget: FHE_WORKSPACE_MB if set, else a third of the device memory free at the
// call plus the scratch the context already holds (which the call reuses), between 1 and 128 GiB.
// Larger batches put more items that share a rotation key into one launch (and fewer launches per
// matmul): at N = 2^16 a 128 GiB budget took 6 % off a step against the former fixed 24 GiB.
size_t workspace_budget_bytes(const fhe_ctx* ctx) {
  if (const char* e = getenv("FHE_WORKSPACE_MB")) {
    size_t mb = (size_t)atoll(e);
    if (mb < 64) mb = 64;
    return mb << 20;
  }
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = (size_t)72 << 30;
  const size_t avail = free_b + ctx->ws_cache.bytes();
  return std::min<size_t>((size_t)128 << 30, std::max<size_t>((size_t)1 << 30, avail / 3));
}

// One batched rotation step over `items`: src[b] -> out[b] rotated left by steps[b] (one key switch).
// gather: no automorphism pass; the key switch reads component 1 through the automorphism and its
// final combine reads component 0 through it, so out[b] must be disjoint from src[b].
// Otherwise both components go to scratch first, and out[b] may equal src[b].
void enqueue_rotation(fhe_ctx* ctx, ArgPack& ap, std::vector<std::function<void()>>& ops, uint32_t nl,
                      const std::vector<const uint64_t*>& src_in, const std::vector<uint32_t>& steps_in,
                      const std::vector<uint64_t*>& out_in, const Workspace& ws, hipStream_t st, bool gather) {
  const Params& p = ctx->p;
  const uint32_t N = p.N, B = (uint32_t)src_in.size();
  if (!B) return;
  // Items that use the same rotation key become neighbours in the launch (key-stationary): the
  // inner-product kernel visits item after item for each (limb, tile), so their key tiles are
  // fetched from HBM once and served from L2 / MALL for the neighbours. The items are independent.
  std::vector<uint32_t> ord(B);
  for (uint32_t b = 0; b < B; ++b) ord[b] = b;
  std::stable_sort(ord.begin(), ord.end(), [&](uint32_t x, uint32_t y) { return steps_in[x] < steps_in[y]; });
  std::vector<const uint64_t*> src(B);
  std::vector<uint32_t> steps(B);
  std::vector<uint64_t*> out(B);
  for (uint32_t b = 0; b < B; ++b) {
    src[b] = src_in[ord[b]];
    steps[b] = steps_in[ord[b]];
    out[b] = out_in[ord[b]];
  }
  std::vector<uint32_t> gal(B);
  std::vector<const uint64_t*> keys(B), add(2 * B), src1(B);
  for (uint32_t b = 0; b < B; ++b) {
    if (gather && out[b] == src[b]) fail(FHE_EINVAL, "rotation with a gathered addend cannot run in place");
    gal[b] = galois_of_step(p, steps[b]);
    keys[b] = rotation_key(ctx, steps[b])->buf.u64();
    add[2 * b] = gather ? src[b] : ws.rtmp + (size_t)b * 2 * nl * N;
    add[2 * b + 1] = nullptr;
    src1[b] = src[b] + (size_t)nl * N;
  }
  const size_t o_src = ap.push(src), o_s1 = ap.push(src1), o_g = ap.push(gal), o_k = ap.push(keys),
               o_a = ap.push(add), o_o = ap.push(out);
  if (gather) {
    // the key switch reads component 1 through the automorphism, the final combine component 0
    ops.push_back([=, &ap] {
      keyswitch(ctx, B, nl, nullptr, 0, ap.at<const uint64_t*>(o_k), ap.at<const uint64_t*>(o_a),
                ap.at<uint64_t*>(o_o), ws.ksws, st, ap.at<uint32_t>(o_g), ap.at<const uint64_t*>(o_s1));
    });
    return;
  }
  ops.push_back([=, &ap] {
    automorph(ctx, B, 2, nl, ap.at<const uint64_t*>(o_src), ap.at<uint32_t>(o_g), ws.rtmp, st);
    keyswitch(ctx, B, nl, ws.rtmp + (size_t)nl * N, (uint64_t)2 * nl * N, ap.at<const uint64_t*>(o_k),
              ap.at<const uint64_t*>(o_a), ap.at<uint64_t*>(o_o), ws.ksws, st);
  });
}

// Hoisted rotation step: src[b] -> out[b] rotated left by steps[b]; the items that rotate the same
// src share its ModUp (one per distinct src) and read its transformed digits through their
// automorphisms (keyswitch_hoisted). out[b] must be disjoint from every src.
void enqueue_rotation_hoisted(fhe_ctx* ctx, ArgPack& ap, std::vector<std::function<void()>>& ops, uint32_t nl,
                              const std::vector<const uint64_t*>& src_in, const std::vector<uint32_t>& steps_in,
                              const std::vector<uint64_t*>& out_in, const Workspace& ws, hipStream_t st) {
  const Params& p = ctx->p;
  const uint32_t N = p.N, B = (uint32_t)src_in.size();
  if (!B) return;
  std::vector<uint32_t> ord(B);
  for (uint32_t b = 0; b < B; ++b) ord[b] = b;
  std::stable_sort(ord.begin(), ord.end(), [&](uint32_t x, uint32_t y) { return steps_in[x] < steps_in[y]; });
  std::unordered_map<const uint64_t*, uint32_t> sid;
  std::vector<const uint64_t*> state_c1, in_ptrs(B), keys(B), add(2 * B);
  std::vector<uint32_t> state_of(B), gal(B);
  std::vector<uint64_t*> out(B);
  for (uint32_t b = 0; b < B; ++b) {
    const uint32_t o = ord[b];
    const uint64_t* src = src_in[o];
    auto it = sid.find(src);
    if (it == sid.end()) {
      it = sid.emplace(src, (uint32_t)state_c1.size()).first;
      state_c1.push_back(src + (size_t)nl * N);
    }
    state_of[b] = it->second;
    in_ptrs[b] = state_c1[it->second];
    gal[b] = galois_of_step(p, steps_in[o]);
    keys[b] = rotation_key(ctx, steps_in[o])->buf.u64();
    add[2 * b] = src;  // component 0, read through the automorphism by the final combine
    add[2 * b + 1] = nullptr;
    out[b] = out_in[o];
  }
  for (uint64_t* q : out)
    if (sid.count(q)) fail(FHE_EINVAL, "hoisted rotation output overlaps an input");
  const uint32_t S = (uint32_t)state_c1.size();
  const std::vector<uint32_t> ident(S, 1u);
  const size_t o_c1 = ap.push(state_c1), o_id = ap.push(ident), o_so = ap.push(state_of), o_in = ap.push(in_ptrs),
               o_g = ap.push(gal), o_k = ap.push(keys), o_a = ap.push(add), o_o = ap.push(out);
  ops.push_back([=, &ap] {
    keyswitch_hoisted(ctx, S, B, nl, ap.at<const uint64_t*>(o_c1), ap.at<uint32_t>(o_id), ap.at<uint32_t>(o_so),
                      ap.at<const uint64_t*>(o_in), ap.at<uint32_t>(o_g), ap.at<const uint64_t*>(o_k),
                      ap.at<const uint64_t*>(o_a), ap.at<uint64_t*>(o_o), ws.ksws, st);
  });
}

}  // namespace

void index_plan(Plan& plan) {
  const size_t nprod = plan.prods.size();
  plan.first.assign(nprod + 1, 0);
  for (const auto& pa : plan.pairs) ++plan.first[pa.prod + 1];
  for (size_t i = 0; i < nprod; ++i) plan.first[i + 1] += plan.first[i];
  plan.by_prod.assign(plan.pairs.size(), 0);
  std::vector<size_t> fill(plan.first.begin(), plan.first.end() - 1);
  for (size_t k = 0; k < plan.pairs.size(); ++k) plan.by_prod[fill[plan.pairs[k].prod]++] = (uint32_t)k;
}

void prepare_result(fhe_ctx* ctx, Job& J, hipStream_t st) {
  const Params& p = ctx->p;
  const uint32_t N = p.N, nl2 = p.nq - 2;
  const size_t chunk_elems = (size_t)2 * nl2 * N;
  if (J.plan.first.size() != J.plan.prods.size() + 1) index_plan(J.plan);
  for (const auto& pr : J.plan.prods)
    if (pr.ca >= J.A->nchunks || pr.cb >= J.B->nchunks) fail(FHE_EINVAL, "plan references a missing operand chunk");
  if (!J.plan.pairs.empty() && !ctx->relin) fail(FHE_EKEY, "relinearisation key not generated");
  for (const auto& pa : J.plan.pairs)
    for (uint32_t s : rotation_steps(p, pa.rot)) (void)rotation_key(ctx, s);
  for (const auto& pr : J.plan.prods)
    for (uint32_t s : rotation_steps(p, pr.d > 0 ? pr.d : -pr.d)) (void)rotation_key(ctx, s);
  fhe_mat* C = J.C;
  C->kind = 2;
  C->rows = J.A->rows;
  C->cols = J.B->cols;
  C->nl = nl2;
  C->nchunks = J.plan.nres;
  C->scale = std::ldexp(1.0, p.d.log_delta + p.d.mask_bits);
  const size_t bytes = (size_t)J.plan.nres * chunk_elems * 8;
  C->data = ctx->results->take(bytes);  // a released result's block of the same size, if kept
  if (!C->data.get()) C->data = DevBuf(bytes, st);
  C->pool = ctx->results;
  HIPCHECK(hipMemsetAsync(C->data.get(), 0, bytes, st));
}

void execute_jobs(fhe_ctx* ctx, std::vector<Job>& jobs, hipStream_t st, bool grouped, bool graph, bool tree,
                  bool hoist) {
  std::vector<Slice> slices;
  for (auto& J : jobs) {
    prepare_result(ctx, J, st);
    slices.push_back(Slice{&J, 0, (int32_t)J.plan.prods.size()});
  }
  ExecOpts o;
  o.grouped = grouped;
  o.graph = graph;
  o.tree = tree;
  o.hoist = hoist;
  execute_slices(ctx, slices, st, o);
}

WsPlan ws_plan(const fhe_ctx* ctx, size_t budget, size_t nprod, size_t npairs) {
  const Params& p = ctx->p;
  const size_t N = p.N, nq = p.nq, nl1 = nq - 1, nl2 = nq - 2;
  const size_t e = 8ull * N;
  const size_t per_prod = e * (2 * nq + 3 * nq + 2 * nq + 2 * nl1 + 2 * nq) +
                          8 * (keyswitch_ws_elems(ctx, 1, (uint32_t)nq) + rescale_ws_elems(ctx, 1, 2, (uint32_t)nq));
  const size_t per_pair = e * (2 * nl1 + 2 * nl2 + 2 * nl2) +
                          8 * (keyswitch_ws_elems(ctx, 1, (uint32_t)nl2) + rescale_ws_elems(ctx, 1, 2, (uint32_t)nl1));
  WsPlan w;
  w.PB = std::max<size_t>(1, std::min<size_t>(nprod, (budget / 3) / per_prod));
  w.BB = std::max<size_t>(1, std::min<size_t>(npairs, (2 * budget / 3) / per_pair));
  w.PB = std::min<size_t>(w.PB, 4096);
  w.BB = std::min<size_t>(w.BB, 8192);
  const size_t PB = w.PB, BB = w.BB;
  const size_t rt = std::max<size_t>(PB * 2 * nq, BB * 2 * nl2) * N;
  const size_t sz_ks = std::max(keyswitch_ws_elems(ctx, (uint32_t)PB, (uint32_t)nq),
                                keyswitch_ws_elems(ctx, (uint32_t)BB, (uint32_t)nl2));
  const size_t sz_rs = std::max(rescale_ws_elems(ctx, (uint32_t)PB, 2, (uint32_t)nq),
                                rescale_ws_elems(ctx, (uint32_t)BB, 2, (uint32_t)nl1));
  w.words = PB * 2 * nq * N + rt + PB * 3 * nq * N + PB * 2 * nq * N + PB * 2 * nl1 * N + BB * 2 * nl1 * N +
            BB * 2 * nl2 * N + sz_ks + sz_rs;
  return w;
}

size_t grouped_resident_words(const Params& p, const Plan& plan, bool tree) {
  const size_t N = p.N, pe = 2 * (size_t)(p.nq - 1) * N, ce = 2 * (size_t)(p.nq - 2) * N;
  size_t nlev = 0;
  if (tree) {
    std::vector<uint64_t> keys;
    for (const auto& pa : plan.pairs) keys.push_back(((uint64_t)(uint32_t)pa.chunk << 32) | pa.rot);
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    const uint32_t rb = (uint32_t)p.rot_bits;
    for (int t = 1; t < p.rot_digits; ++t) {
      std::vector<uint64_t> lk;
      for (uint64_t k : keys) lk.push_back((k & ~0xffffffffull) | ((k & 0xffffffffull) >> (rb * t)));
      std::sort(lk.begin(), lk.end());
      nlev += (size_t)(std::unique(lk.begin(), lk.end()) - lk.begin());
    }
  }
  return plan.prods.size() * pe + nlev * ce;
}

GraphEntry::~GraphEntry() {
  if (exec) (void)hipGraphExecDestroy(exec);
}

namespace {

// A ciphertext entering the tail of the sequence: second rescale (with its one-hot mask fused in or
// applied first when `galois` is used), target rotation, accumulation into result chunk `chunk`.
struct TailItem {
  const uint64_t* src;
  uint32_t galois;
  int32_t chunk;
  uint32_t rot;
};

using Ops = std::vector<std::function<void()>>;

// Runs batches of launches: each batch's pointer tables are uploaded on `ls`, then its launches run
// at once (eager) or are kept for a graph capture (deferred).
struct Runner {
  hipStream_t ls;
  bool defer;
  std::vector<std::unique_ptr<ArgPack>>& packs;
  std::vector<Ops> pending;
  ArgPack& pack() {
    packs.emplace_back(new ArgPack());
    return *packs.back();
  }
  void submit(ArgPack& ap, Ops& ops) {
    ap.upload(ls);
    if (defer) {
      pending.push_back(std::move(ops));
    } else {
      for (auto& op : ops) op();
    }
  }
};

// EvalMult -> Relinearize -> Rescale of the products ids[k] (after their alignment rotations) into
// ws.prod slot k, [2][nq - 1][N] each.
void enqueue_products(fhe_ctx* ctx, ArgPack& ap, Ops& ops, const Plan& plan, const std::vector<const Job*>& job_of,
                      const int32_t* ids, size_t npb, const Workspace& ws, hipStream_t st, bool hoist,
                      uint64_t* const* dest = nullptr) {
  const Params& p = ctx->p;
  const uint32_t N = p.N, nq = p.nq, nl1 = nq - 1;
  // (1) Alignment rotations (Algorithm 1): rotate the operand whose value sits at the later slot, by
  // the slot difference, one key switch per nonzero rotation digit (low digit first). A rotation
  // state is (source ciphertext, amount applied so far); products of the batch that reach the same
  // state share its buffer, so each distinct intermediate rotation is computed once. States live in
  // 2 npb slots (the align buffers and the relinearised products' buffers, free until step (2)
  // writes them); a step's outputs take slots no live state holds, so no key switch writes a buffer
  // another one of the same launch reads.
  const uint32_t rbits = (uint32_t)p.rot_bits, rmask = (1u << rbits) - 1;
  std::vector<const uint64_t*> cur_src(npb), opa(npb), opb(npb), base(npb);
  std::vector<uint32_t> amt(npb, 0);
  std::vector<int32_t> slot_of(npb, -1);  // -1: the state is the source operand itself
  std::vector<int32_t> refs(2 * npb, 0);
  auto slot_ptr = [&](int32_t sl) -> uint64_t* {
    return sl < (int32_t)npb ? ws.align + (size_t)sl * 2 * nq * N : ws.pfull + (size_t)(sl - npb) * 2 * nq * N;
  };
  for (size_t k = 0; k < npb; ++k) {
    const PlanProduct& pr = plan.prods[ids[k]];
    opa[k] = job_of[pr.job]->A->chunk(pr.ca, N);
    opb[k] = job_of[pr.job]->B->chunk(pr.cb, N);
    cur_src[k] = base[k] = pr.d > 0 ? opb[k] : opa[k];
    amt[k] = pr.d == 0 ? 0u : (uint32_t)((pr.d > 0 ? pr.d : -pr.d) % (int32_t)p.S);
  }
  for (int t = 0; t < p.rot_digits; ++t) {
    std::vector<const uint64_t*> src;
    std::vector<uint32_t> st_amt;
    std::vector<uint64_t*> out;
    std::vector<char> taken(2 * npb, 0);
    std::unordered_map<uint64_t, int32_t> made;  // (source index, prefix) -> output slot of this step
    std::unordered_map<const uint64_t*, uint32_t> src_id;
    std::vector<int32_t> new_slot(npb, -2);
    int32_t next_free = 0;
    for (size_t k = 0; k < npb; ++k) {
      const uint32_t rt_ = (amt[k] >> (rbits * t)) & rmask;
      if (!rt_) continue;
      const uint32_t sid = src_id.emplace(base[k], (uint32_t)src_id.size()).first->second;
      const uint32_t prefix = amt[k] & (uint32_t)((rbits * (t + 1) >= 32) ? ~0u : ((1u << (rbits * (t + 1))) - 1));
      const uint64_t key = ((uint64_t)sid << 32) | prefix;
      auto it = made.find(key);
      if (it == made.end()) {
        while (next_free < (int32_t)(2 * npb) && (refs[next_free] > 0 || taken[next_free])) ++next_free;
        if (next_free >= (int32_t)(2 * npb)) fail(FHE_EINVAL, "internal: no free rotation-state slot");
        taken[next_free] = 1;
        it = made.emplace(key, next_free).first;
        src.push_back(cur_src[k]);
        st_amt.push_back(rt_ << (rbits * t));
        out.push_back(slot_ptr(next_free));
      }
      new_slot[k] = it->second;
    }
    if (hoist)
      enqueue_rotation_hoisted(ctx, ap, ops, nq, src, st_amt, out, ws, st);
    else
      enqueue_rotation(ctx, ap, ops, nq, src, st_amt, out, ws, st, true);
    for (size_t k = 0; k < npb; ++k) {
      if (new_slot[k] == -2) continue;
      if (slot_of[k] >= 0) --refs[slot_of[k]];
      slot_of[k] = new_slot[k];
      ++refs[slot_of[k]];
      cur_src[k] = slot_ptr(slot_of[k]);
    }
  }
  for (size_t k = 0; k < npb; ++k) {
    const PlanProduct& pr = plan.prods[ids[k]];
    if (pr.d > 0) opb[k] = cur_src[k];
    if (pr.d < 0) opa[k] = cur_src[k];
  }
  // (2) EvalMult + Relinearize + Rescale (Algorithm 2, first three steps), once per product.
  std::vector<const uint64_t*> keys(npb, ctx->relin->buf.u64()), add(2 * npb), pin(npb);
  std::vector<uint64_t*> pout(npb), rout(npb);
  for (size_t k = 0; k < npb; ++k) {
    add[2 * k] = ws.tens + k * 3 * nq * N;
    add[2 * k + 1] = ws.tens + k * 3 * nq * N + (size_t)nq * N;
    pout[k] = ws.pfull + k * 2 * nq * N;
    pin[k] = pout[k];
    rout[k] = dest ? dest[k] : ws.prod + k * 2 * nl1 * N;
  }
  const size_t o_a = ap.push(opa), o_b = ap.push(opb), o_k = ap.push(keys), o_ad = ap.push(add),
               o_po = ap.push(pout), o_pi = ap.push(pin), o_ro = ap.push(rout);
  const uint32_t Bn = (uint32_t)npb;
  ops.push_back([=, &ap] {
    tensor(ctx, Bn, nq, ap.at<const uint64_t*>(o_a), ap.at<const uint64_t*>(o_b), ws.tens, st);
    keyswitch(ctx, Bn, nq, ws.tens + (size_t)2 * nq * N, (uint64_t)3 * nq * N, ap.at<const uint64_t*>(o_k),
              ap.at<const uint64_t*>(o_ad), ap.at<uint64_t*>(o_po), ws.ksws, st);
    rescale(ctx, Bn, 2, nq, ap.at<const uint64_t*>(o_pi), ap.at<uint64_t*>(o_ro), ws.rsws, st);
  });
}

// The tail of Algorithm 2 for up to BB items at level top - 1 (sorted by result chunk, then
// rotation): (masked) rescale, target rotation, accumulation into the result chunks.
void enqueue_tail(fhe_ctx* ctx, ArgPack& ap, Ops& ops, const std::vector<TailItem>& items, bool masked,
                  const Workspace& ws, uint64_t* const* res, hipStream_t st, uint64_t* alt_base = nullptr) {
  const Params& p = ctx->p;
  const uint32_t N = p.N, nl1 = p.nq - 1, nl2 = p.nq - 2;
  const size_t nb = items.size();
  if (!nb) return;
  // Without a separate mask multiply the mask buffer is free: the target rotation steps alternate
  // between it (or alt_base, [nb][2][nl1][N], when the inputs live in the mask buffer) and cur,
  // starting where an even number of steps ends in cur.
  const bool pingpong = !masked || rescale_fuses_mask(ctx);
  const uint32_t rbits = p.rot_bits, rmask = (1u << rbits) - 1;
  std::vector<const uint64_t*> min_(nb), rin(nb);
  std::vector<uint32_t> mg(nb);
  std::vector<uint64_t*> mout(nb), cur(nb), alt(nb), where(nb);
  for (size_t k = 0; k < nb; ++k) {
    const TailItem& it = items[k];
    min_[k] = it.src;
    mg[k] = it.galois;
    mout[k] = ws.msk + k * 2 * nl1 * N;
    rin[k] = mout[k];
    cur[k] = ws.cur + k * 2 * nl2 * N;
    alt[k] = (alt_base ? alt_base : ws.msk) + k * 2 * nl1 * N;
    int nz = 0;
    for (int t = 0; t < p.rot_digits; ++t) nz += ((it.rot >> (rbits * t)) & rmask) != 0;
    where[k] = (pingpong && (nz & 1)) ? alt[k] : cur[k];
  }
  const size_t o_mi = ap.push(min_), o_mg = ap.push(mg), o_mo = ap.push(mout), o_ri = ap.push(rin),
               o_cu = ap.push(pingpong ? where : cur);
  const uint32_t Bn = (uint32_t)nb;
  ops.push_back([=, &ap] {
    if (!masked) {
      rescale(ctx, Bn, 2, nl1, ap.at<const uint64_t*>(o_mi), ap.at<uint64_t*>(o_cu), ws.rsws, st);
    } else if (rescale_fuses_mask(ctx)) {  // mask multiply applied inside the rescale's reads
      rescale(ctx, Bn, 2, nl1, ap.at<const uint64_t*>(o_mi), ap.at<uint64_t*>(o_cu), ws.rsws, st,
              ap.at<uint32_t>(o_mg));
    } else {
      mask_mul(ctx, Bn, nl1, ap.at<const uint64_t*>(o_mi), ap.at<uint32_t>(o_mg), ap.at<uint64_t*>(o_mo), st);
      rescale(ctx, Bn, 2, nl1, ap.at<const uint64_t*>(o_ri), ap.at<uint64_t*>(o_cu), ws.rsws, st);
    }
  });
  for (int t = 0; t < p.rot_digits; ++t) {
    std::vector<const uint64_t*> src;
    std::vector<uint32_t> st_amt;
    std::vector<uint64_t*> out;
    for (size_t k = 0; k < nb; ++k) {
      const uint32_t rt_ = (items[k].rot >> (rbits * t)) & rmask;
      if (!rt_) continue;
      uint64_t* dst = pingpong ? (where[k] == cur[k] ? alt[k] : cur[k]) : cur[k];
      src.push_back(where[k]);
      st_amt.push_back(rt_ << (rbits * t));
      out.push_back(dst);
      where[k] = dst;
    }
    enqueue_rotation(ctx, ap, ops, nl2, src, st_amt, out, ws, st, pingpong);
  }
  std::vector<uint32_t> seg;
  for (size_t k = 0; k < nb;) {
    const int32_t ch = items[k].chunk;
    size_t k2 = k;
    while (k2 < nb && items[k2].chunk == ch) ++k2;
    seg.push_back((uint32_t)ch);
    seg.push_back((uint32_t)k);
    seg.push_back((uint32_t)k2);
    k = k2;
  }
  const size_t o_sg = ap.push(seg);
  const uint32_t nseg = (uint32_t)(seg.size() / 3);
  const uint32_t ncontrib = (uint32_t)nb;
  ops.push_back([=, &ap] { accumulate(ctx, nseg, ncontrib, nl2, ap.at<uint32_t>(o_sg), ws.cur, res, st); });
}

size_t group_budget_bytes() {
  const char* e = getenv("FHE_GROUP_MB");
  long long mb = e ? atoll(e) : 49152;
  if (mb < 1) mb = 1;
  return (size_t)mb << 20;
}

// Grouped tail: the masked products of all pairs sharing (result chunk, target rotation) are summed
// (exact, mod q) into one ciphertext per group, which is rescaled, rotated and accumulated once.
// The products a pass of groups uses are computed first and kept resident (a product serves about
// ten pairs in different groups); each batch of groups then builds its sums with one k_mask_sum
// launch straight into the tail's input buffer. When all products do not fit the group budget, the
// groups run in passes, each recomputing the products its pairs use.
void execute_grouped(fhe_ctx* ctx, const Plan& plan, const std::vector<const Job*>& job_of, const Workspace& ws,
                     size_t PB, size_t BB, uint64_t* const* res, Runner& run, DevBuf& gbuf, bool tree, bool hoist,
                     size_t group_bytes) {
  const hipStream_t st = run.ls;
  const Params& p = ctx->p;
  const uint32_t N = p.N, nl1 = p.nq - 1;
  const size_t npairs = plan.pairs.size(), nprod = plan.prods.size();
  // groups ordered by (chunk, rotation): equal rotation keys sit together in the tail batches
  std::vector<uint64_t> keys(npairs);
  for (size_t k = 0; k < npairs; ++k) keys[k] = ((uint64_t)(uint32_t)plan.pairs[k].chunk << 32) | plan.pairs[k].rot;
  std::vector<uint64_t> gkeys(keys);
  std::sort(gkeys.begin(), gkeys.end());
  gkeys.erase(std::unique(gkeys.begin(), gkeys.end()), gkeys.end());
  const size_t ng = gkeys.size();
  std::vector<size_t> gfirst(ng + 1, 0);
  std::vector<uint32_t> gpair(npairs), pg(npairs);
  for (size_t k = 0; k < npairs; ++k) {
    pg[k] = (uint32_t)(std::lower_bound(gkeys.begin(), gkeys.end(), keys[k]) - gkeys.begin());
    ++gfirst[pg[k] + 1];
  }
  for (size_t g = 0; g < ng; ++g) gfirst[g + 1] += gfirst[g];
  {
    std::vector<size_t> fill(gfirst.begin(), gfirst.end() - 1);
    for (size_t k = 0; k < npairs; ++k) gpair[fill[pg[k]]++] = (uint32_t)k;
  }
  // resident products (at most PS) plus the tail's second ping-pong buffers
  const size_t pe = (size_t)2 * nl1 * N;
  const size_t budget = (group_bytes ? group_bytes : group_budget_bytes()) / 8;
  const size_t alt_elems = BB * pe;
  // store size: the budget, but never less than the largest group's distinct products
  size_t gmax = 1;
  {
    std::vector<char> seen(nprod, 0);
    for (size_t g = 0; g < ng; ++g) {
      size_t c = 0;
      for (size_t k = gfirst[g]; k < gfirst[g + 1]; ++k) {
        const int32_t pid = plan.pairs[gpair[k]].prod;
        if (!seen[pid]) {
          seen[pid] = 1;
          ++c;
        }
      }
      for (size_t k = gfirst[g]; k < gfirst[g + 1]; ++k) seen[plan.pairs[gpair[k]].prod] = 0;
      gmax = std::max(gmax, c);
    }
  }
  const size_t PS = std::min<size_t>(nprod, std::max<size_t>(gmax, budget / pe));
  // Digit tree: partial sums of level t = 1 .. D-1 keyed (chunk, rotation >> (b t)), sorted, so
  // that the keys of one level that feed the same key of the next are contiguous.
  const uint32_t rb = (uint32_t)p.rot_bits, rlow = (1u << rb) - 1;
  const size_t ce = (size_t)2 * (p.nq - 2) * N;  // a ciphertext two levels below the top
  std::vector<std::vector<uint64_t>> lkeys(tree ? (size_t)p.rot_digits : 0);
  std::vector<size_t> lbase(lkeys.size(), 0);
  size_t nlev = 0;
  for (size_t t = 1; t < lkeys.size(); ++t) {
    for (uint64_t gk : gkeys) lkeys[t].push_back((gk & ~0xffffffffull) | ((gk & 0xffffffffull) >> (rb * t)));
    std::sort(lkeys[t].begin(), lkeys[t].end());
    lkeys[t].erase(std::unique(lkeys[t].begin(), lkeys[t].end()), lkeys[t].end());
    lbase[t] = nlev;
    nlev += lkeys[t].size();
  }
  const size_t gwords = PS * pe + alt_elems + nlev * ce;
  if (gbuf.bytes() < gwords * 8) {
    gbuf.reset();
    gbuf = DevBuf(gwords * 8, st);
  }
  uint64_t* store = gbuf.u64();
  uint64_t* alt = store + PS * pe;
  uint64_t* lev = alt + alt_elems;
  auto lev_index = [&](size_t t, uint64_t key) -> size_t {
    return lbase[t] + (size_t)(std::lower_bound(lkeys[t].begin(), lkeys[t].end(), key) - lkeys[t].begin());
  };
  uint64_t* const* lev1_ptrs = nullptr;  // device table of the level-1 partial sums
  if (nlev) {
    std::vector<uint64_t*> ptrs(nlev);
    for (size_t i = 0; i < nlev; ++i) ptrs[i] = lev + i * ce;
    ArgPack& ap = run.pack();
    Ops ops;
    const size_t o_p = ap.push(ptrs);
    uint64_t* lz = lev;
    const uint64_t nz = (uint64_t)nlev * ce;
    ops.push_back([=] { fill_zero(ctx, nz, lz, st); });
    run.submit(ap, ops);
    lev1_ptrs = ap.at<uint64_t*>(o_p);
  }
  std::vector<int32_t> slot(nprod, -1);
  size_t g0 = 0;
  while (g0 < ng) {
    // the pass: groups [g0, g1) whose products fit in the store (at least one group)
    std::vector<int32_t> need;
    size_t g1 = g0;
    while (g1 < ng) {
      size_t add = 0;
      for (size_t k = gfirst[g1]; k < gfirst[g1 + 1]; ++k) {
        const int32_t pid = plan.pairs[gpair[k]].prod;
        if (slot[pid] == -1) {
          slot[pid] = -2;  // counted for this group
          ++add;
        }
      }
      for (size_t k = gfirst[g1]; k < gfirst[g1 + 1]; ++k) {
        const int32_t pid = plan.pairs[gpair[k]].prod;
        if (slot[pid] == -2) slot[pid] = -1;
      }
      if (g1 > g0 && need.size() + add > PS) break;
      for (size_t k = gfirst[g1]; k < gfirst[g1 + 1]; ++k) {
        const int32_t pid = plan.pairs[gpair[k]].prod;
        if (slot[pid] == -1) {
          slot[pid] = (int32_t)need.size();
          need.push_back(pid);
        }
      }
      ++g1;
    }
    // products of the pass, in product order (shared alignment prefixes sit together)
    std::vector<int32_t> order(need);
    std::sort(order.begin(), order.end());
    for (size_t b0 = 0; b0 < order.size(); b0 += PB) {
      const size_t npb = std::min(order.size(), b0 + PB) - b0;
      std::vector<uint64_t*> dest(npb);
      for (size_t k = 0; k < npb; ++k) dest[k] = store + (size_t)slot[order[b0 + k]] * pe;
      ArgPack& ap = run.pack();
      Ops ops;
      enqueue_products(ctx, ap, ops, plan, job_of, order.data() + b0, npb, ws, st, hoist, dest.data());
      run.submit(ap, ops);
    }
    // groups of the pass in tail batches: masked sums into the mask buffer, then the tail
    for (size_t t0 = g0; t0 < g1; t0 += BB) {
      const size_t t1 = std::min(g1, t0 + BB);
      std::vector<uint32_t> seg, gal;
      std::vector<const uint64_t*> in;
      std::vector<TailItem> items;
      for (size_t g = t0; g < t1; ++g) {
        const size_t e0 = in.size();
        for (size_t k = gfirst[g]; k < gfirst[g + 1]; ++k) {
          const PlanPair& pa = plan.pairs[gpair[k]];
          in.push_back(store + (size_t)slot[pa.prod] * pe);
          gal.push_back(mask_galois(p, pa.min_pos));
        }
        seg.push_back((uint32_t)(g - t0));
        seg.push_back((uint32_t)e0);
        seg.push_back((uint32_t)in.size());
        seg.push_back(1u);
        if (nlev) {  // level 0 of the tree: the low digit only, into the level-1 partial sum
          const uint64_t k1 = (gkeys[g] & ~0xffffffffull) | ((gkeys[g] & 0xffffffffull) >> rb);
          items.push_back(TailItem{ws.msk + (g - t0) * pe, 0u, (int32_t)lev_index(1, k1), (uint32_t)gkeys[g] & rlow});
        } else {
          items.push_back(TailItem{ws.msk + (g - t0) * pe, 0u, (int32_t)(gkeys[g] >> 32), (uint32_t)gkeys[g]});
        }
      }
      ArgPack& ap = run.pack();
      Ops ops;
      const size_t o_sg = ap.push(seg), o_in = ap.push(in), o_ga = ap.push(gal);
      const uint32_t nseg = (uint32_t)(seg.size() / 4), nent = (uint32_t)in.size();
      uint64_t* msk = ws.msk;
      ops.push_back([=, &ap] {
        mask_sum(ctx, nseg, nent, nl1, ap.at<uint32_t>(o_sg), ap.at<const uint64_t*>(o_in), ap.at<uint32_t>(o_ga), msk,
                 st);
      });
      enqueue_tail(ctx, ap, ops, items, false, ws, nlev ? lev1_ptrs : res, st, alt);
      run.submit(ap, ops);
    }
    for (int32_t pid : need) slot[pid] = -1;
    g0 = g1;
  }
  // Levels 1 .. D-1 of the tree: rotate each partial sum by its digit t (one key switch, none for a
  // zero digit) and add it into the partial sum of the next level (the result chunk after the last).
  for (size_t t = 1; t < lkeys.size(); ++t) {
    const bool last = t + 1 == lkeys.size();
    std::vector<uint64_t*> next_ptrs;
    if (!last) {
      next_ptrs.resize(lkeys[t + 1].size());
      for (size_t i = 0; i < next_ptrs.size(); ++i) next_ptrs[i] = lev + (lbase[t + 1] + i) * ce;
    }
    const std::vector<uint64_t>& K = lkeys[t];
    for (size_t t0 = 0; t0 < K.size(); t0 += BB) {
      const size_t t1 = std::min(K.size(), t0 + BB);
      std::vector<const uint64_t*> src, contrib;
      std::vector<uint32_t> steps, seg;
      std::vector<uint64_t*> out;
      int64_t cur_target = -1;
      for (size_t i = t0; i < t1; ++i) {
        const uint32_t rest = (uint32_t)(K[i] & 0xffffffffull), digit = rest & rlow;
        const uint64_t* acc = lev + (lbase[t] + i) * ce;
        if (digit) {
          uint64_t* o = ws.cur + (i - t0) * ce;
          src.push_back(acc);
          steps.push_back(digit << (rb * t));
          out.push_back(o);
          contrib.push_back(o);
        } else {
          contrib.push_back(acc);
        }
        const uint64_t nk = (K[i] & ~0xffffffffull) | (rest >> rb);
        const int64_t target = last ? (int64_t)(K[i] >> 32) : (int64_t)(lev_index(t + 1, nk) - lbase[t + 1]);
        if (target != cur_target) {
          if (cur_target >= 0) seg.push_back((uint32_t)contrib.size() - 1);
          seg.push_back((uint32_t)target);
          seg.push_back((uint32_t)contrib.size() - 1);
          cur_target = target;
        }
      }
      seg.push_back((uint32_t)contrib.size());
      ArgPack& ap = run.pack();
      Ops ops;
      enqueue_rotation(ctx, ap, ops, p.nq - 2, src, steps, out, ws, st, true);
      const size_t o_c = ap.push(contrib), o_s = ap.push(seg);
      const size_t o_n = last ? 0 : ap.push(next_ptrs);
      const uint32_t nseg = (uint32_t)(seg.size() / 3), ncon = (uint32_t)contrib.size();
      ops.push_back([=, &ap] {
        accumulate_ptr(ctx, nseg, ncon, p.nq - 2, ap.at<uint32_t>(o_s), ap.at<const uint64_t*>(o_c),
                       last ? res : ap.at<uint64_t*>(o_n), st);
      });
      run.submit(ap, ops);
    }
  }
}

void run_per_pair(fhe_ctx* ctx, const Plan& plan, const std::vector<const Job*>& job_of, const Workspace& ws,
                  size_t PB, size_t BB, uint64_t* const* res, Runner& run, bool hoist);

}  // namespace

void execute_slices(fhe_ctx* ctx, std::vector<Slice>& slices, hipStream_t st, const ExecOpts& opts) {
  const bool tree = opts.tree, grouped = opts.grouped || tree, graph = opts.graph, hoist = opts.hoist;
  const Params& p = ctx->p;
  const uint32_t N = p.N, nq = p.nq, nl1 = nq - 1, nl2 = nq - 2;
  std::lock_guard<std::recursive_mutex> exec_lock(ctx->exec_mu);
  // Merge the slices: products [lo, hi) of each job and their pairs, with result-chunk pointers.
  Plan plan;
  std::vector<uint64_t*> result_ptr;
  std::vector<const Job*> job_of;
  for (auto& sl : slices) {
    const Job& J = *sl.job;
    const int32_t jid = (int32_t)job_of.size();
    job_of.push_back(&J);
    const int32_t prod0 = (int32_t)plan.prods.size(), chunk0 = (int32_t)result_ptr.size();
    for (int c = 0; c < J.plan.nres; ++c) result_ptr.push_back(J.C->chunk(c, N));
    for (int32_t pi = sl.lo; pi < sl.hi; ++pi) {
      PlanProduct pr = J.plan.prods[pi];
      pr.job = jid;
      plan.prods.push_back(pr);
      for (size_t k = J.plan.first[pi]; k < J.plan.first[pi + 1]; ++k) {
        PlanPair pa = J.plan.pairs[J.plan.by_prod[k]];
        pa.prod = prod0 + (pi - sl.lo);
        pa.chunk += chunk0;
        plan.pairs.push_back(pa);
      }
    }
  }
  if (plan.pairs.empty()) {
    HIPCHECK(hipStreamSynchronize(st));
    return;
  }
  // A captured launch stream for these operands, ranges, plan mode and schedule, on this scratch.
  std::vector<uint64_t> key{(tree ? 2u : grouped ? 1u : 0u) | (hoist ? 4u : 0u), p.k1, p.rows_nt, slices.size()};
  for (auto& sl : slices)
    for (uint64_t v : {sl.job->A->id, sl.job->B->id, (uint64_t)sl.job->pair_lo, (uint64_t)sl.job->pair_hi,
                       (uint64_t)sl.lo, (uint64_t)sl.hi})
      key.push_back(v);
  if (graph) {
    for (auto& g : ctx->graphs) {
      if (g->key != key || g->ws_base != ctx->ws_cache.get() || g->ws_bytes != ctx->ws_cache.bytes() ||
          g->nres != result_ptr.size())
        continue;
      HIPCHECK(hipMemcpyAsync(g->result_dev.get(), result_ptr.data(), result_ptr.size() * 8, hipMemcpyHostToDevice,
                              st));
      const int tok = prof_begin("graph_replay", st);
      HIPCHECK(hipGraphLaunch(g->exec, st));
      prof_end(tok, st, 0.0);
      prof_count("keyswitch", g->n_ks);
      prof_count("rescale", g->n_rescale);
      HIPCHECK(hipStreamSynchronize(st));
      return;
    }
  }
  // Launch stream: the caller's, or the context's capture stream when recording a graph.
  const hipStream_t ls = graph ? ctx->capture_stream.get() : st;
  std::shared_ptr<GraphEntry> entry = graph ? std::make_shared<GraphEntry>() : nullptr;
  DevBuf result_local = upload(result_ptr, ls);
  index_plan(plan);
  const size_t nprod = plan.prods.size();

  // Batch sizes from the workspace budget.
  const WsPlan wp = ws_plan(ctx, opts.ws_bytes ? opts.ws_bytes : workspace_budget_bytes(ctx), nprod, plan.pairs.size());
  const size_t PB = wp.PB, BB = wp.BB;

  Workspace ws;
  const size_t rt = std::max<size_t>(PB * 2 * nq, BB * 2 * nl2) * N;
  const size_t sz_align = PB * 2 * nq * N, sz_tens = PB * 3 * nq * N, sz_pfull = PB * 2 * nq * N,
               sz_prod = PB * 2 * nl1 * N, sz_msk = BB * 2 * nl1 * N, sz_cur = BB * 2 * nl2 * N;
  const size_t sz_ks = std::max(keyswitch_ws_elems(ctx, (uint32_t)PB, nq), keyswitch_ws_elems(ctx, (uint32_t)BB, nl2));
  const size_t sz_rs =
      std::max(rescale_ws_elems(ctx, (uint32_t)PB, 2, nq), rescale_ws_elems(ctx, (uint32_t)BB, 2, nl1));
  const size_t total = sz_align + rt + sz_tens + sz_pfull + sz_prod + sz_msk + sz_cur + sz_ks + sz_rs;
  if (total != wp.words) fail(FHE_EINVAL, "internal: workspace layout differs from its plan");
  if (ctx->ws_cache.bytes() < total * 8) {  // grow-only scratch kept by the context between calls
    HIPCHECK(hipStreamSynchronize(st));      // earlier work on the old scratch has finished
    ctx->graphs.clear();                      // graphs captured on the old scratch are stale
    ctx->ws_cache.reset();
    ctx->ws_cache = DevBuf(total * 8, st);
  }
  uint64_t* w = ctx->ws_cache.u64();
  ws.align = w; w += sz_align;
  ws.rtmp = w; w += rt;
  ws.tens = w; w += sz_tens;
  ws.pfull = w; w += sz_pfull;
  ws.prod = w; w += sz_prod;
  ws.msk = w; w += sz_msk;
  ws.cur = w; w += sz_cur;
  ws.ksws = w; w += sz_ks;
  ws.rsws = w;

  uint64_t* const* res = (uint64_t* const*)result_local.get();
  std::vector<std::unique_ptr<ArgPack>> local_packs;
  // grouped form: resident products. A graph keeps its own; direct calls reuse the context's (a
  // fresh allocation and release per call cost more than a small call's work); a call with an
  // explicit group budget (the server's, which charges it per request) has its own, released after
  // the final synchronisation.
  DevBuf local_gbuf;
  Runner run{ls, graph, graph ? entry->packs : local_packs, {}};
  DevBuf& gbuf = graph ? entry->gbuf : opts.group_bytes ? local_gbuf : ctx->group_cache;
  if (grouped) {
    execute_grouped(ctx, plan, job_of, ws, PB, BB, res, run, gbuf, tree, hoist, opts.group_bytes);
  } else {
    run_per_pair(ctx, plan, job_of, ws, PB, BB, res, run, hoist);
  }
  if (!graph) {
    HIPCHECK(hipStreamSynchronize(st));
    return;
  }
  // Record the deferred launches as one graph, keep it on the context, launch it on the caller's
  // stream. The pointer tables were uploaded on the capture stream before recording.
  HIPCHECK(hipStreamSynchronize(ls));
  hipGraph_t g = nullptr;
  int64_t n_ks = 0, n_rs = 0;
  HIPCHECK(hipStreamBeginCapture(ls, hipStreamCaptureModeRelaxed));
  try {
    CaptureScope cs;
    for (auto& ops : run.pending)
      for (auto& op : ops) op();
    n_ks = cs.count("keyswitch");
    n_rs = cs.count("rescale");
  } catch (...) {
    hipGraph_t junk = nullptr;
    (void)hipStreamEndCapture(ls, &junk);
    if (junk) (void)hipGraphDestroy(junk);
    throw;
  }
  HIPCHECK(hipStreamEndCapture(ls, &g));
  hipGraphExec_t ex = nullptr;
  const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIPCHECK(ie);
  entry->exec = ex;
  entry->key = key;
  entry->result_dev = std::move(result_local);
  entry->nres = result_ptr.size();
  entry->ws_base = ctx->ws_cache.get();
  entry->ws_bytes = ctx->ws_cache.bytes();
  entry->n_ks = n_ks;
  entry->n_rescale = n_rs;
  if (ctx->graphs.size() >= 2) ctx->graphs.erase(ctx->graphs.begin());
  ctx->graphs.push_back(entry);
  const int tok = prof_begin("graph_replay", st);
  HIPCHECK(hipGraphLaunch(ex, st));
  prof_end(tok, st, 0.0);
  prof_count("keyswitch", n_ks);
  prof_count("rescale", n_rs);
  HIPCHECK(hipStreamSynchronize(st));
}

namespace {

void run_per_pair(fhe_ctx* ctx, const Plan& plan, const std::vector<const Job*>& job_of, const Workspace& ws,
                  size_t PB, size_t BB, uint64_t* const* res, Runner& run, bool hoist) {
  const Params& p = ctx->p;
  const uint32_t N = p.N, nl1 = p.nq - 1;
  const hipStream_t st = run.ls;
  const size_t nprod = plan.prods.size();
  const std::vector<size_t>& first = plan.first;
  const std::vector<uint32_t>& by_prod = plan.by_prod;
  std::vector<int32_t> ids(nprod);
  for (size_t i = 0; i < nprod; ++i) ids[i] = (int32_t)i;
  for (size_t p0 = 0; p0 < nprod; p0 += PB) {
    const size_t p1 = std::min(nprod, p0 + PB), npb = p1 - p0;
    ArgPack& ap = run.pack();
    Ops ops;
    enqueue_products(ctx, ap, ops, plan, job_of, ids.data() + p0, npb, ws, st, hoist);
    // (3) Pairs of these products: mask, rescale, target rotation, accumulate.
    std::vector<uint32_t> pairs(by_prod.begin() + first[p0], by_prod.begin() + first[p1]);
    std::stable_sort(pairs.begin(), pairs.end(), [&](uint32_t x, uint32_t y) {
      const PlanPair &a = plan.pairs[x], &b = plan.pairs[y];
      if (a.chunk != b.chunk) return a.chunk < b.chunk;
      return a.rot < b.rot;
    });
    for (size_t q0 = 0; q0 < pairs.size(); q0 += BB) {
      const size_t q1 = std::min(pairs.size(), q0 + BB);
      std::vector<TailItem> items;
      for (size_t k = q0; k < q1; ++k) {
        const PlanPair& pa = plan.pairs[pairs[k]];
        items.push_back(TailItem{ws.prod + (size_t)(pa.prod - p0) * 2 * nl1 * N, mask_galois(p, pa.min_pos), pa.chunk,
                                 pa.rot});
      }
      enqueue_tail(ctx, ap, ops, items, true, ws, res, st);
    }
    run.submit(ap, ops);
  }
}

}  // namespace

}  // namespace fhe
