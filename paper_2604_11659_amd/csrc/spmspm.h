// Sparse x sparse ciphertext matmul: planner (Algorithm 1) and batched executor (Algorithm 2).
#pragma once
#include "ckks.h"

namespace fhe {

// A distinct product (ca, cb, d): operand chunks and the alignment d = lb - la (B is rotated left by d
// when d > 0, A by -d when d < 0). Every matched pair with the same triple shares the product.
struct PlanProduct {
  int32_t ca, cb, d;
  int32_t job = 0;  // which matmul of a batch the operands belong to
};

// One matched pair after alignment: its product, the slot min_pos isolated by the mask, the result
// chunk and the left-rotation amount (mod S) that moves min_pos to the row-major target slot.
struct PlanPair {
  int32_t prod;
  int32_t min_pos;
  int32_t chunk;  // result chunk (for a merged batch plan: index into all jobs' result chunks)
  uint32_t rot;
};

struct Plan {
  std::vector<PlanProduct> prods;
  std::vector<PlanPair> pairs;
  int nres = 1;           // result chunks
  int64_t matched = 0;    // matched pairs traversed (up to the end of the range; all for a full range)
  // pairs grouped by product: pairs[by_prod[first[i] .. first[i+1])] belong to product i
  std::vector<size_t> first;
  std::vector<uint32_t> by_prod;
};

void index_plan(Plan& plan);

// Validates a CSR/CSC pattern (indptr non-decreasing from 0 to nnz, indices in range and strictly
// ascending per row/column).
void check_pattern(int32_t outer, int32_t inner, const int32_t* indptr, const int32_t* indices);

// Algorithm 1 over A (CSR) and B (CSC), keeping the pairs with traversal index in [begin, end).
// With nonzero_a / nonzero_b (flags over the stored entries of A and B in packing order), a matched
// pair whose two entries are both flagged zero is skipped and not counted in the traversal index (the
// naive sparse method of the paper's evaluation, on operands that store every entry).
Plan build_plan(const Params& p, const fhe_mat* A, const fhe_mat* B, int64_t begin, int64_t end,
                const uint8_t* nonzero_a = nullptr, const uint8_t* nonzero_b = nullptr);

// One matmul of a batch: operands, its plan, its result handle.
struct Job {
  const fhe_mat* A;
  const fhe_mat* B;
  Plan plan;
  fhe_mat* C;
  int64_t pair_lo = 0, pair_hi = INT64_MAX;  // the traversal range the plan was built for
};

// Executes one or many matmuls as a single stream of batched launches: the products and pairs of all
// jobs are merged, so small matmuls share launches and pairs with equal rotation keys sit together.
// Each job's C receives its dense result chunks (two levels below the top).
// grouped: the pairs of a job sharing (result chunk, target rotation) are summed after their masks
// and go through one second rescale and one target rotation (different ciphertext bits from the
// per-pair form, same decryption up to noise).
// graph: capture the launch stream in a HIP graph kept on the context (at most two, most recent
// kept) and replay it when the same operand handles, ranges, plan mode and NTT split come again;
// results are bit-identical to the eager launches. Only the result-chunk pointer table changes
// between replays (rewritten before each launch, outside the graph).
// tree (implies grouped): the groups' target rotations are shared digit by digit (level t rotates
// the partial sums of equal (chunk, digits above t) once by digit t).
// hoist: the alignment rotation steps share the ModUp of their input (keyswitch_hoisted).
void execute_jobs(fhe_ctx* ctx, std::vector<Job>& jobs, hipStream_t st, bool grouped = false, bool graph = false,
                  bool tree = false, bool hoist = false);

// Plan mode and memory limits of one execution.
struct ExecOpts {
  bool grouped = false, graph = false, tree = false, hoist = false;
  size_t ws_bytes = 0;     // executor scratch budget (0: FHE_WORKSPACE_MB, default a third of free HBM, <= 128 GiB)
  size_t group_bytes = 0;  // grouped plans: budget of the resident products (0: FHE_GROUP_MB, default 49152 MiB)
};

// Executor scratch layout for a budget: batch sizes (products per launch PB, pairs per tail launch BB)
// and the words the scratch takes, for a step with nprod products and npairs pairs.
struct WsPlan {
  size_t PB = 1, BB = 1, words = 0;
};
WsPlan ws_plan(const fhe_ctx* ctx, size_t budget_bytes, size_t nprod, size_t npairs);

// Device words a grouped execution of `plan` keeps beyond the executor scratch and the tail's second
// ping-pong buffers: every product resident (2 (nq - 1) N words each) plus, for the digit tree, one
// partial sum (2 (nq - 2) N words) per distinct (result chunk, higher rotation digits) of each level.
size_t grouped_resident_words(const Params& p, const Plan& plan, bool tree);

// A captured matmul launch stream and everything its kernels read that is not an operand or key.
struct GraphEntry {
  std::vector<uint64_t> key;
  hipGraphExec_t exec = nullptr;
  std::vector<std::unique_ptr<ArgPack>> packs;  // device pointer tables the kernels read
  DevBuf result_dev;                            // result-chunk pointers, rewritten per replay
  size_t nres = 0;
  DevBuf gbuf;                                  // grouped form: resident products
  const void* ws_base = nullptr;                // executor scratch the graph was captured on
  size_t ws_bytes = 0;
  int64_t n_ks = 0, n_rescale = 0;              // work per replay (profiler counters)
  ~GraphEntry();
};

// Resumable execution: prepare_result validates keys/operands and zeroes C; execute_slices runs the
// products [lo, hi) of several prepared jobs (and all their pairs) as one merged launch stream,
// accumulating into each job's C. Synchronises `st` before returning. Serialised per context.
struct Slice {
  Job* job;
  int32_t lo, hi;
};
void prepare_result(fhe_ctx* ctx, Job& J, hipStream_t st);
void execute_slices(fhe_ctx* ctx, std::vector<Slice>& slices, hipStream_t st, const ExecOpts& opts);

// Counts of key-switch work in the plan: [F, products, align KS, relin KS, target KS, result chunks].
void plan_counts(const Params& p, const Plan& plan, int64_t out[6]);

// Grouped form: [groups (distinct result chunk, target rotation), their target key switches, the
// target key switches of the digit tree].
void plan_group_counts(const Params& p, const Plan& plan, int64_t out[3]);

}  // namespace fhe
