// Sparse x sparse ciphertext matmul: planner (Algorithm 1) and batched executor (Algorithm 2).
#pragma once
#include "ckks.h"

namespace fhe {

// A distinct product (ca, cb, d): operand chunks and the alignment d = lb - la (B is rotated left by d
// when d > 0, A by -d when d < 0). Every matched pair with the same triple shares the product.
struct PlanProduct {
  int32_t ca, cb, d;
};

// One matched pair after alignment: its product, the slot min_pos isolated by the mask, the result
// chunk and the left-rotation amount (mod S) that moves min_pos to the row-major target slot.
struct PlanPair {
  int32_t prod;
  int32_t min_pos;
  int32_t chunk;
  uint32_t rot;
};

struct Plan {
  std::vector<PlanProduct> prods;
  std::vector<PlanPair> pairs;
  int nres = 1;           // result chunks
  int64_t matched = 0;    // matched pairs of the full traversal
};

// Validates a CSR/CSC pattern (indptr non-decreasing from 0 to nnz, indices in range and strictly
// ascending per row/column).
void check_pattern(int32_t outer, int32_t inner, const int32_t* indptr, const int32_t* indices);

// Algorithm 1 over A (CSR) and B (CSC), keeping the pairs with traversal index in [begin, end).
Plan build_plan(const Params& p, const fhe_mat* A, const fhe_mat* B, int64_t begin, int64_t end);

// Executes the plan; C receives the dense result chunks (two levels below the top).
void execute_plan(fhe_ctx* ctx, const fhe_mat* A, const fhe_mat* B, const Plan& plan, hipStream_t st, fhe_mat* C);

// Counts of key-switch work in the plan: [F, products, align KS, relin KS, target KS, result chunks].
void plan_counts(const Params& p, const Plan& plan, int64_t out[6]);

}  // namespace fhe
