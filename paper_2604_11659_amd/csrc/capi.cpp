// extern "C" entry points: argument checks, error translation, handle lifetimes.
#include <cmath>
#include <cstring>

#include "spmspm.h"

namespace fhe {
void set_allocator(fhe_alloc_fn a, fhe_free_fn f, void* user);
}

using namespace fhe;

namespace {

thread_local std::string g_err;

template <class F>
int guarded(F f) {
  try {
    g_err.clear();
    f();
    return FHE_OK;
  } catch (const Error& e) {
    g_err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return FHE_ENOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return FHE_EINVAL;
  }
}

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

}  // namespace

namespace fhe {
int set_error(int code, const char* msg) {
  g_err = msg;
  return code;
}
}  // namespace fhe

namespace {

void need(const void* p, const char* what) {
  if (!p) fail(FHE_EINVAL, std::string(what) + " is NULL");
}

void set_dev(const fhe_ctx* ctx) { HIPCHECK(hipSetDevice(ctx->device)); }

fhe_mat* encrypt_matrix(fhe_ctx* ctx, const fhe_sk* sk, int kind, int32_t rows, int32_t cols, const int32_t* indptr,
                        const int32_t* indices, const double* values, uint64_t seed, void* stream) {
  need(ctx, "ctx");
  need(sk, "sk");
  const int32_t outer = kind == 0 ? rows : cols, inner = kind == 0 ? cols : rows;
  check_pattern(outer, inner, indptr, indices);
  const int64_t nnz = indptr[outer];
  if (nnz > 0) need(values, "values");
  set_dev(ctx);
  std::unique_ptr<fhe_mat> m(new fhe_mat());
  m->kind = kind;
  m->rows = rows;
  m->cols = cols;
  m->nnz = nnz;
  m->indptr.assign(indptr, indptr + outer + 1);
  m->indices.assign(indices, indices + nnz);
  const double delta = kind == 0 ? std::ldexp(1.0, ctx->p.d.log_delta) : (double)ctx->p.moduli[ctx->p.nq - 1];
  encrypt_values(ctx, sk, values, nnz, delta, seed, as_stream(stream), m.get());
  return m.release();
}

void check_operands(const fhe_mat* A, const fhe_mat* B) {
  need(A, "A");
  need(B, "B");
  if (A->kind != 0 || B->kind != 1) fail(FHE_EINVAL, "A must be a CSR operand and B a CSC operand");
  if (A->cols != B->rows) fail(FHE_ESHAPE, "A.cols != B.rows");
}

}  // namespace

extern "C" {

int fhe_set_allocator(fhe_alloc_fn alloc, fhe_free_fn free_, void* user) {
  return guarded([&] {
    if ((alloc == nullptr) != (free_ == nullptr)) fail(FHE_EINVAL, "alloc and free must both be set or both NULL");
    set_allocator(alloc, free_, user);
  });
}

int fhe_params_create(const fhe_params_desc* desc, fhe_ctx** out) {
  return guarded([&] {
    need(desc, "desc");
    need(out, "out");
    *out = nullptr;
    std::unique_ptr<fhe_ctx> ctx(new fhe_ctx());
    ctx_init(ctx.get(), desc);
    *out = ctx.release();
  });
}

void fhe_ctx_free(fhe_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  delete ctx;
}

int fhe_ctx_primes(const fhe_ctx* ctx, uint64_t* out, size_t cap) {
  int n = 0;
  int rc = guarded([&] {
    need(ctx, "ctx");
    n = ctx->p.nmod();
    if (out) {
      if (cap < (size_t)n) fail(FHE_ESHAPE, "output buffer too small");
      memcpy(out, ctx->p.moduli.data(), (size_t)n * 8);
    }
  });
  return rc ? rc : n;
}

int fhe_keygen(fhe_ctx* ctx, uint64_t seed, void* stream, fhe_sk** sk_out) {
  return guarded([&] {
    need(ctx, "ctx");
    need(sk_out, "sk_out");
    *sk_out = nullptr;
    set_dev(ctx);
    std::unique_ptr<fhe_sk> sk(new fhe_sk());
    keygen(ctx, seed, as_stream(stream), sk.get());
    *sk_out = sk.release();
  });
}

void fhe_sk_free(fhe_sk* sk) { delete sk; }

int fhe_keygen_rotations(fhe_ctx* ctx, const fhe_sk* sk, const int32_t* amounts, size_t n, void* stream) {
  return guarded([&] {
    need(ctx, "ctx");
    need(sk, "sk");
    if (n) need(amounts, "amounts");
    set_dev(ctx);
    std::vector<uint32_t> steps;
    for (size_t i = 0; i < n; ++i)
      for (uint32_t s : rotation_steps(ctx->p, amounts[i])) steps.push_back(s);
    keygen_rotation_steps(ctx, sk, steps, as_stream(stream));
  });
}

int fhe_encrypt_csr(fhe_ctx* ctx, const fhe_sk* sk, int32_t rows, int32_t cols, const int32_t* indptr,
                    const int32_t* indices, const double* values, uint64_t seed, void* stream, fhe_mat** out) {
  return guarded([&] {
    need(out, "out");
    *out = nullptr;
    *out = encrypt_matrix(ctx, sk, 0, rows, cols, indptr, indices, values, seed, stream);
  });
}

int fhe_encrypt_csc(fhe_ctx* ctx, const fhe_sk* sk, int32_t rows, int32_t cols, const int32_t* indptr,
                    const int32_t* indices, const double* values, uint64_t seed, void* stream, fhe_mat** out) {
  return guarded([&] {
    need(out, "out");
    *out = nullptr;
    *out = encrypt_matrix(ctx, sk, 1, rows, cols, indptr, indices, values, seed, stream);
  });
}

int fhe_spmspm_pairs(fhe_ctx* ctx, const fhe_mat* A, const fhe_mat* B, int64_t pair_begin, int64_t pair_end,
                     void* stream, fhe_mat** C_out) {
  return guarded([&] {
    need(ctx, "ctx");
    need(C_out, "C_out");
    *C_out = nullptr;
    check_operands(A, B);
    if (pair_begin < 0 || pair_end < pair_begin) fail(FHE_EINVAL, "bad pair range");
    set_dev(ctx);
    std::unique_ptr<fhe_mat> C(new fhe_mat());
    std::vector<Job> jobs(1);
    jobs[0] = Job{A, B, build_plan(ctx->p, A, B, pair_begin, pair_end), C.get()};
    execute_jobs(ctx, jobs, as_stream(stream));
    *C_out = C.release();
  });
}

int fhe_spmspm_plan(fhe_ctx* ctx, size_t cnt, const fhe_mat* const* A, const fhe_mat* const* B,
                    const int64_t* pair_begin, const int64_t* pair_end, int32_t mode, void* stream, fhe_mat** C_out) {
  return guarded([&] {
    need(ctx, "ctx");
    need(C_out, "C_out");
    if (cnt) {
      need(A, "A");
      need(B, "B");
    }
    for (size_t i = 0; i < cnt; ++i) C_out[i] = nullptr;
    const int32_t plan_mode = mode & ~(FHE_PLAN_GRAPH | FHE_PLAN_HOIST);
    if (plan_mode != FHE_PLAN_PER_PAIR && plan_mode != FHE_PLAN_GROUPED && plan_mode != FHE_PLAN_TREE)
      fail(FHE_EINVAL, "unknown plan mode");
    if ((pair_begin == nullptr) != (pair_end == nullptr)) fail(FHE_EINVAL, "pair_begin and pair_end go together");
    for (size_t i = 0; i < cnt; ++i) {
      check_operands(A[i], B[i]);
      if (pair_begin && (pair_begin[i] < 0 || pair_end[i] < pair_begin[i])) fail(FHE_EINVAL, "bad pair range");
    }
    set_dev(ctx);
    std::vector<std::unique_ptr<fhe_mat>> Cs(cnt);
    std::vector<Job> jobs(cnt);
    for (size_t i = 0; i < cnt; ++i) {
      Cs[i].reset(new fhe_mat());
      const int64_t lo = pair_begin ? pair_begin[i] : 0, hi = pair_end ? pair_end[i] : INT64_MAX;
      jobs[i] = Job{A[i], B[i], build_plan(ctx->p, A[i], B[i], lo, hi), Cs[i].get(), lo, hi};
    }
    execute_jobs(ctx, jobs, as_stream(stream), plan_mode == FHE_PLAN_GROUPED, (mode & FHE_PLAN_GRAPH) != 0,
                 plan_mode == FHE_PLAN_TREE, (mode & FHE_PLAN_HOIST) != 0);
    for (size_t i = 0; i < cnt; ++i) C_out[i] = Cs[i].release();
  });
}

int fhe_spmspm_batch_pairs(fhe_ctx* ctx, size_t cnt, const fhe_mat* const* A, const fhe_mat* const* B,
                           const int64_t* pair_begin, const int64_t* pair_end, void* stream, fhe_mat** C_out) {
  return fhe_spmspm_plan(ctx, cnt, A, B, pair_begin, pair_end, FHE_PLAN_PER_PAIR, stream, C_out);
}

int fhe_spmspm_batch(fhe_ctx* ctx, size_t cnt, const fhe_mat* const* A, const fhe_mat* const* B, void* stream,
                     fhe_mat** C_out) {
  return fhe_spmspm_batch_pairs(ctx, cnt, A, B, nullptr, nullptr, stream, C_out);
}

int fhe_autotune(fhe_ctx* ctx, void* stream, const fhe_mat* A, const fhe_mat* B, int64_t pairs, int32_t batch,
                 int32_t* k1_out, int32_t* rows_out, double* ms_out, int32_t* n_tried, int32_t* k1_tried,
                 int32_t* rows_tried, double* ms_tried, int32_t cap) {
  return guarded([&] {
    need(ctx, "ctx");
    if (cap < 0 || (cap > 0 && (!k1_tried || !rows_tried || !ms_tried))) fail(FHE_EINVAL, "bad report arrays");
    if ((A == nullptr) != (B == nullptr)) fail(FHE_EINVAL, "A and B go together");
    set_dev(ctx);
    std::vector<TuneTrial> tried;
    TuneTrial best;
    if (A) {
      check_operands(A, B);
      autotune_plan(ctx, as_stream(stream), A, B, pairs, tried, best);
    } else {
      autotune_split(ctx, as_stream(stream), batch < 1 ? 0u : (uint32_t)batch, tried, best);
    }
    for (size_t i = 0; i < tried.size() && (int32_t)i < cap; ++i) {
      k1_tried[i] = tried[i].k1;
      rows_tried[i] = tried[i].rows;
      ms_tried[i] = tried[i].ms;
    }
    if (k1_out) *k1_out = best.k1;
    if (rows_out) *rows_out = best.rows;
    if (ms_out) *ms_out = best.ms;
    if (n_tried) *n_tried = (int32_t)tried.size();
  });
}

int fhe_spmspm(fhe_ctx* ctx, const fhe_mat* A, const fhe_mat* B, void* stream, fhe_mat** C_out) {
  return fhe_spmspm_pairs(ctx, A, B, 0, INT64_MAX, stream, C_out);
}

int fhe_plan_stats(fhe_ctx* ctx, const fhe_mat* A, const fhe_mat* B, int64_t counts[6]) {
  return guarded([&] {
    need(ctx, "ctx");
    need(counts, "counts");
    check_operands(A, B);
    Plan plan = build_plan(ctx->p, A, B, 0, INT64_MAX);
    plan_counts(ctx->p, plan, counts);
  });
}

int fhe_spmspm_naive_sparse(fhe_ctx* ctx, const fhe_mat* A, const fhe_mat* B, const uint8_t* nonzero_a,
                            const uint8_t* nonzero_b, void* stream, fhe_mat** C_out) {
  return guarded([&] {
    need(ctx, "ctx");
    need(C_out, "C_out");
    *C_out = nullptr;
    check_operands(A, B);
    if (A->nnz) need(nonzero_a, "nonzero_a");
    if (B->nnz) need(nonzero_b, "nonzero_b");
    set_dev(ctx);
    std::unique_ptr<fhe_mat> C(new fhe_mat());
    std::vector<Job> jobs(1);
    static const uint8_t none = 0;
    jobs[0] = Job{A, B, build_plan(ctx->p, A, B, 0, INT64_MAX, nonzero_a ? nonzero_a : &none,
                                   nonzero_b ? nonzero_b : &none),
                  C.get()};
    execute_jobs(ctx, jobs, as_stream(stream));
    *C_out = C.release();
  });
}

int fhe_plan_stats_naive_sparse(fhe_ctx* ctx, const fhe_mat* A, const fhe_mat* B, const uint8_t* nonzero_a,
                                const uint8_t* nonzero_b, int64_t counts[6]) {
  return guarded([&] {
    need(ctx, "ctx");
    need(counts, "counts");
    check_operands(A, B);
    if (A->nnz) need(nonzero_a, "nonzero_a");
    if (B->nnz) need(nonzero_b, "nonzero_b");
    static const uint8_t none = 0;
    Plan plan = build_plan(ctx->p, A, B, 0, INT64_MAX, nonzero_a ? nonzero_a : &none, nonzero_b ? nonzero_b : &none);
    plan_counts(ctx->p, plan, counts);
  });
}

int fhe_plan_groups(fhe_ctx* ctx, const fhe_mat* A, const fhe_mat* B, int64_t counts[3]) {
  return guarded([&] {
    need(ctx, "ctx");
    need(counts, "counts");
    check_operands(A, B);
    Plan plan = build_plan(ctx->p, A, B, 0, INT64_MAX);
    plan_group_counts(ctx->p, plan, counts);
  });
}

int fhe_plan_pattern(int32_t log_n, int32_t rot_digits, int32_t m, int32_t k, int32_t n, const int32_t* indptr_a,
                     const int32_t* indices_a, const int32_t* indptr_b, const int32_t* indices_b, int64_t counts[6]) {
  return guarded([&] {
    need(counts, "counts");
    if (log_n < 2 || log_n > 20 || rot_digits < 1 || rot_digits > log_n - 1) fail(FHE_EINVAL, "bad log_n / rot_digits");
    check_pattern(m, k, indptr_a, indices_a);
    check_pattern(n, k, indptr_b, indices_b);
    Params p;
    p.logN = (uint32_t)log_n;
    p.N = 1u << log_n;
    p.S = p.N / 2;
    p.rot_digits = rot_digits;
    p.rot_bits = (int)((p.logN - 1 + rot_digits - 1) / rot_digits);
    fhe_mat A, B;
    A.kind = 0;
    A.rows = m;
    A.cols = k;
    A.indptr.assign(indptr_a, indptr_a + m + 1);
    A.indices.assign(indices_a, indices_a + indptr_a[m]);
    B.kind = 1;
    B.rows = k;
    B.cols = n;
    B.indptr.assign(indptr_b, indptr_b + n + 1);
    B.indices.assign(indices_b, indices_b + indptr_b[n]);
    Plan plan = build_plan(p, &A, &B, 0, INT64_MAX);
    plan_counts(p, plan, counts);
  });
}

int fhe_plan_rotations(fhe_ctx* ctx, const fhe_mat* A, const fhe_mat* B, int32_t* out, size_t cap, size_t* n_out) {
  return guarded([&] {
    need(ctx, "ctx");
    need(n_out, "n_out");
    check_operands(A, B);
    Plan plan = build_plan(ctx->p, A, B, 0, INT64_MAX);
    std::vector<char> seen(ctx->p.S, 0);
    for (const auto& pr : plan.prods)
      for (uint32_t s : rotation_steps(ctx->p, pr.d > 0 ? pr.d : -pr.d)) seen[s] = 1;
    for (const auto& pa : plan.pairs)
      for (uint32_t s : rotation_steps(ctx->p, pa.rot)) seen[s] = 1;
    size_t n = 0;
    for (uint32_t s = 1; s < ctx->p.S; ++s)
      if (seen[s]) {
        if (out && n < cap) out[n] = (int32_t)s;
        ++n;
      }
    *n_out = n;
  });
}

int fhe_decrypt_decode(fhe_ctx* ctx, const fhe_sk* sk, const fhe_mat* M, void* stream, double* out, size_t cap) {
  return guarded([&] {
    need(ctx, "ctx");
    need(sk, "sk");
    need(M, "M");
    need(out, "out");
    const int64_t count = M->kind == 2 ? (int64_t)M->rows * M->cols : M->nnz;
    if (cap < (size_t)count) fail(FHE_ESHAPE, "output buffer too small");
    set_dev(ctx);
    const uint32_t S = ctx->p.S;
    std::vector<double> slots;
    for (int c = 0; c < M->nchunks; ++c) {
      const int64_t lo = (int64_t)c * S;
      if (lo >= count) break;
      decrypt_decode_chunk(ctx, sk, M->chunk(c, ctx->p.N), M->nl, M->scale, as_stream(stream), slots);
      const int64_t hi = std::min<int64_t>(count, lo + S);
      for (int64_t t = lo; t < hi; ++t) out[t] = slots[t - lo];
    }
  });
}

int fhe_mat_info(const fhe_mat* M, int32_t* kind, int32_t* rows, int32_t* cols, int32_t* chunks, int32_t* limbs,
                 double* scale) {
  return guarded([&] {
    need(M, "M");
    if (kind) *kind = M->kind;
    if (rows) *rows = M->rows;
    if (cols) *cols = M->cols;
    if (chunks) *chunks = M->nchunks;
    if (limbs) *limbs = M->nl;
    if (scale) *scale = M->scale;
  });
}

int fhe_mat_export(fhe_ctx* ctx, const fhe_mat* M, int32_t chunk, uint64_t* out, size_t cap, void* stream) {
  return guarded([&] {
    need(ctx, "ctx");
    need(M, "M");
    need(out, "out");
    if (chunk < 0 || chunk >= M->nchunks) fail(FHE_EINVAL, "chunk index out of range");
    const size_t n = (size_t)2 * M->nl * ctx->p.N;
    if (cap < n) fail(FHE_ESHAPE, "output buffer too small");
    set_dev(ctx);
    export_coeffs(ctx, M->chunk(chunk, ctx->p.N), 2, M->nl, as_stream(stream), out);
  });
}

void fhe_mat_free(fhe_mat* M) { delete M; }

int fhe_ct_import(fhe_ctx* ctx, const uint64_t* coeffs, int32_t ncomp, int32_t limbs, double scale, void* stream,
                  fhe_ct** out) {
  return guarded([&] {
    need(ctx, "ctx");
    need(coeffs, "coeffs");
    need(out, "out");
    *out = nullptr;
    if (ncomp < 2 || ncomp > 3) fail(FHE_EINVAL, "ncomp must be 2 or 3");
    if (limbs < 1 || limbs > ctx->p.nq) fail(FHE_EINVAL, "limbs out of range");
    const uint32_t N = ctx->p.N;
    const size_t n = (size_t)ncomp * limbs * N;
    for (int c = 0; c < ncomp; ++c)
      for (int i = 0; i < limbs; ++i)
        for (uint32_t k = 0; k < N; ++k)
          if (coeffs[((size_t)c * limbs + i) * N + k] >= ctx->p.moduli[i]) fail(FHE_EINVAL, "residue >= modulus");
    set_dev(ctx);
    hipStream_t st = as_stream(stream);
    std::unique_ptr<fhe_ct> ct(new fhe_ct());
    ct->ncomp = ncomp;
    ct->nl = limbs;
    ct->scale = scale;
    ct->data = DevBuf(n * 8, st);
    HIPCHECK(hipMemcpyAsync(ct->data.get(), coeffs, n * 8, hipMemcpyHostToDevice, st));
    ntt_forward(ctx, LimbBatch{ct->data.u64(), (uint32_t)limbs, (uint32_t)ncomp, (uint64_t)limbs * N, (uint32_t)limbs, 0},
                st);
    HIPCHECK(hipStreamSynchronize(st));
    *out = ct.release();
  });
}

int fhe_ct_export(fhe_ctx* ctx, const fhe_ct* ct, uint64_t* out, size_t cap, void* stream) {
  return guarded([&] {
    need(ctx, "ctx");
    need(ct, "ct");
    need(out, "out");
    const size_t n = (size_t)ct->ncomp * ct->nl * ctx->p.N;
    if (cap < n) fail(FHE_ESHAPE, "output buffer too small");
    set_dev(ctx);
    export_coeffs(ctx, ct->data.u64(), ct->ncomp, ct->nl, as_stream(stream), out);
  });
}

int fhe_ct_info(const fhe_ct* ct, int32_t* ncomp, int32_t* limbs, double* scale) {
  return guarded([&] {
    need(ct, "ct");
    if (ncomp) *ncomp = ct->ncomp;
    if (limbs) *limbs = ct->nl;
    if (scale) *scale = ct->scale;
  });
}

namespace {
fhe_ct* new_ct(const fhe_ctx* ctx, int ncomp, int nl, double scale, hipStream_t st) {
  fhe_ct* ct = new fhe_ct();
  ct->ncomp = ncomp;
  ct->nl = nl;
  ct->scale = scale;
  try {
    ct->data = DevBuf((size_t)ncomp * nl * ctx->p.N * 8, st);
  } catch (...) {
    delete ct;
    throw;
  }
  return ct;
}
void need2(const fhe_ct* ct) {
  if (ct->ncomp != 2) fail(FHE_ESHAPE, "expected a 2-component ciphertext");
}
}  // namespace

int fhe_ct_rotate(fhe_ctx* ctx, const fhe_ct* ct, int32_t r, void* stream, fhe_ct** out) {
  return guarded([&] {
    need(ctx, "ctx");
    need(ct, "ct");
    need(out, "out");
    *out = nullptr;
    need2(ct);
    set_dev(ctx);
    std::unique_ptr<fhe_ct> o(new_ct(ctx, 2, ct->nl, ct->scale, as_stream(stream)));
    ct_rotate(ctx, ct->data.u64(), ct->nl, r, o->data.u64(), as_stream(stream));
    *out = o.release();
  });
}

int fhe_ct_rotate_into(fhe_ctx* ctx, const fhe_ct* ct, int32_t r, fhe_ct* out, void* stream) {
  return guarded([&] {
    need(ctx, "ctx");
    need(ct, "ct");
    need(out, "out");
    need2(ct);
    need2(out);
    if (out->nl != ct->nl) fail(FHE_ESHAPE, "out has another limb count than ct");
    set_dev(ctx);
    ct_rotate_noalloc(ctx, ct->data.u64(), (uint32_t)ct->nl, r, out->data.u64(), as_stream(stream));
    out->scale = ct->scale;
  });
}

int fhe_ct_mult_relin(fhe_ctx* ctx, const fhe_ct* a, const fhe_ct* b, void* stream, fhe_ct** out) {
  return guarded([&] {
    need(ctx, "ctx");
    need(a, "a");
    need(b, "b");
    need(out, "out");
    *out = nullptr;
    need2(a);
    need2(b);
    if (a->nl != b->nl) fail(FHE_ESHAPE, "operands at different levels");
    set_dev(ctx);
    std::unique_ptr<fhe_ct> o(new_ct(ctx, 2, a->nl, a->scale * b->scale, as_stream(stream)));
    ct_mult_relin(ctx, a->data.u64(), b->data.u64(), a->nl, o->data.u64(), as_stream(stream));
    *out = o.release();
  });
}

int fhe_ct_rescale(fhe_ctx* ctx, const fhe_ct* ct, void* stream, fhe_ct** out) {
  return guarded([&] {
    need(ctx, "ctx");
    need(ct, "ct");
    need(out, "out");
    *out = nullptr;
    if (ct->nl < 2) fail(FHE_ELEVEL, "rescale needs at least two limbs");
    set_dev(ctx);
    const double ql = (double)ctx->p.moduli[ct->nl - 1];
    std::unique_ptr<fhe_ct> o(new_ct(ctx, ct->ncomp, ct->nl - 1, ct->scale / ql, as_stream(stream)));
    ct_rescale(ctx, ct->data.u64(), ct->ncomp, ct->nl, o->data.u64(), as_stream(stream));
    *out = o.release();
  });
}

int fhe_ct_mask(fhe_ctx* ctx, const fhe_ct* ct, int32_t slot, void* stream, fhe_ct** out) {
  return guarded([&] {
    need(ctx, "ctx");
    need(ct, "ct");
    need(out, "out");
    *out = nullptr;
    need2(ct);
    if (slot < 0 || (uint32_t)slot >= ctx->p.S) fail(FHE_EINVAL, "slot out of range");
    if (ct->nl > ctx->p.nq - 1) fail(FHE_ESHAPE, "mask multiply needs a ciphertext below the top level");
    set_dev(ctx);
    const double dm = std::ldexp((double)ctx->p.moduli[ctx->p.nq - 2], ctx->p.d.mask_bits);
    std::unique_ptr<fhe_ct> o(new_ct(ctx, 2, ct->nl, ct->scale * dm, as_stream(stream)));
    ct_mask(ctx, ct->data.u64(), ct->nl, slot, o->data.u64(), as_stream(stream));
    *out = o.release();
  });
}

int fhe_ct_add(fhe_ctx* ctx, const fhe_ct* a, const fhe_ct* b, void* stream, fhe_ct** out) {
  return guarded([&] {
    need(ctx, "ctx");
    need(a, "a");
    need(b, "b");
    need(out, "out");
    *out = nullptr;
    if (a->ncomp != b->ncomp || a->nl != b->nl) fail(FHE_ESHAPE, "operands of different shape");
    set_dev(ctx);
    std::unique_ptr<fhe_ct> o(new_ct(ctx, a->ncomp, a->nl, a->scale, as_stream(stream)));
    add_ct(ctx, a->ncomp, a->nl, a->data.u64(), b->data.u64(), o->data.u64(), as_stream(stream));
    HIPCHECK(hipStreamSynchronize(as_stream(stream)));
    *out = o.release();
  });
}

void fhe_ct_free(fhe_ct* ct) { delete ct; }

int fhe_profile_enable(int on) {
  return guarded([&] { prof_enable(on != 0); });
}

int fhe_profile_read(fhe_kernel_stat* out, size_t cap) {
  int n = 0;
  int rc = guarded([&] {
    auto rows = prof_summary();
    n = (int)rows.size();
    for (size_t i = 0; i < rows.size() && out && i < cap; ++i) {
      memset(&out[i], 0, sizeof(out[i]));
      strncpy(out[i].name, rows[i].name.c_str(), sizeof(out[i].name) - 1);
      out[i].launches = rows[i].launches;
      out[i].total_ms = rows[i].ms;
      out[i].bytes = rows[i].bytes;
      out[i].mulmods = rows[i].mulmods;
    }
  });
  return rc ? rc : n;
}

int fhe_bench_mulmod(int32_t device, int32_t kind, int32_t iters, void* stream, double* per_s) {
  return guarded([&] {
    need(per_s, "per_s");
    if (iters < 1) fail(FHE_EINVAL, "iters must be positive");
    HIPCHECK(hipSetDevice(device));
    *per_s = bench_mulmod(kind, (uint32_t)iters, as_stream(stream));
  });
}

const char* fhe_last_error(void) { return g_err.c_str(); }

}  // extern "C"
