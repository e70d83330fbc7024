// Entry points of the HIP kernel layer, called by the C-ABI implementation.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

struct gq_ctx;

// QBX orders with compiled center kernels (the per-center coefficient arrays live in registers).
#define GQ_PQ_LIST(X) X(4) X(6) X(8) X(10) X(12) X(16) X(20)

namespace gq {

bool pq_supported(int pq);

// The compiled QBX orders, ascending.
const std::vector<int> &compiled_pq();


// Maximum densities per launch (the batch dimension of every kernel's grid).
constexpr int kMaxDensBatch = 128;

// Copies the natural-log table of the direct-interaction kernels to the current device; called
// once per context, with its device current, before any evaluation.
hipError_t upload_log_table();

// Elementwise device log (fn 1) or reciprocal (fn 2) of n values on stream s.
hipError_t run_math(int fn, int64_t n, const double *x, double *out, hipStream_t s);

// nd densities (rows of d1/d2 with strides ld1/ld2): gather strengths, run the FMM stages (or
// direct QBX), write nd output rows of n_tgt values with stride ld_out. Kind 4 (S and D of the
// same densities, FMM only, 2 nd workspace slots) writes the S rows to out and the D rows to
// out2, both with stride ld_out.
hipError_t run_eval(gq_ctx *ctx, int kind, const double *d1, int64_t ld1, const double *d2,
                    int64_t ld2, double *out, int64_t ld_out, int nd, bool direct,
                    double *out2 = nullptr);

}  // namespace gq
