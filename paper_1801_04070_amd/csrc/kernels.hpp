// Entry points of the HIP kernel layer, called by the C-ABI implementation.
#pragma once

#include <hip/hip_runtime.h>

struct gq_ctx;

// QBX orders with compiled center kernels (the per-center coefficient arrays live in registers).
#define GQ_PQ_LIST(X) X(4) X(6) X(8) X(10) X(12) X(16)

namespace gq {

bool pq_supported(int pq);

// One density: gather strengths, run the FMM stages (or direct QBX), write out[0..n_tgt).
hipError_t run_eval(gq_ctx *ctx, int kind, const double *d1, const double *d2, double *out,
                    bool direct);

}  // namespace gq
