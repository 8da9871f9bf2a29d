// Batched contraction of many independent lattices (batch.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "plan.hpp"
#include "tn.h"

namespace tn {

struct BatchImpl;

tn_status batch_workspace(const Plan* const* plans, int32_t n, int32_t prec, size_t* bytes,
                          std::string& err);
// threads: 256, 512 or 1024 per workgroup (one workgroup per lattice);
// split: the costliest `split` lattices advance in lock-step, every step
// spread over the GPU, beside the one-workgroup kernel for the rest.
tn_status batch_create(const Plan* const* plans, int32_t n, int32_t prec, int32_t threads,
                       void* ws, size_t ws_bytes, BatchImpl** out, std::string& err,
                       int32_t split = 0);
tn_status batch_run(BatchImpl* b, const double* const* const* sites, hipStream_t stream,
                    tn_result* outs, std::string& err);
void batch_destroy(BatchImpl* b);
int32_t batch_grid(const BatchImpl* b);

}  // namespace tn
