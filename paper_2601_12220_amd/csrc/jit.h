// Run-time build of the generic template for plans with expression operands
// (BES_EXPR): the expression bodies are compiled with hipRTC into a copy of
// the generic device code (kernels/generic_body.inc), once per (device,
// dtype, bodies) and kept for the life of the process.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "desc.h"

namespace bes {

// The generic kernel and its split-zeroing kernel for these bodies on the
// current device (compiled on the first call).  BES_OK or an error code of
// bes.h with `err` set (the compiler log on a build failure).
int jit_generic(bool f64, const std::vector<std::string> &exprs, hipFunction_t *kernel,
                hipFunction_t *zero, std::string &err);

// launch_generic with the run-time built kernels.
hipError_t launch_generic_jit(hipFunction_t kernel, hipFunction_t zero, const GenEinsum *dev,
                              const GenEinsum &host, const GenPtrs &ptrs, hipStream_t stream);

}  // namespace bes
