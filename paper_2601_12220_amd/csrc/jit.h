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

// The run-time built kernels for one set of bodies: the generic kernel with
// 64-bit and with 32-bit index decoding (for narrow descriptors) and the
// split-zeroing kernel.
struct JitKernels {
  hipFunction_t wide = nullptr;
  hipFunction_t narrow = nullptr;
  hipFunction_t zero = nullptr;
};

// The kernels for these bodies on the current device (compiled on the first
// call).  BES_OK or an error code of bes.h with `err` set (the compiler log
// on a build failure).
int jit_generic(bool f64, const std::vector<std::string> &exprs, JitKernels *k,
                std::string &err);

// launch_generic with the run-time built kernels.
hipError_t launch_generic_jit(const JitKernels &k, const GenEinsum *dev, const GenEinsum &host,
                              const GenPtrs &ptrs, hipStream_t stream);

}  // namespace bes
