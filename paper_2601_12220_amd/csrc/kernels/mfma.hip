// MFMA dense-contraction template (gfx950): placeholder until the tiled
// kernel lands; the planner does not select it yet.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace bes {

hipError_t launch_mfma(const MfmaArgs &, int, int, hipStream_t) { return hipErrorNotSupported; }

}  // namespace bes
