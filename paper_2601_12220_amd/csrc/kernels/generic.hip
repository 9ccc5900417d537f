// Generic batched-einsum template and the persistent batched launch (gfx950).
//
// The per-output evaluation (generic_body.inc) covers any batched einsum
// within the descriptor limits.
//
// The persistent kernel runs many batched einsums in one launch: every block
// pulls (einsum, slot, tile) work items off a device counter until the list
// is exhausted; the last block to finish resets the counters, so the launch
// can be captured once in a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"
#include "../../../include/bes.h"

namespace bes {

namespace {

// Expression operands are evaluated by the run-time build only (jit.cpp);
// the static kernels never see one.
template <typename T>
__device__ __forceinline__ T bes_expr(int, T, T) {
  return (T)0;
}

#include "generic_body.inc"

template <typename T, bool NARROW>
__global__ void __launch_bounds__(256) generic_kernel(const GenEinsum *__restrict__ G,
                                                      const GenPtrs P, int64_t tiles_per_slot) {
  generic_block<T, NARROW>(G, P, tiles_per_slot);
}

// Block row blockIdx.y is the einsum of the persistent table.
template <typename T>
__global__ void __launch_bounds__(256) zero_split_outputs(const GenEinsum *__restrict__ table,
                                                          const GenPtrs *__restrict__ ptrs) {
  zero_slots<T>(table[blockIdx.y], ptrs[blockIdx.y]);
}

template <typename T>
__global__ void __launch_bounds__(256) zero_split_one(const GenEinsum *__restrict__ G,
                                                      const GenPtrs P) {
  zero_slots<T>(*G, P);
}

// W: minimum waves per SIMD the register allocation must allow.  The FP32
// instantiations are held to 128 VGPRs (4 waves, one per resident block of
// the persistent grid): their loop waits on loads and gains from the waves
// more than it loses to a few spills outside it.  The FP64 ones would spill
// heavily and keep the compiler's choice.
template <typename T, bool NARROW, int W>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W)))
persistent_kernel(const GenEinsum *__restrict__ table, const GenPtrs *__restrict__ ptrs,
                  const GenItem *__restrict__ items, int n_items, unsigned *counters) {
  __shared__ int item;
  for (;;) {
    if (threadIdx.x == 0) item = (int)atomicAdd(&counters[0], 1u);
    __syncthreads();
    const int it = item;
    __syncthreads();
    if (it >= n_items) break;
    const GenItem w = items[it];
    gen_tile<T, NARROW>(&table[w.einsum], &ptrs[w.einsum], w.slot, w.first, w.count, w.chunk);
  }
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned done = atomicAdd(&counters[1], 1u);
    if (done == gridDim.x - 1) {
      atomicExch(&counters[0], 0u);
      atomicExch(&counters[1], 0u);
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) fill_zero(T *__restrict__ p, int64_t n) {
  for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < n;
       f += (int64_t)gridDim.x * blockDim.x)
    p[f] = (T)0;
}

}  // namespace

hipError_t launch_fill_zero(void *p, int64_t n, int elem_bytes, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
  if (elem_bytes == 8)
    hipLaunchKernelGGL(fill_zero<double>, dim3(g), dim3(256), 0, stream, (double *)p, n);
  else if (elem_bytes == 4)
    hipLaunchKernelGGL(fill_zero<float>, dim3(g), dim3(256), 0, stream, (float *)p, n);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_generic(bool f64, const GenEinsum *dev, const GenEinsum &host,
                          const GenPtrs &ptrs, hipStream_t stream) {
  if (host.out_size <= 0 || host.n_slots <= 0) return hipSuccess;
  const int64_t tiles = (host.out_size + host.tile - 1) / host.tile;
  const int64_t blocks = tiles * host.n_slots * (host.split > 1 ? host.split : 1);
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (host.split > 1) {
    const int64_t n = host.out_size * host.n_slots;
    const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    if (f64)
      hipLaunchKernelGGL(zero_split_one<double>, dim3(g), dim3(256), 0, stream, dev, ptrs);
    else
      hipLaunchKernelGGL(zero_split_one<float>, dim3(g), dim3(256), 0, stream, dev, ptrs);
  }
  dim3 grid((unsigned)blocks), block(256);
  if (f64 && host.narrow)
    hipLaunchKernelGGL((generic_kernel<double, true>), grid, block, 0, stream, dev, ptrs, tiles);
  else if (f64)
    hipLaunchKernelGGL((generic_kernel<double, false>), grid, block, 0, stream, dev, ptrs, tiles);
  else if (host.narrow)
    hipLaunchKernelGGL((generic_kernel<float, true>), grid, block, 0, stream, dev, ptrs, tiles);
  else
    hipLaunchKernelGGL((generic_kernel<float, false>), grid, block, 0, stream, dev, ptrs, tiles);
  return hipGetLastError();
}

hipError_t launch_persistent(bool f64, const GenEinsum *table, const GenPtrs *ptrs,
                             const GenItem *items, int n_items, unsigned *counters, int grid,
                             hipStream_t stream, int n_einsums, bool any_split, bool narrow) {
  if (n_items <= 0) return hipSuccess;
  if (grid < 1) grid = 1;
  if (any_split) {
    if (f64)
      hipLaunchKernelGGL(zero_split_outputs<double>, dim3(64, n_einsums), dim3(256), 0, stream,
                         table, ptrs);
    else
      hipLaunchKernelGGL(zero_split_outputs<float>, dim3(64, n_einsums), dim3(256), 0, stream,
                         table, ptrs);
  }
  if (f64 && narrow)
    hipLaunchKernelGGL((persistent_kernel<double, true, 1>), dim3(grid), dim3(256), 0, stream,
                       table, ptrs, items, n_items, counters);
  else if (f64)
    hipLaunchKernelGGL((persistent_kernel<double, false, 1>), dim3(grid), dim3(256), 0, stream,
                       table, ptrs, items, n_items, counters);
  else if (narrow)
    hipLaunchKernelGGL((persistent_kernel<float, true, 4>), dim3(grid), dim3(256), 0, stream,
                       table, ptrs, items, n_items, counters);
  else
    hipLaunchKernelGGL((persistent_kernel<float, false, 4>), dim3(grid), dim3(256), 0, stream,
                       table, ptrs, items, n_items, counters);
  return hipGetLastError();
}

}  // namespace bes
