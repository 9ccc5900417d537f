// Generic batched-einsum template and the persistent batched launch (gfx950).
//
// Evaluates Eq. (1) per member for any notation within the descriptor limits:
// each group of `lanes` work-items owns one output element; its lanes split
// the outer rows of the contracted index space, walk the innermost contracted
// index with a tight strided loop, and combine their partial sums with
// wavefront shuffles.  Functional operands (views, alpha*op(S0)+beta(+S1),
// tetrahedron Jacobians) are evaluated where they are read.
//
// The persistent kernel runs many batched einsums in one launch: every block
// pulls (einsum, slot, tile) work items off a device counter until the list
// is exhausted; the last block to finish resets the counters, so the launch
// can be captured once in a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "../../../include/bes.h"

namespace bes {

namespace {

template <typename T>
__device__ __forceinline__ T gen_op(int op, T v) {
  switch (op) {
    case BES_OP_SIN: return sin(v);
    case BES_OP_COS: return cos(v);
    case BES_OP_SQUARE: return v * v;
    default: return v;
  }
}

template <typename T>
__device__ __forceinline__ T gen_value(const GenLayout &L, const T *p0, const T *p1, int64_t q0,
                                       int64_t q1) {
  switch (L.kind) {
    case GEN_ARRAY: return p0[q0];
    case GEN_TET: return p0[q0] - p0[q1];
    case GEN_ELEMENTWISE: return (T)L.alpha * gen_op<T>(L.op, p0[q0]) + (T)L.beta;
    default: return (T)L.alpha * gen_op<T>(L.op, p0[q0]) + (T)L.beta + p1[q1];
  }
}

// One tile [first, first + count) of output elements of one slot.
template <typename T>
__device__ void gen_tile(const GenEinsum *__restrict__ G, const GenPtrs *__restrict__ P,
                         int slot, int64_t first, int64_t count) {
  const int lanes = G->lanes;
  const int sub = threadIdx.x & (lanes - 1);
  const int per_pass = blockDim.x / lanes;
  const int n_ops = G->n_ops, n_out = G->n_out, n_con = G->n_con;
  const int64_t con_size = G->con_size;
  const int64_t ext_last = n_con > 0 ? G->con_ext[n_con - 1] : 1;
  const int64_t rows = (n_con > 0 && con_size > 0) ? con_size / ext_last : (n_con == 0 ? 1 : 0);
  T *__restrict__ outp = (T *)P->out[slot];
  const int64_t end = first + count;
  for (int64_t base = first; base < end; base += per_pass) {
    const int64_t o = base + threadIdx.x / lanes;
    const bool active = o < end;
    int64_t oidx[BES_GEN_MAX_IDX];
    {
      int64_t rem = active ? o : first;
#pragma unroll
      for (int d = BES_GEN_MAX_IDX - 1; d >= 0; --d) {
        if (d < n_out) {
          oidx[d] = rem % G->out_ext[d];
          rem /= G->out_ext[d];
        } else {
          oidx[d] = 0;
        }
      }
    }
    T acc = 0;
    for (int q = G->slot_m0[slot]; q < G->slot_m1[slot]; ++q) {
      const int m = G->slot_members[q];
      const GenLayout *L[BES_GEN_MAX_OPS];
      const T *p0[BES_GEN_MAX_OPS];
      const T *p1[BES_GEN_MAX_OPS];
      int64_t b0[BES_GEN_MAX_OPS], b1[BES_GEN_MAX_OPS], i0[BES_GEN_MAX_OPS], i1[BES_GEN_MAX_OPS];
#pragma unroll
      for (int k = 0; k < BES_GEN_MAX_OPS; ++k) {
        if (k >= n_ops) break;
        L[k] = &G->lay[G->layout[m][k]];
        p0[k] = (const T *)P->src[m][k][0];
        p1[k] = (const T *)P->src[m][k][1];
        int64_t a0 = L[k]->off0, a1 = L[k]->off1;
        for (int d = 0; d < n_out; ++d) {
          a0 += oidx[d] * L[k]->so0[d];
          a1 += oidx[d] * L[k]->so1[d];
        }
        b0[k] = a0;
        b1[k] = a1;
        i0[k] = n_con > 0 ? L[k]->sc0[n_con - 1] : 0;
        i1[k] = n_con > 0 ? L[k]->sc1[n_con - 1] : 0;
      }
      for (int64_t row = sub; row < rows; row += lanes) {
        int64_t r0[BES_GEN_MAX_OPS], r1[BES_GEN_MAX_OPS];
#pragma unroll
        for (int k = 0; k < BES_GEN_MAX_OPS; ++k) {
          r0[k] = k < n_ops ? b0[k] : 0;
          r1[k] = k < n_ops ? b1[k] : 0;
        }
        int64_t rem = row;
        for (int d = n_con - 2; d >= 0; --d) {
          const int64_t c = rem % G->con_ext[d];
          rem /= G->con_ext[d];
#pragma unroll
          for (int k = 0; k < BES_GEN_MAX_OPS; ++k) {
            if (k >= n_ops) break;
            r0[k] += c * L[k]->sc0[d];
            r1[k] += c * L[k]->sc1[d];
          }
        }
        for (int64_t c = 0; c < ext_last; ++c) {
          T prod = gen_value<T>(*L[0], p0[0], p1[0], r0[0], r1[0]);
          r0[0] += i0[0];
          r1[0] += i1[0];
#pragma unroll
          for (int k = 1; k < BES_GEN_MAX_OPS; ++k) {
            if (k >= n_ops) break;
            prod *= gen_value<T>(*L[k], p0[k], p1[k], r0[k], r1[k]);
            r0[k] += i0[k];
            r1[k] += i1[k];
          }
          acc += prod;
        }
      }
    }
    for (int off = lanes >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (active && sub == 0) outp[o] = acc;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) generic_kernel(const GenEinsum *__restrict__ G,
                                                      const GenPtrs P, int64_t tiles_per_slot) {
  const int slot = (int)(blockIdx.x / tiles_per_slot);
  const int64_t t = blockIdx.x % tiles_per_slot;
  const int64_t first = t * G->tile;
  int64_t count = G->out_size - first;
  if (count > G->tile) count = G->tile;
  if (count <= 0) return;
  gen_tile<T>(G, &P, slot, first, count);
}

template <typename T>
__global__ void __launch_bounds__(256) persistent_kernel(const GenEinsum *__restrict__ table,
                                                         const GenPtrs *__restrict__ ptrs,
                                                         const GenItem *__restrict__ items,
                                                         int n_items, unsigned *counters) {
  __shared__ int item;
  for (;;) {
    if (threadIdx.x == 0) item = (int)atomicAdd(&counters[0], 1u);
    __syncthreads();
    const int it = item;
    __syncthreads();
    if (it >= n_items) break;
    const GenItem w = items[it];
    gen_tile<T>(&table[w.einsum], &ptrs[w.einsum], w.slot, w.first, w.count);
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

}  // namespace

hipError_t launch_generic(bool f64, const GenEinsum *dev, const GenEinsum &host,
                          const GenPtrs &ptrs, hipStream_t stream) {
  if (host.out_size <= 0 || host.n_slots <= 0) return hipSuccess;
  const int64_t tiles = (host.out_size + host.tile - 1) / host.tile;
  const int64_t blocks = tiles * host.n_slots;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  dim3 grid((unsigned)blocks), block(256);
  if (f64)
    hipLaunchKernelGGL(generic_kernel<double>, grid, block, 0, stream, dev, ptrs, tiles);
  else
    hipLaunchKernelGGL(generic_kernel<float>, grid, block, 0, stream, dev, ptrs, tiles);
  return hipGetLastError();
}

hipError_t launch_persistent(bool f64, const GenEinsum *table, const GenPtrs *ptrs,
                             const GenItem *items, int n_items, unsigned *counters, int grid,
                             hipStream_t stream) {
  if (n_items <= 0) return hipSuccess;
  if (grid < 1) grid = 1;
  if (f64)
    hipLaunchKernelGGL(persistent_kernel<double>, dim3(grid), dim3(256), 0, stream, table, ptrs,
                       items, n_items, counters);
  else
    hipLaunchKernelGGL(persistent_kernel<float>, dim3(grid), dim3(256), 0, stream, table, ptrs,
                       items, n_items, counters);
  return hipGetLastError();
}

}  // namespace bes
