// Generic batched-einsum template and the persistent batched launch (gfx950).
//
// Evaluates Eq. (1) per member for any notation within the descriptor limits:
// each group of `lanes` work-items owns one output element; a contracted
// index carried by one operand only is summed inside that operand (a factored
// order of the same sum), the lanes split the space of the shared contracted
// indices, and their partial sums meet in wavefront shuffles.  Functional
// operands (views, alpha*op(S0)+beta(+S1), tetrahedron Jacobians) are
// evaluated where they are read.
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

// Sum of operand k's value over its exclusive contracted indices, the rest
// of the position fixed at (a0, a1): a plain loop, innermost index walked by
// stride.  Without exclusive indices it is the single value.
template <typename T>
__device__ __forceinline__ T ex_sum(const GenEinsum *__restrict__ G, const GenLayout &L,
                                    const T *p0, const T *p1, int k, int64_t a0, int64_t a1) {
  const int nd = G->ex_n[k];
  if (nd == 0) return gen_value<T>(L, p0, p1, a0, a1);
  if (G->ex_size[k] == 0) return (T)0;
  const int d0 = G->ex_off[k], dl = d0 + nd - 1;
  const int64_t inner = G->con_ext[dl];
  const int64_t outer = G->ex_size[k] / inner;
  const int64_t s0 = L.sc0[dl], s1 = L.sc1[dl];
  T sum = 0;
  for (int64_t orow = 0; orow < outer; ++orow) {
    int64_t q0 = a0, q1 = a1, rem = orow;
    for (int d = dl - 1; d >= d0; --d) {
      const int64_t c = rem % G->con_ext[d];
      rem /= G->con_ext[d];
      q0 += c * L.sc0[d];
      q1 += c * L.sc1[d];
    }
    for (int64_t c = 0; c < inner; ++c) {
      sum += gen_value<T>(L, p0, p1, q0, q1);
      q0 += s0;
      q1 += s1;
    }
  }
  return sum;
}

// One tile [first, first + count) of output elements of one slot.  Per
// output: the operands without shared contracted indices are summed over
// their exclusive indices once; the shared index space is split across the
// `lanes` work-items of the output, each row taking the product of the other
// operands' exclusive sums; the lanes' partial sums meet in wavefront
// shuffles.
template <typename T>
__device__ void gen_tile(const GenEinsum *__restrict__ G, const GenPtrs *__restrict__ P,
                         int slot, int64_t first, int64_t count, int chunk) {
  const int lanes = G->lanes;
  const int sub = threadIdx.x & (lanes - 1);
  const int per_pass = blockDim.x / lanes;
  const int n_ops = G->n_ops, n_out = G->n_out, n_sh = G->n_sh;
  const int64_t sh_size = G->sh_size;
  const int row_dep = G->row_dep;
  const int split = G->split;
  // rows [lo, hi) of the shared space belong to this chunk
  const int64_t lo = split > 1 ? sh_size * chunk / split : 0;
  const int64_t hi = split > 1 ? sh_size * (chunk + 1) / split : sh_size;
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
      int64_t b0[BES_GEN_MAX_OPS], b1[BES_GEN_MAX_OPS];
      T fac = 1;
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
        if (!((row_dep >> k) & 1)) fac *= ex_sum<T>(G, *L[k], p0[k], p1[k], k, a0, a1);
      }
      T part = 0;
      for (int64_t row = lo + sub; row < hi; row += lanes) {
        int64_t r0[BES_GEN_MAX_OPS], r1[BES_GEN_MAX_OPS];
#pragma unroll
        for (int k = 0; k < BES_GEN_MAX_OPS; ++k) {
          r0[k] = k < n_ops ? b0[k] : 0;
          r1[k] = k < n_ops ? b1[k] : 0;
        }
        int64_t rem = row;
        for (int d = n_sh - 1; d >= 0; --d) {
          const int64_t c = rem % G->con_ext[d];
          rem /= G->con_ext[d];
#pragma unroll
          for (int k = 0; k < BES_GEN_MAX_OPS; ++k) {
            if (k >= n_ops) break;
            r0[k] += c * L[k]->sc0[d];
            r1[k] += c * L[k]->sc1[d];
          }
        }
        T prod = 1;
#pragma unroll
        for (int k = 0; k < BES_GEN_MAX_OPS; ++k) {
          if (k >= n_ops) break;
          if ((row_dep >> k) & 1) prod *= ex_sum<T>(G, *L[k], p0[k], p1[k], k, r0[k], r1[k]);
        }
        part += prod;
      }
      acc += fac * part;
    }
    for (int off = lanes >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (active && sub == 0) {
      int64_t oa = o;
      if (!G->o_dense) {
        oa = G->o_off[slot];
        for (int d = 0; d < n_out; ++d) oa += oidx[d] * G->o_str[slot][d];
      }
      // chunks meet in the zeroed output; accumulating slots add into the
      // caller's values (atomically: several slots may address one buffer)
      if (split > 1 || G->o_acc[slot]) atomicAdd(&outp[oa], acc);
      else outp[oa] = acc;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) generic_kernel(const GenEinsum *__restrict__ G,
                                                      const GenPtrs P, int64_t tiles_per_slot) {
  // block = (slot, tile, chunk), chunk fastest
  const int split = G->split;
  const int chunk = (int)(blockIdx.x % split);
  const int64_t st = blockIdx.x / split;
  const int slot = (int)(st / tiles_per_slot);
  const int64_t t = st % tiles_per_slot;
  const int64_t first = t * G->tile;
  int64_t count = G->out_size - first;
  if (count > G->tile) count = G->tile;
  if (count <= 0) return;
  gen_tile<T>(G, &P, slot, first, count, chunk);
}

// Address of output element o (linear in the output's index order) of slot
// s under the slot's layout.
__device__ __forceinline__ int64_t gen_out_addr(const GenEinsum &G, int s, int64_t o) {
  if (G.o_dense) return o;
  int64_t a = G.o_off[s], rem = o;
  for (int d = G.n_out - 1; d >= 0; --d) {
    const int64_t c = rem % G.out_ext[d];
    rem /= G.out_ext[d];
    a += c * G.o_str[s][d];
  }
  return a;
}

// Zero the overwritten outputs of a split einsum (its chunks add into them).
template <typename T>
__device__ void zero_slots(const GenEinsum &G, const GenPtrs &P) {
  if (G.split <= 1) return;
  const int64_t total = G.out_size * G.n_slots;
  for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < total;
       f += (int64_t)gridDim.x * blockDim.x) {
    const int s = (int)(f / G.out_size);
    if (G.o_acc[s]) continue;
    ((T *)P.out[s])[gen_out_addr(G, s, f - s * G.out_size)] = (T)0;
  }
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
    gen_tile<T>(&table[w.einsum], &ptrs[w.einsum], w.slot, w.first, w.count, w.chunk);
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
  if (f64)
    hipLaunchKernelGGL(generic_kernel<double>, grid, block, 0, stream, dev, ptrs, tiles);
  else
    hipLaunchKernelGGL(generic_kernel<float>, grid, block, 0, stream, dev, ptrs, tiles);
  return hipGetLastError();
}

hipError_t launch_persistent(bool f64, const GenEinsum *table, const GenPtrs *ptrs,
                             const GenItem *items, int n_items, unsigned *counters, int grid,
                             hipStream_t stream, int n_einsums, bool any_split) {
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
  if (f64)
    hipLaunchKernelGGL(persistent_kernel<double>, dim3(grid), dim3(256), 0, stream, table, ptrs,
                       items, n_items, counters);
  else
    hipLaunchKernelGGL(persistent_kernel<float>, dim3(grid), dim3(256), 0, stream, table, ptrs,
                       items, n_items, counters);
  return hipGetLastError();
}

}  // namespace bes
