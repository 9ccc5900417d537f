// FEM-stream template for gfx950.
//
// Batched einsums of the DG-FEM local-gradient class (Section "Batched einsums
// in DG-FEM Operators"): a long stream index e present in the output and in
// the per-element operands U (and G), and one small operand S without e that
// every element reuses.  Per element e, for each stage-1 group g and each of
// its members m:
//   T[r, i]       = sum_j S_g[r, i, j] U_g[e, j]
//   out_m[e,x,i]  = sum_r G_m[e, x, r] T[r, i]
// which is the factored contraction order (loop permutation and hoisting) the
// paper's transformations use to cut FLOPs; members whose S and U are the same
// arguments share T (the reuse that motivates batching in the first place).
//
// Mapping: one work-item per element, grid-stride over e.  S is read with
// wave-uniform addresses straight from global memory, so the compiler keeps
// it in scalar registers (s_load) and every v_fma takes it as the scalar
// operand: no LDS traffic for the shared operand.  Functional operands (the
// functions M(A)) are evaluated in registers as the sources are read:
// alpha*op(S0)+beta(+S1) for U and G, and the tetrahedron Jacobian from the
// four vertex coordinates for G.
#include <hip/hip_runtime.h>

#include "../fem_shapes.h"
#include "kernels.h"
#include "../../../include/bes.h"

namespace bes {

namespace {

template <typename T>
__device__ __forceinline__ T apply_op(int op, T v) {
  switch (op) {
    case BES_OP_SIN: return sin(v);
    case BES_OP_COS: return cos(v);
    case BES_OP_SQUARE: return v * v;
    default: return v;
  }
}

// U_g[e, 0..NJ) into registers.
template <typename T, int NJ>
__device__ __forceinline__ void load_u(const FemSrc &s, int64_t e, T (&u)[NJ]) {
  const T *__restrict__ p0 = (const T *)s.p0 + s.off0 + e * s.s0[0];
  const int64_t sj = s.s0[1];
  if (s.kind == FEM_SRC_ARRAY) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) u[j] = p0[j * sj];
    return;
  }
  const T alpha = (T)s.alpha, beta = (T)s.beta;
  const int op = s.op;
#pragma unroll
  for (int j = 0; j < NJ; ++j) u[j] = alpha * apply_op<T>(op, p0[j * sj]) + beta;
  if (s.p1) {
    const T *__restrict__ p1 = (const T *)s.p1 + s.off1 + e * s.s1[0];
    const int64_t sj1 = s.s1[1];
#pragma unroll
    for (int j = 0; j < NJ; ++j) u[j] += p1[j * sj1];
  }
}

// G_m[e, 0..NX, 0..NR) into registers.
template <typename T, int NX, int NR>
__device__ __forceinline__ void load_g(const FemSrc &s, int64_t e, T (&g)[NX][NR]) {
  if (s.kind == FEM_SRC_TET) {
    // V[e, vertex, coordinate]; J[x][r] = V[r+1][x] - V[0][x]
    const T *__restrict__ V = (const T *)s.p0 + s.off0 + e * s.s0[0];
    const int64_t sv = s.s0[1], sc = s.s0[2];
    T v[4][3];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) v[k][c] = V[k * sv + c * sc];
    const bool swapped = s.s1[0] != 0;
#pragma unroll
    for (int x = 0; x < NX; ++x)
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int xx = swapped ? r : x, rr = swapped ? x : r;
        g[x][r] = v[(rr + 1) % 4][xx % 3] - v[0][xx % 3];
      }
    return;
  }
  const T *__restrict__ p0 = (const T *)s.p0 + s.off0 + e * s.s0[0];
  const int64_t sx = s.s0[1], sr = s.s0[2];
#pragma unroll
  for (int x = 0; x < NX; ++x)
#pragma unroll
    for (int r = 0; r < NR; ++r) g[x][r] = p0[x * sx + r * sr];
  if (s.kind == FEM_SRC_ELEMENTWISE) {
    const T alpha = (T)s.alpha, beta = (T)s.beta;
#pragma unroll
    for (int x = 0; x < NX; ++x)
#pragma unroll
      for (int r = 0; r < NR; ++r) g[x][r] = alpha * apply_op<T>(s.op, g[x][r]) + beta;
    if (s.p1) {
      const T *__restrict__ p1 = (const T *)s.p1 + s.off1 + e * s.s1[0];
#pragma unroll
      for (int x = 0; x < NX; ++x)
#pragma unroll
        for (int r = 0; r < NR; ++r) g[x][r] += p1[x * s.s1[1] + r * s.s1[2]];
    }
  }
}

template <typename T, int NI, int NJ, int NR, int NX, int MPG>
__global__ void __launch_bounds__(256) fem_stream_kernel(const FemArgs a) {
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < a.E; e += step) {
    for (int g = 0; g < a.n_groups; ++g) {
      const FemGroup &G = a.grp[g];
      T u[NJ];
      load_u<T, NJ>(G.u, e, u);
      const int m0 = G.m0, nm = G.m1 - G.m0;
      const bool has_g = a.mem[m0].g.kind != FEM_SRC_NONE;
      T gm[MPG][NX][NR];
#pragma unroll
      for (int q = 0; q < MPG; ++q)
        if (q < nm && has_g) load_g<T, NX, NR>(a.mem[m0 + q].g, e, gm[q]);
      const T *__restrict__ S = (const T *)G.S;
      for (int i = 0; i < NI; ++i) {
        T t[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const T *__restrict__ Srow = S + ((int64_t)r * NI + i) * NJ;
          T acc = 0;
#pragma unroll
          for (int j = 0; j < NJ; ++j) acc = fma(Srow[j], u[j], acc);
          t[r] = acc;
        }
#pragma unroll
        for (int q = 0; q < MPG; ++q) {
          if (q >= nm) break;
          const FemMember &M = a.mem[m0 + q];
          T *__restrict__ o = (T *)M.out + e * M.oe + i * M.oi;
          if (!has_g) {
            o[0] = t[0];
            continue;
          }
#pragma unroll
          for (int x = 0; x < NX; ++x) {
            T acc = 0;
#pragma unroll
            for (int r = 0; r < NR; ++r) acc = fma(gm[q][x][r], t[r], acc);
            o[x * M.ox] = acc;
          }
        }
      }
    }
  }
}

template <typename T, int NI, int NJ, int NR, int NX>
hipError_t launch_shape(const FemArgs &a, int mpg, dim3 grid, dim3 block, hipStream_t s) {
  if (mpg == 1)
    hipLaunchKernelGGL((fem_stream_kernel<T, NI, NJ, NR, NX, 1>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((fem_stream_kernel<T, NI, NJ, NR, NX, 3>), grid, block, 0, s, a);
  return hipGetLastError();
}

// Split groups with more than `mpg` members into several groups that share
// S and U (T is then recomputed per chunk).
FemArgs chunk_groups(const FemArgs &in, int mpg) {
  FemArgs out = in;
  out.n_groups = 0;
  for (int g = 0; g < in.n_groups; ++g) {
    for (int m = in.grp[g].m0; m < in.grp[g].m1; m += mpg) {
      FemGroup G = in.grp[g];
      G.m0 = m;
      G.m1 = m + mpg < in.grp[g].m1 ? m + mpg : in.grp[g].m1;
      out.grp[out.n_groups++] = G;
    }
  }
  return out;
}

}  // namespace

int device_cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cached[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

hipError_t launch_fem(bool f64, int NI, int NJ, int NR, int NX, const FemArgs &a, int block,
                      int blocks_per_cu, hipStream_t stream) {
  if (a.E <= 0) return hipSuccess;
  int maxm = 0;
  for (int g = 0; g < a.n_groups; ++g) maxm = std::max(maxm, a.grp[g].m1 - a.grp[g].m0);
  const int mpg = maxm <= 1 ? 1 : 3;
  FemArgs c = chunk_groups(a, mpg);
  if (c.n_groups > BES_FEM_MAX_GROUPS) return hipErrorInvalidValue;
  if (block != 64 && block != 128 && block != 256) block = 256;
  if (blocks_per_cu < 1) blocks_per_cu = 1;
  int64_t need = (a.E + block - 1) / block;
  int64_t cap = (int64_t)device_cu_count() * blocks_per_cu * (256 / block);
  dim3 grid((unsigned)std::min<int64_t>(need, cap)), blk(block);
#define BES_FEM_DISPATCH(ni, nj, nr, nx)                                              \
  if (NI == ni && NJ == nj && NR == nr && NX == nx)                                   \
    return f64 ? launch_shape<double, ni, nj, nr, nx>(c, mpg, grid, blk, stream)      \
               : launch_shape<float, ni, nj, nr, nx>(c, mpg, grid, blk, stream);
  BES_FEM_SHAPES(BES_FEM_DISPATCH)
#undef BES_FEM_DISPATCH
  return hipErrorInvalidValue;
}

}  // namespace bes
