// FEM-stream template for gfx950.
//
// Batched einsums of the DG-FEM local-gradient class (Section "Batched einsums
// in DG-FEM Operators"): a long stream index e present in the output and in
// the per-element operands U (and G), and one small operand S without e that
// every element reuses.  Per element e, for each stage-1 group g and each of
// its members m:
//   T[r, i]       = sum_j S_g[r, i, j] U_g[e, j]
//   out_m[e,x,i]  = sum_r G_m[e, x, r] T[r, i]
// the factored contraction order (loop permutation and hoisting) the paper's
// DG-FEM transformations use to cut FLOPs; members whose S and U are the same
// arguments share T (the operand reuse that motivates batching).
//
// Mapping (one wave per block, a tile of 64 consecutive elements per wave,
// one element per lane):
//   * staging: every per-element source is read with coalesced loads (lane k
//     reads flat position k, k+64, ... of the tile's rows) and written to LDS
//     transposed, [component][lane] with an odd pitch, so each lane then reads
//     its own element's components without bank conflicts.  Element-wise
//     functional operands (alpha*op(S0)+beta+S1) are evaluated during that
//     coalesced pass, in registers; the tetrahedron Jacobian is formed from
//     the staged vertex row;
//   * stage 1 runs j-outer over S packed as [r][j][i]: S is wave-uniform, so
//     it lives in scalar registers (contiguous s_load) and is the scalar
//     operand of every v_fma; T[r][i] stays in vector registers;
//   * stage 2 writes each (member, x) output row for the 64 elements to LDS
//     and then to HBM as one contiguous run per element (consecutive lanes,
//     consecutive addresses).
#include <hip/hip_runtime.h>

#include "../fem_shapes.h"
#include "kernels.h"
#include "../../../include/bes.h"

namespace bes {

namespace {

constexpr int kTile = 64;      // elements per wave tile = lanes per wave
constexpr int kPitch = kTile + 1;
constexpr int kMaxRow = 12;    // staged G row width (TET: 4 x 3 vertex coords)

template <typename T>
__device__ __forceinline__ T apply_op(int op, T v) {
  switch (op) {
    case BES_OP_SIN: return sin(v);
    case BES_OP_COS: return cos(v);
    case BES_OP_SQUARE: return v * v;
    default: return v;
  }
}

// Out-of-line element-wise function: keeps the transcendental expansions from
// being interleaved across a whole unrolled row (register pressure).
template <typename T>
__device__ __noinline__ T elementwise_call(int op, T v, T alpha, T beta, T w) {
  return alpha * apply_op<T>(op, v) + beta + w;
}

// Stage `W` components of every element of the tile [e0, e0 + n) into
// lds[c * kPitch + el].  Component c of element e sits at
//   p0[off0 + e * s0e + pos0(c)]  (and p1[off1 + e * s1e + pos1(c)])
// where pos(c) = (c / div) * sa + (c % div) * sb.  Loads walk the flat index
// f = el * W + c with consecutive lanes on consecutive f (coalesced when the
// rows are dense).  Element-wise prologues are applied here.
// In-tile offsets are 32-bit element counts from a wave-uniform base pointer
// (the planner guarantees they fit), so each load needs one address VGPR.
template <typename T, int W, int DIV, bool EW>
__device__ __forceinline__ void stage_rows(T *__restrict__ lds, const FemSrc &s, int64_t sa0,
                                           int64_t sb0, int64_t sa1, int64_t sb1, int64_t e0,
                                           int n, int lane) {
  const T *__restrict__ p0 = (const T *)s.p0 + s.off0 + e0 * s.s0[0];
  const int se0 = (int)s.s0[0], a0 = (int)sa0, b0 = (int)sb0;
  const bool ew = EW && s.kind == FEM_SRC_ELEMENTWISE;
  const bool two = ew && s.p1 != nullptr;
  const T *__restrict__ p1 = two ? (const T *)s.p1 + s.off1 + e0 * s.s1[0] : p0;
  const int se1 = (int)s.s1[0], a1 = (int)sa1, b1 = (int)sb1;
  const T alpha = (T)s.alpha, beta = (T)s.beta;
  if (n == kTile) {
    // Full tile: W loads per lane, all issued before any is consumed so their
    // HBM latencies overlap; the prologue and the LDS writes follow.
    T v[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const int f = lane + kTile * k;
      const int el = f / W, c = f - el * W;
      const int ca = c / DIV, cb = c - ca * DIV;
      v[k] = p0[el * se0 + ca * a0 + cb * b0];
    }
    if (ew) {
      T w[W];
#pragma unroll
      for (int k = 0; k < W; ++k) {
        const int f = lane + kTile * k;
        const int el = f / W, c = f - el * W;
        const int ca = c / DIV, cb = c - ca * DIV;
        w[k] = two ? p1[el * se1 + ca * a1 + cb * b1] : (T)0;
      }
#pragma unroll
      for (int k = 0; k < W; ++k) {
        if constexpr (EW) v[k] = elementwise_call<T>(s.op, v[k], alpha, beta, w[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const int f = lane + kTile * k;
      const int el = f / W, c = f - el * W;
      lds[c * kPitch + el] = v[k];
    }
    return;
  }
  const int total = n * W;
  for (int f = lane; f < total; f += kTile) {
    const int el = f / W, c = f - el * W;
    const int ca = c / DIV, cb = c - ca * DIV;
    T v = p0[el * se0 + ca * a0 + cb * b0];
    if constexpr (EW) {
      if (ew) v = elementwise_call<T>(s.op, v, alpha, beta, two ? p1[el * se1 + ca * a1 + cb * b1] : (T)0);
    }
    lds[c * kPitch + el] = v;
  }
}

// Tetrahedron Jacobian of this lane's element from its staged vertex row
// (components vertex * 3 + coordinate): J[x][r] = V[r+1][x] - V[0][x]; the
// kernel's (x, r) may be the operand's (r, x).  NX = NR = 3 on this path.
template <typename T, int NX, int NR>
__device__ __forceinline__ void tet_from_lds(const T *__restrict__ lds, int lane, bool swapped,
                                             T (&g)[NX][NR]) {
  T v[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) v[k][c] = lds[(k * 3 + c) * kPitch + lane];
#pragma unroll
  for (int x = 0; x < NX; ++x)
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const T jxr = v[(r + 1) & 3][x % 3] - v[0][x % 3];
      const T jrx = v[(x + 1) & 3][r % 3] - v[0][r % 3];
      g[x][r] = swapped ? jrx : jxr;
    }
}

// Kernels that may meet tetrahedron-Jacobian G operands: x = r = 3 and one
// member per group (the launcher keeps such groups at one member).
template <int NX, int NR, int MPG>
constexpr bool kTetCapable = NX == 3 && NR == 3 && MPG == 1;

// G_m[e, x, r] of every member of the group into registers.
//   Shared row (G.g_row > 0): one coalesced, fully unrolled pass stages the
//   row p0 + g_off + e * se + c, c < g_row, for the 64 elements; each member
//   then reads its components (views: offset off0 + x*sx + r*sr in the row;
//   tetrahedra: the 12 vertex coordinates).
//   Otherwise each member's components are staged in turn (rolled loop).
template <typename T, int NX, int NR, int MPG, bool EW>
__device__ __forceinline__ void load_group_g(T *__restrict__ lds, const FemArgs &a,
                                             const FemGroup &G, int m0, int nm, int64_t e0, int n,
                                             int lane, T (&gm)[MPG][NX][NR]) {
  if (G.g_row > 0) {
    const FemSrc &s0 = a.mem[m0].g;
    const T *__restrict__ pb = (const T *)s0.p0 + G.g_off + e0 * s0.s0[0];
    const int se = (int)s0.s0[0], row = G.g_row;
    if (n == kTile) {
      T v[kMaxRow];
#pragma unroll
      for (int k = 0; k < kMaxRow; ++k) {
        const int f = lane + kTile * k;
        const int el = f / kMaxRow, c = f - el * kMaxRow;
        v[k] = c < row ? pb[el * se + c] : (T)0;
      }
#pragma unroll
      for (int k = 0; k < kMaxRow; ++k) {
        const int f = lane + kTile * k;
        const int el = f / kMaxRow, c = f - el * kMaxRow;
        lds[c * kPitch + el] = v[k];
      }
    } else {
      for (int f = lane; f < n * row; f += kTile) {
        const int el = f / row, c = f - el * row;
        lds[c * kPitch + el] = pb[el * se + c];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MPG; ++q) {
      if (q >= nm) break;
      const FemSrc &s = a.mem[m0 + q].g;
      if (kTetCapable<NX, NR, MPG> && s.kind == FEM_SRC_TET) {
        if constexpr (kTetCapable<NX, NR, MPG>) tet_from_lds<T, NX, NR>(lds, lane, s.s1[0] != 0, gm[q]);
      } else {
        const int off = (int)s.off0, sx = (int)s.s0[1], sr = (int)s.s0[2];
#pragma unroll
        for (int x = 0; x < NX; ++x)
#pragma unroll
          for (int r = 0; r < NR; ++r) gm[q][x][r] = lds[(off + x * sx + r * sr) * kPitch + lane];
      }
    }
    __syncthreads();
    return;
  }
  for (int q = 0; q < nm && q < MPG; ++q) {
    const FemSrc &s = a.mem[m0 + q].g;
    const bool tet = s.kind == FEM_SRC_TET;
    const int W = tet ? 12 : NX * NR;
    const int div = tet ? 3 : NR;
    const int64_t sa = s.s0[1], sb = s.s0[2];
    const T *__restrict__ p0 = (const T *)s.p0 + s.off0 + e0 * s.s0[0];
    const T *__restrict__ p1 =
        s.p1 ? (const T *)s.p1 + s.off1 + e0 * s.s1[0] : nullptr;
    for (int f = lane; f < n * W; f += kTile) {
      const int el = f / W, c = f - el * W;
      const int ca = c / div, cb = c - ca * div;
      T v = p0[el * s.s0[0] + ca * sa + cb * sb];
      if constexpr (EW) {
        if (s.kind == FEM_SRC_ELEMENTWISE)
          v = elementwise_call<T>(s.op, v, (T)s.alpha, (T)s.beta,
                                  p1 ? p1[el * s.s1[0] + ca * s.s1[1] + cb * s.s1[2]] : (T)0);
      }
      lds[c * kPitch + el] = v;
    }
    __syncthreads();
    // Every member is read with static indices in the q-unrolled loop below.
#pragma unroll
    for (int qq = 0; qq < MPG; ++qq) {
      if (qq != q) continue;
      if (kTetCapable<NX, NR, MPG> && tet) {
        if constexpr (kTetCapable<NX, NR, MPG>) tet_from_lds<T, NX, NR>(lds, lane, s.s1[0] != 0, gm[qq]);
      } else {
#pragma unroll
        for (int x = 0; x < NX; ++x)
#pragma unroll
          for (int r = 0; r < NR; ++r) gm[qq][x][r] = lds[(x * NR + r) * kPitch + lane];
      }
    }
    __syncthreads();
  }
}

template <typename T, int NI, int NJ, int NR, int NX, int MPG, bool EW>
__global__ void __launch_bounds__(kTile) fem_stream_kernel(const FemArgs a,
                                                           const T *__restrict__ Spack) {
  constexpr int kRowsU = NJ > NI ? NJ : NI;
  __shared__ T lds_u[kRowsU * kPitch];   // U staging, then output staging
  __shared__ T lds_g[kMaxRow * kPitch];  // G staging
  const int lane = threadIdx.x;
  const int64_t n_tiles = (a.E + kTile - 1) / kTile;
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int64_t e0 = tile * kTile;
    const int n = (int)(a.E - e0 < kTile ? a.E - e0 : kTile);
    for (int g = 0; g < a.n_groups; ++g) {
      const FemGroup &G = a.grp[g];
      const int m0 = G.m0, nm = G.m1 - G.m0;
      const bool has_g = a.mem[m0].g.kind != FEM_SRC_NONE;
      // G of every member of the group (registers).
      T gm[MPG][NX][NR];
      if (has_g) load_group_g<T, NX, NR, MPG, EW>(lds_g, a, G, m0, nm, e0, n, lane, gm);
      // U rows of the tile, prologue applied, transposed into LDS.
      stage_rows<T, NJ, NJ, EW>(lds_u, G.u, 0, G.u.s0[1], 0, G.u.s1[1], e0, n, lane);
      __syncthreads();
      // Stage 1: T[r][i] = sum_j S[r][j][i] u[j], S uniform (scalar operand).
      T t[NR][NI];
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int i = 0; i < NI; ++i) t[r][i] = 0;
      // r outer, j inner: one step needs the NI values S[r][j][:] (NI scalar
      // register pairs), so the scalar file can hold the next step's S too.
      const T *__restrict__ S = Spack + (int64_t)g * NR * NJ * NI;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
#pragma unroll 2
        for (int j = 0; j < NJ; ++j) {
          const T uj = lds_u[j * kPitch + lane];
          const T *__restrict__ Srow = S + ((int64_t)r * NJ + j) * NI;
#pragma unroll
          for (int i = 0; i < NI; ++i) t[r][i] = fma(Srow[i], uj, t[r][i]);
        }
      }
      __syncthreads();
      // Stage 2 and contiguous stores, one (member, x) row block at a time.
#pragma unroll
      for (int q = 0; q < MPG; ++q) {
        if (q >= nm) break;
        const FemMember &M = a.mem[m0 + q];
        T *__restrict__ outp = (T *)M.out + e0 * M.oe;
#pragma unroll
        for (int x = 0; x < NX; ++x) {
#pragma unroll
          for (int i = 0; i < NI; ++i) {
            T acc;
            if (has_g) {
              acc = gm[q][x][0] * t[0][i];
#pragma unroll
              for (int r = 1; r < NR; ++r) acc = fma(gm[q][x][r], t[r][i], acc);
            } else {
              acc = t[0][i];
            }
            lds_u[i * kPitch + lane] = acc;
          }
          __syncthreads();
          T *__restrict__ ox = outp + x * M.ox;
          const int oe = (int)M.oe, oi = (int)M.oi;
          if (n == kTile) {
#pragma unroll 4
            for (int k = 0; k < NI; ++k) {
              const int f = lane + kTile * k;
              const int el = f / NI, i = f - el * NI;
              ox[el * oe + i * oi] = lds_u[i * kPitch + el];
            }
          } else {
            const int total = n * NI;
            for (int f = lane; f < total; f += kTile) {
              const int el = f / NI, i = f - el * NI;
              ox[el * oe + i * oi] = lds_u[i * kPitch + el];
            }
          }
          __syncthreads();
        }
      }
    }
  }
}

// S of every group packed as [group][r][j][i] from the caller's strides.
struct PackArgs {
  const void *S[BES_FEM_MAX_GROUPS];
  int64_t sr[BES_FEM_MAX_GROUPS], si[BES_FEM_MAX_GROUPS], sj[BES_FEM_MAX_GROUPS];
  int n_groups, NR, NI, NJ;
};

template <typename T>
__global__ void __launch_bounds__(256) pack_s_kernel(const PackArgs a, T *__restrict__ dst) {
  const int per = a.NR * a.NJ * a.NI;
  const int total = per * a.n_groups;
  for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < total; f += gridDim.x * blockDim.x) {
    const int g = f / per;
    int rem = f - g * per;
    const int r = rem / (a.NJ * a.NI);
    rem -= r * a.NJ * a.NI;
    const int j = rem / a.NI, i = rem - j * a.NI;
    dst[f] = ((const T *)a.S[g])[r * a.sr[g] + i * a.si[g] + j * a.sj[g]];
  }
}

template <typename T, int NI, int NJ, int NR, int NX>
hipError_t launch_shape(const FemArgs &a, const T *spack, int mpg, bool ew, dim3 grid,
                        hipStream_t s) {
  // Functional (element-wise) operands get their own instantiation, so the
  // plain kernels carry no prologue code; those keep one member per group.
  if (ew)
    hipLaunchKernelGGL((fem_stream_kernel<T, NI, NJ, NR, NX, 1, true>), grid, dim3(kTile), 0, s,
                       a, spack);
  else if (mpg == 1)
    hipLaunchKernelGGL((fem_stream_kernel<T, NI, NJ, NR, NX, 1, false>), grid, dim3(kTile), 0, s,
                       a, spack);
  else
    hipLaunchKernelGGL((fem_stream_kernel<T, NI, NJ, NR, NX, 3, false>), grid, dim3(kTile), 0, s,
                       a, spack);
  return hipGetLastError();
}

// Split groups with more than `mpg` members into several groups that share
// S and U (T is then recomputed per chunk).
FemArgs chunk_groups(const FemArgs &in, int mpg, int *group_of_chunk) {
  FemArgs out = in;
  out.n_groups = 0;
  for (int g = 0; g < in.n_groups; ++g) {
    for (int m = in.grp[g].m0; m < in.grp[g].m1; m += mpg) {
      if (out.n_groups >= BES_FEM_MAX_GROUPS) {
        out.n_groups = BES_FEM_MAX_GROUPS + 1;
        return out;
      }
      FemGroup G = in.grp[g];
      G.m0 = m;
      G.m1 = m + mpg < in.grp[g].m1 ? m + mpg : in.grp[g].m1;
      group_of_chunk[out.n_groups] = g;
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

size_t fem_workspace_bytes(bool f64, int NI, int NJ, int NR) {
  return (size_t)BES_FEM_MAX_GROUPS * NR * NJ * NI * (f64 ? 8 : 4);
}

hipError_t launch_fem(bool f64, int NI, int NJ, int NR, int NX, const FemArgs &a, void *workspace,
                      int blocks_per_cu, hipStream_t stream) {
  if (a.E <= 0) return hipSuccess;
  if (!workspace) return hipErrorInvalidValue;
  int maxm = 0;
  for (int g = 0; g < a.n_groups; ++g) maxm = std::max(maxm, a.grp[g].m1 - a.grp[g].m0);
  bool ew = false, tet = false;
  for (int g = 0; g < a.n_groups; ++g) ew |= a.grp[g].u.kind == FEM_SRC_ELEMENTWISE;
  for (int m = 0; m < a.n_members; ++m) {
    ew |= a.mem[m].g.kind == FEM_SRC_ELEMENTWISE;
    tet |= a.mem[m].g.kind == FEM_SRC_TET;
  }
  const int mpg = (maxm <= 1 || ew || tet) ? 1 : 3;
  int chunk_src[BES_FEM_MAX_GROUPS + 1];
  FemArgs c = chunk_groups(a, mpg, chunk_src);
  if (c.n_groups > BES_FEM_MAX_GROUPS) return hipErrorInvalidValue;
  // Pack S of every chunk (chunks of one group repeat its S).
  PackArgs pk;
  pk.n_groups = c.n_groups;
  pk.NR = NR;
  pk.NI = NI;
  pk.NJ = NJ;
  for (int k = 0; k < c.n_groups; ++k) {
    pk.S[k] = c.grp[k].S;
    pk.sr[k] = c.grp[k].ss[0];
    pk.si[k] = c.grp[k].ss[1];
    pk.sj[k] = c.grp[k].ss[2];
  }
  const int pack_total = NR * NJ * NI * c.n_groups;
  dim3 pgrid((pack_total + 255) / 256);
  if (f64)
    hipLaunchKernelGGL(pack_s_kernel<double>, pgrid, dim3(256), 0, stream, pk, (double *)workspace);
  else
    hipLaunchKernelGGL(pack_s_kernel<float>, pgrid, dim3(256), 0, stream, pk, (float *)workspace);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (blocks_per_cu < 1) blocks_per_cu = 1;
  const int64_t tiles = (a.E + kTile - 1) / kTile;
  const int64_t cap = (int64_t)device_cu_count() * blocks_per_cu;
  dim3 grid((unsigned)std::min<int64_t>(tiles, cap));
#define BES_FEM_DISPATCH(ni, nj, nr, nx)                                                  \
  if (NI == ni && NJ == nj && NR == nr && NX == nx)                                       \
    return f64 ? launch_shape<double, ni, nj, nr, nx>(c, (const double *)workspace, mpg, ew, grid, \
                                                      stream)                             \
               : launch_shape<float, ni, nj, nr, nx>(c, (const float *)workspace, mpg, ew, grid, \
                                                     stream);
  BES_FEM_SHAPES(BES_FEM_DISPATCH)
#undef BES_FEM_DISPATCH
  return hipErrorInvalidValue;
}

}  // namespace bes
