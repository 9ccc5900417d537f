// FEM-stream template, "apply" class, for gfx950.
//
// The face-mass and local-divergence batched einsums of Section "Batched
// einsums in DG-FEM Operators" (their kernel patterns are listed in Appendix
// "DG-FEM Batched Einsum Kernel Patterns").  Per element e and member m:
//   W_m[c, j]   = sum_x G[x, c, e] U_m[x, e, j]      (face mass: G[c, e] U_m[c, e, j])
//   out_m[e, i] = sum_{c, j} S[c, i, j] W_m[c, j]
// i.e. the streamed operand is first combined with the per-element geometry
// terms, then the shared reference matrix is applied -- the reverse of the
// local-gradient class, whose shared matrix acts first.  Members share S and
// G (the reference matrix and the geometry of the mesh); each has its own
// streamed field U_m.
//
// Mapping: one element per lane, 64-element tiles, four independent waves per
// block.  S sits in LDS once per block as [c][j][i] (every wave reads the
// same address: an LDS broadcast feeds the FMA); a wave takes (tile, member)
// work items, keeps its element's geometry terms and all NI outputs in
// registers, and streams U through a private LDS staging area JC columns at a
// time: coalesced global loads, transposed to [x][j][lane] at an odd pitch,
// then each lane reads its own element's values.  W is never stored: each
// combined value goes straight into the NI output FMAs.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"
#include "../../../include/bes.h"

namespace bes {

namespace {

constexpr int kTile = 64;
constexpr int kPitch = kTile + 1;
constexpr int kWaves = 4;            // independent waves per block

// Ordering of one wave's own LDS accesses: LDS executes a wave's
// instructions in order; only the compiler must not move accesses across.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <typename T>
__device__ __forceinline__ T apply_op(int op, T v) {
  switch (op) {
    case BES_OP_SIN: return sin(v);
    case BES_OP_COS: return cos(v);
    case BES_OP_SQUARE: return v * v;
    default: return v;
  }
}

// Columns of U staged per pass: a divisor of NJ near 5 keeps the staging area
// small (LDS is shared with S and three other waves).
template <int NJ>
constexpr int kJC = (NJ % 5 == 0) ? 5 : (NJ % 4 == 0 ? 4 : (NJ <= 6 ? NJ : 1));

template <int NI>
constexpr int kNIP = (NI + 1) & ~1;   // S rows padded to an even length

// S re-laid as [c][j][i] (rows padded to NIP) for the scalar-operand
// variant, which reads it through the scalar data cache.
template <typename T>
__global__ void __launch_bounds__(256) apply_pack_kernel(const FemApplyArgs a, T *__restrict__ dst,
                                                         int NI, int NJ, int NC, int NIP) {
  const T *__restrict__ S = (const T *)a.S;
  for (int f = blockIdx.x * 256 + threadIdx.x; f < NC * NJ * NIP; f += gridDim.x * 256) {
    const int i = f % NIP, cj = f / NIP;
    const int c = cj / NJ, j = cj - c * NJ;
    dst[f] = i < NI ? S[c * a.ss[0] + i * a.ss[1] + j * a.ss[2]] : (T)0;
  }
}

// SREG: S is read from the packed copy `Sp` at wave-uniform addresses, so it
// reaches the FMAs through the scalar data cache as scalar operands (for S
// that fits in that cache); otherwise S sits in LDS and every lane reads the
// same address (a broadcast).
template <typename T, int NI, int NJ, int NC, int NX, bool DIAG, bool EW, bool SREG>
__global__ void __launch_bounds__(kWaves * kTile)
    fem_apply_kernel(const FemApplyArgs a, const T *__restrict__ Sp, int64_t n_items) {
  constexpr int JC = kJC<NJ>;
  constexpr int NIP = kNIP<NI>;
  constexpr int NG = DIAG ? NC : NX * NC;     // geometry values per element
  __shared__ T S_l[SREG ? 2 : NC * NJ * NIP];
  __shared__ T X_l[kWaves][NX * JC * kPitch];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // S into LDS as [c][j][i] from the caller's strides (once per block).
  if constexpr (!SREG) {
    const T *__restrict__ S = (const T *)a.S;
    for (int f = threadIdx.x; f < NC * NJ * NIP; f += kWaves * kTile) {
      const int i = f % NIP, cj = f / NIP;
      const int c = cj / NJ, j = cj - c * NJ;
      S_l[f] = i < NI ? S[c * a.ss[0] + i * a.ss[1] + j * a.ss[2]] : (T)0;
    }
    __syncthreads();
  }
  T *__restrict__ X = X_l[wave];
  const int b = a.n_members;
  const T alpha = (T)a.alpha, beta = (T)a.beta;
  const int64_t stride = (int64_t)gridDim.x * kWaves;
  for (int64_t item = (int64_t)blockIdx.x * kWaves + wave; item < n_items; item += stride) {
    const int64_t tile = item / b;
    const int m = (int)(item - tile * b);
    const int64_t e0 = tile * kTile;
    const int64_t e = e0 + lane;
    const bool valid = e < a.E;
    const int n_el = (int)min((int64_t)kTile, a.E - e0);
    // geometry terms of this lane's element
    T g[NG];
    {
      const T *__restrict__ G = (const T *)a.G;
#pragma unroll
      for (int q = 0; q < NG; ++q) {
        const int x = DIAG ? 0 : q / NC, c = DIAG ? q : q % NC;
        g[q] = valid ? G[x * a.gs[0] + c * a.gs[1] + e * a.gs[2]] : (T)0;
      }
    }
    T y[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) y[i] = (T)0;
    const FemApplyMember &M = a.mem[m];
    // per-tile bases are wave-uniform; per-lane offsets within a tile are
    // 32-bit (the planner checks that they fit)
    const T *__restrict__ U0 = (const T *)M.u0 + M.uoff0 + e0 * M.us0[1];
    const T *__restrict__ U1 =
        M.u1 ? (const T *)M.u1 + M.uoff1 + e0 * M.us1[1] : U0;
    const int se0 = (int)M.us0[1], sj0 = (int)M.us0[2];
    const int se1 = (int)M.us1[1], sj1 = (int)M.us1[2];
#pragma unroll 1
    for (int jc = 0; jc < NJ; jc += JC) {
      // stage U[x][e0 .. e0+63][jc .. jc+JC) as X[x][jj][element]: all loads
      // of the pass first, then the LDS writes
      T v[NX][JC];
#pragma unroll
      for (int x = 0; x < NX; ++x) {
        const T *__restrict__ px = U0 + x * M.us0[0] + (int64_t)jc * sj0;
#pragma unroll
        for (int q = 0; q < JC; ++q) {
          const int f = lane + kTile * q;
          const int el = f / JC, jj = f - el * JC;
          v[x][q] = el < n_el ? px[el * se0 + jj * sj0] : (T)0;
        }
      }
#pragma unroll
      for (int x = 0; x < NX; ++x)
#pragma unroll
        for (int q = 0; q < JC; ++q) {
          const int f = lane + kTile * q;
          const int el = f / JC, jj = f - el * JC;
          X[(x * JC + jj) * kPitch + el] = v[x][q];
        }
      if constexpr (EW) {
        // element-wise functional operand alpha*op(U0) + beta (+ U1) on the
        // staged values: a rolled loop keeps one copy of op's code
        wave_sync();
#pragma unroll 1
        for (int k = 0; k < NX * JC; ++k) {
          const int x = k / JC, q = k - x * JC;
          const int f = lane + kTile * q;
          const int el = f / JC, jj = f - el * JC;
          T *cell = &X[(x * JC + jj) * kPitch + el];
          const T w = (M.u1 && el < n_el)
                          ? U1[x * M.us1[0] + (int64_t)jc * sj1 + el * se1 + jj * sj1]
                          : (T)0;
          if (el < n_el) *cell = alpha * apply_op<T>(a.op, *cell) + beta + w;
        }
      }
      wave_sync();
#pragma unroll
      for (int jj = 0; jj < JC; ++jj) {
        T u[NX];
#pragma unroll
        for (int x = 0; x < NX; ++x) u[x] = X[(x * JC + jj) * kPitch + lane];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          T w;
          if constexpr (DIAG) {
            w = g[c] * u[c];
          } else {
            w = g[c] * u[0];
#pragma unroll
            for (int x = 1; x < NX; ++x) w = fma(g[x * NC + c], u[x], w);
          }
          const T *__restrict__ srow = SREG ? Sp + (c * NJ + jc + jj) * NIP
                                            : &S_l[(c * NJ + jc + jj) * NIP];
#pragma unroll
          for (int i = 0; i < NI; ++i) y[i] = fma(srow[i], w, y[i]);
        }
      }
      wave_sync();
    }
    if (valid) {
      T *__restrict__ out = (T *)M.out + e * M.oe;
#pragma unroll
      for (int i = 0; i < NI; ++i) out[i * M.oi] = y[i];
    }
  }
}

template <typename T, int NI, int NJ, int NC, int NX, bool DIAG>
hipError_t launch_apply_shape(const FemApplyArgs &a, const T *Sp, int blocks_per_cu,
                              bool sreg, hipStream_t stream) {
  const int64_t tiles = (a.E + kTile - 1) / kTile;
  const int64_t items = tiles * a.n_members;
  const int64_t cap = (int64_t)device_cu_count() * std::max(1, blocks_per_cu);
  const int64_t blocks = std::min<int64_t>((items + kWaves - 1) / kWaves, cap);
  const dim3 grid((unsigned)blocks), block(kWaves * kTile);
  // the functional-operand prologue has its own instantiations, so the plain
  // path carries none of its code or registers
  const bool ew = a.u_kind == FEM_SRC_ELEMENTWISE;
  if (ew && sreg)
    hipLaunchKernelGGL((fem_apply_kernel<T, NI, NJ, NC, NX, DIAG, true, true>), grid, block, 0,
                       stream, a, Sp, items);
  else if (ew)
    hipLaunchKernelGGL((fem_apply_kernel<T, NI, NJ, NC, NX, DIAG, true, false>), grid, block, 0,
                       stream, a, Sp, items);
  else if (sreg)
    hipLaunchKernelGGL((fem_apply_kernel<T, NI, NJ, NC, NX, DIAG, false, true>), grid, block, 0,
                       stream, a, Sp, items);
  else
    hipLaunchKernelGGL((fem_apply_kernel<T, NI, NJ, NC, NX, DIAG, false, false>), grid, block, 0,
                       stream, a, Sp, items);
  return hipGetLastError();
}

}  // namespace

size_t fem_apply_workspace_bytes(bool f64, int NI, int NJ, int NC) {
  return (size_t)NC * NJ * ((NI + 1) & ~1) * (f64 ? 8 : 4);
}

hipError_t launch_fem_apply(bool f64, int NI, int NJ, int NC, int NX, bool diag,
                            const FemApplyArgs &a, void *workspace, int blocks_per_cu,
                            int variant, hipStream_t stream, hipEvent_t ev_start,
                            hipEvent_t ev_stop) {
  if (a.E <= 0 || a.n_members <= 0) return hipSuccess;
  // variant 2: S as scalar operands; 0 and 1: S in LDS (measured faster on
  // most shapes; the tuner picks per shape)
  const bool sreg = variant == 2;
  if (sreg && !workspace) return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
  if (sreg) {
    const int NIP = (NI + 1) & ~1;
    const int total = NC * NJ * NIP;
    const unsigned g = (unsigned)std::min(64, (total + 255) / 256);
    if (f64)
      hipLaunchKernelGGL(apply_pack_kernel<double>, dim3(g), dim3(256), 0, stream, a,
                         (double *)workspace, NI, NJ, NC, NIP);
    else
      hipLaunchKernelGGL(apply_pack_kernel<float>, dim3(g), dim3(256), 0, stream, a,
                         (float *)workspace, NI, NJ, NC, NIP);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (ev_start && (e = hipEventRecord(ev_start, stream)) != hipSuccess) return e;
  e = hipErrorInvalidValue;
#define BES_APPLY_DISPATCH(ni, nj, nc, nx, dg)                                              \
  if (NI == ni && NJ == nj && NC == nc && NX == nx && diag == dg)                           \
    e = f64 ? launch_apply_shape<double, ni, nj, nc, nx, dg>(a, (const double *)workspace,  \
                                                             blocks_per_cu, sreg, stream)   \
            : launch_apply_shape<float, ni, nj, nc, nx, dg>(a, (const float *)workspace,    \
                                                            blocks_per_cu, sreg, stream);
  BES_FEM_APPLY_SHAPES(BES_APPLY_DISPATCH)
#undef BES_APPLY_DISPATCH
  if (e != hipSuccess) return e;
  if (ev_stop && (e = hipEventRecord(ev_stop, stream)) != hipSuccess) return e;
  return hipSuccess;
}

}  // namespace bes
