// MFMA dense-contraction template for gfx950 (FP32 in, FP32 accumulate).
//
// A batched einsum whose members are pure two-operand contractions is, after
// merging each index group (M: free indices of A, N: free indices of B, K:
// contracted) into one strided axis, a GEMM per member:
//   C_s[M, N] = sum over members m of slot s of A_m[M, K] B_m[K, N]
// with arbitrary strides on A, B and C (no transposed copy is ever made: tiles
// are read in whichever direction is contiguous and written to LDS in the
// layout the matrix cores consume).  Slots summing several members are the
// adjoint contractions of a shared operand.
//
// Tiling: 128 x 128 output tile per block of 4 waves, each wave 64 x 64 as
// 4 x 4 tiles of v_mfma_f32_16x16x4_f32; K staged 16 deep in LDS with register
// prefetch of the next stage.  Blocks are ordered so that the tiles one XCD
// processes form a compact band (its L2 keeps the shared A and B panels).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace bes {

namespace {

constexpr int BM = 128, BN = 128, BK = 16;
constexpr int LDA = BM + 4;   // LDS row pitch (floats) of As[k][m]
constexpr int LDB = BN + 4;   // LDS row pitch (floats) of Bs[k][n]

typedef float floatx4 __attribute__((ext_vector_type(4)));

// One K stage of the A tile (BM x BK) into registers, 2 x float4 per thread.
// kcontig: A[m][k..k+3] contiguous (sak == 1); else mcontig: A[m..m+3][k]
// contiguous (sam == 1); otherwise element-wise.
struct TileRegs {
  floatx4 v[2];
};

__device__ __forceinline__ void load_a(const MfmaMember &mb, int64_t m0, int64_t k0, int t,
                                       TileRegs &r) {
  const float *__restrict__ A = mb.A;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int f = t + 256 * h;  // 512 float4 per tile
    if (mb.sak == 1) {
      const int m = f >> 2, q = f & 3;
      const float *p = A + (m0 + m) * mb.sam + k0 + 4 * q;
      r.v[h] = *(const floatx4 *)p;
    } else if (mb.sam == 1) {
      const int k = f >> 5, q = f & 31;
      const float *p = A + (k0 + k) * mb.sak + m0 + 4 * q;
      r.v[h] = *(const floatx4 *)p;
    } else {
      const int m = f >> 2, q = f & 3;
#pragma unroll
      for (int c = 0; c < 4; ++c) r.v[h][c] = A[(m0 + m) * mb.sam + (k0 + 4 * q + c) * mb.sak];
    }
  }
}

__device__ __forceinline__ void store_a(float *__restrict__ As, const MfmaMember &mb, int t,
                                        const TileRegs &r) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int f = t + 256 * h;
    if (mb.sam == 1 && mb.sak != 1) {
      const int k = f >> 5, q = f & 31;
      *(floatx4 *)&As[k * LDA + 4 * q] = r.v[h];
    } else {
      const int m = f >> 2, q = f & 3;
#pragma unroll
      for (int c = 0; c < 4; ++c) As[(4 * q + c) * LDA + m] = r.v[h][c];
    }
  }
}

__device__ __forceinline__ void load_b(const MfmaMember &mb, int64_t n0, int64_t k0, int t,
                                       TileRegs &r) {
  const float *__restrict__ B = mb.B;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int f = t + 256 * h;
    if (mb.sbn == 1) {
      const int k = f >> 5, q = f & 31;
      const float *p = B + (k0 + k) * mb.sbk + n0 + 4 * q;
      r.v[h] = *(const floatx4 *)p;
    } else if (mb.sbk == 1) {
      const int n = f >> 2, q = f & 3;
      const float *p = B + (n0 + n) * mb.sbn + k0 + 4 * q;
      r.v[h] = *(const floatx4 *)p;
    } else {
      const int k = f >> 5, q = f & 31;
#pragma unroll
      for (int c = 0; c < 4; ++c) r.v[h][c] = B[(k0 + k) * mb.sbk + (n0 + 4 * q + c) * mb.sbn];
    }
  }
}

__device__ __forceinline__ void store_b(float *__restrict__ Bs, const MfmaMember &mb, int t,
                                        const TileRegs &r) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int f = t + 256 * h;
    if (mb.sbk == 1 && mb.sbn != 1) {
      const int n = f >> 2, q = f & 3;
#pragma unroll
      for (int c = 0; c < 4; ++c) Bs[(4 * q + c) * LDB + n] = r.v[h][c];
    } else {
      const int k = f >> 5, q = f & 31;
      *(floatx4 *)&Bs[k * LDB + 4 * q] = r.v[h];
    }
  }
}

__global__ void __launch_bounds__(256) mfma_gemm_kernel(const MfmaArgs a, int tiles_m,
                                                        int tiles_n) {
  __shared__ float As[2][BK * LDA];
  __shared__ float Bs[2][BK * LDB];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // XCD-aware order: blocks are dealt round-robin to the 8 XCDs; give each
  // XCD a contiguous range of logical tiles.
  const int tiles = tiles_m * tiles_n;
  const int per_slot = tiles;
  int bid = blockIdx.x;
  const int slot = bid / per_slot;
  bid -= slot * per_slot;
  int logical = bid;
  if (per_slot % 8 == 0) logical = (bid % 8) * (per_slot / 8) + bid / 8;
  const int tm = logical / tiles_n, tn = logical - tm * tiles_n;
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const MfmaSlot &S = a.slot[slot];

  floatx4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int64_t kt = a.K / BK;
  const int64_t steps = kt * (S.m1 - S.m0);
  TileRegs ra, rb;
  {
    const MfmaMember &mb = a.mem[S.m0];
    load_a(mb, m0, 0, t, ra);
    load_b(mb, n0, 0, t, rb);
    store_a(As[0], mb, t, ra);
    store_b(Bs[0], mb, t, rb);
  }
  __syncthreads();
  for (int64_t s = 0; s < steps; ++s) {
    const int buf = (int)(s & 1);
    const bool more = s + 1 < steps;
    int nm = 0;
    int64_t nk0 = 0;
    if (more) {
      nm = S.m0 + (int)((s + 1) / kt);
      nk0 = ((s + 1) % kt) * BK;
      load_a(a.mem[nm], m0, nk0, t, ra);
      load_b(a.mem[nm], n0, nk0, t, rb);
    }
    const float *__restrict__ as = As[buf];
    const float *__restrict__ bs = Bs[buf];
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      float fa[4], fb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) fa[i] = as[kr * LDA + wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) fb[j] = bs[kr * LDB + wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
    if (more) {
      store_a(As[buf ^ 1], a.mem[nm], t, ra);
      store_b(Bs[buf ^ 1], a.mem[nm], t, rb);
    }
    __syncthreads();
  }
  // D[i][j] of a 16x16 tile sits in lane j + 16 * (i / 4), register i % 4:
  // each lane holds 4 consecutive m of one n.  With C contiguous along m
  // (a permuted output layout) those 4 values are one 16-byte store.
  float *__restrict__ C = S.C;
  const bool vec_m = S.scm == 1 && (S.scn & 3) == 0 && ((uintptr_t)C & 15) == 0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t mb = m0 + wm * 64 + i * 16 + 4 * (lane >> 4);
      const int64_t n = n0 + wn * 64 + j * 16 + (lane & 15);
      if (vec_m) {
        floatx4 *p = (floatx4 *)(C + mb + n * S.scn);
        *p = S.acc ? *p + acc[i][j] : acc[i][j];
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          float *p = C + (mb + c) * S.scm + n * S.scn;
          *p = S.acc ? *p + acc[i][j][c] : acc[i][j][c];
        }
      }
    }
}

}  // namespace

bool mfma_shape_ok(int64_t M, int64_t N, int64_t K) {
  return M > 0 && N > 0 && K > 0 && M % BM == 0 && N % BN == 0 && K % BK == 0 &&
         (M / BM) * (N / BN) <= (1 << 24);
}

bool mfma_args_ok(const MfmaArgs &a) {
  if (!mfma_shape_ok(a.M, a.N, a.K) || a.n_slots < 1) return false;
  for (int m = 0; m < a.n_members; ++m) {
    const MfmaMember &mb = a.mem[m];
    // vector loads need 16-byte aligned rows along the contiguous direction
    if (mb.sak == 1 && (mb.sam % 4 || ((uintptr_t)mb.A & 15))) return false;
    if (mb.sak != 1 && mb.sam == 1 && (mb.sak % 4 || ((uintptr_t)mb.A & 15))) return false;
    if (mb.sbn == 1 && (mb.sbk % 4 || ((uintptr_t)mb.B & 15))) return false;
    if (mb.sbn != 1 && mb.sbk == 1 && (mb.sbn % 4 || ((uintptr_t)mb.B & 15))) return false;
  }
  return true;
}

hipError_t launch_mfma(const MfmaArgs &a, int /*tile_m*/, int /*tile_n*/, hipStream_t stream) {
  if (!mfma_args_ok(a)) return hipErrorInvalidValue;
  const int tm = (int)(a.M / BM), tn = (int)(a.N / BN);
  dim3 grid((unsigned)(tm * tn * a.n_slots));
  hipLaunchKernelGGL(mfma_gemm_kernel, grid, dim3(256), 0, stream, a, tm, tn);
  return hipGetLastError();
}

}  // namespace bes
