// GETT template for gfx950: any binary contraction on the matrix cores.
//
// A batched einsum whose members are pure two-operand contractions, with any
// grouping of the free and contracted indices and any strides (permuted
// views, transposed layouts -- the TCCG-style contractions of Section "TCCG
// Benchmark suite with Unmaterialized Operands"), evaluated as
//   C_s[M, N] (+)= sum_m sum_K (aA A_m[M, K] + bA) (aB B_m[K, N] + bB)
// without materializing a transposed or affine copy: every tile element is
// gathered through per-operand offset tables (address = row offset of its M
// or N multi-index + column offset of its K multi-index, both precomputed on
// the host), the affine map is applied in registers on the way to LDS, and
// out-of-range elements of ragged edge tiles enter as exact zeros.
//
// Tiling: 64 x 64 output tile per block of four waves (2 x 2, 32 x 32 each as
// 2 x 2 MFMA tiles of 16 x 16), K staged 16 deep through double-buffered LDS
// with register prefetch of the next stage.  FP64 runs v_mfma_f64_16x16x4f64,
// FP32 v_mfma_f32_16x16x4f32.  Each operand's tile is read along whichever
// of its two groups is contiguous in memory (host flag), so that neighbouring
// lanes read neighbouring addresses.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace bes {

namespace {

constexpr int BM = 64, BN = 64, BK = 16;
constexpr int kThreads = 256;

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename T>
struct MatrixCore;

// v_mfma_f64_16x16x4f64: A[m][k] in lane m + 16 k, B[k][n] in lane n + 16 k,
// D[m][n] item v of lane l with m = 4 v + l / 16, n = l % 16.
template <>
struct MatrixCore<double> {
  typedef d4v acc_t;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int v, int lane) { return 4 * v + (lane >> 4); }
};

// v_mfma_f32_16x16x4f32: same A and B layouts, D[m][n] item v of lane l with
// m = 4 (l / 16) + v, n = l % 16.
template <>
struct MatrixCore<float> {
  typedef f4v acc_t;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int v, int lane) { return 4 * (lane >> 4) + v; }
};

// Gather of one K stage of a 64 x 16 operand tile into registers (4 values
// per thread).  `fast` = the tile is read along its 16-wide K side (A) or
// along its 64-wide side (B): the host picks the side with unit stride.
struct Stage {
  int64_t o[4];      // element offsets (row + column), or -1 when out of range
};

template <typename T>
__device__ __forceinline__ void gather(const T *__restrict__ base, const Stage &s, T alpha, T beta,
                                       T (&v)[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) v[q] = s.o[q] >= 0 ? fma(alpha, base[s.o[q]], beta) : (T)0;
}

// Zero the overwritten outputs of a split-K launch (its partial tiles add
// into them); grid-stride over (slot, m, n).
template <typename T>
__global__ void __launch_bounds__(kThreads) gett_zero_kernel(const GettArgs a) {
  const int64_t per = a.M * a.N, total = per * a.n_slots;
  for (int64_t f = blockIdx.x * (int64_t)kThreads + threadIdx.x; f < total;
       f += (int64_t)gridDim.x * kThreads) {
    const int sl = (int)(f / per);
    if (a.slot[sl].acc) continue;
    const int64_t r = f - sl * per, m = r / a.N, n = r - m * a.N;
    ((T *)a.slot[sl].C)[a.tab[a.slot[sl].rowC + m] + a.tab[a.slot[sl].colC + n]] = (T)0;
  }
}

template <typename T>
__global__ void __launch_bounds__(kThreads) gett_kernel(const GettArgs a, int tiles_m,
                                                        int tiles_n) {
  typedef MatrixCore<T> MC;
  constexpr int LDA = BM + 1, LDB = BN + 1;
  __shared__ T As[2][BK * LDA];
  __shared__ T Bs[2][BK * LDB];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // block = (slot, tile, K range), K range fastest; tiles are dealt so that
  // each of the 8 XCDs gets a contiguous band (its L2 holds the shared panels)
  const int tiles = tiles_m * tiles_n;
  const int ks = (int)(blockIdx.x % a.ksplit);
  int bid = (int)(blockIdx.x / a.ksplit);
  const int sl = bid / tiles;
  bid -= sl * tiles;
  const int logical = (tiles % 8 == 0) ? (bid % 8) * (tiles / 8) + bid / 8 : bid;
  const int tm = logical / tiles_n, tn = logical - tm * tiles_n;
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const GettSlot &S = a.slot[sl];
  const int64_t *__restrict__ tab = a.tab;
  const int64_t M = a.M, N = a.N, K = a.K;

  typename MC::acc_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = typename MC::acc_t{0, 0, 0, 0};

  // K stages [kb, ke) of every member of the slot belong to this block
  const int64_t ktot = (K + BK - 1) / BK;
  const int64_t kb = ktot * ks / a.ksplit, ke = ktot * (ks + 1) / a.ksplit;
  const int64_t kt = ke - kb;
  const int64_t steps = kt * (S.m1 - S.m0);

  // Offsets of this thread's 4 A values and 4 B values at K stage k0.
  auto stage_a = [&](const GettMember &mb, int64_t k0, Stage &s) {
    const int64_t *rowA = tab + mb.rowA, *colA = tab + mb.colA;
    if (mb.a_kfast) {            // kk = t % 16, m = t / 16 + 16 q
      const int64_t k = k0 + (t & 15);
      const int64_t ck = k < K ? colA[k] : 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t m = m0 + (t >> 4) + 16 * q;
        s.o[q] = (k < K && m < M) ? rowA[m] + ck : -1;
      }
    } else {                     // m = t % 64, kk = t / 64 + 4 q
      const int64_t m = m0 + (t & 63);
      const int64_t rm = m < M ? rowA[m] : 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t k = k0 + (t >> 6) + 4 * q;
        s.o[q] = (k < K && m < M) ? rm + colA[k] : -1;
      }
    }
  };
  auto stage_b = [&](const GettMember &mb, int64_t k0, Stage &s) {
    const int64_t *rowB = tab + mb.rowB, *colB = tab + mb.colB;
    if (mb.b_nfast) {            // n = t % 64, kk = t / 64 + 4 q
      const int64_t n = n0 + (t & 63);
      const int64_t cn = n < N ? colB[n] : 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t k = k0 + (t >> 6) + 4 * q;
        s.o[q] = (k < K && n < N) ? rowB[k] + cn : -1;
      }
    } else {                     // kk = t % 16, n = t / 16 + 16 q
      const int64_t k = k0 + (t & 15);
      const int64_t rk = k < K ? rowB[k] : 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t n = n0 + (t >> 4) + 16 * q;
        s.o[q] = (k < K && n < N) ? rk + colB[n] : -1;
      }
    }
  };
  auto put_a = [&](T *__restrict__ dst, const GettMember &mb, const T (&v)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int m = mb.a_kfast ? (t >> 4) + 16 * q : (t & 63);
      const int kk = mb.a_kfast ? (t & 15) : (t >> 6) + 4 * q;
      dst[kk * LDA + m] = v[q];
    }
  };
  auto put_b = [&](T *__restrict__ dst, const GettMember &mb, const T (&v)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int n = mb.b_nfast ? (t & 63) : (t >> 4) + 16 * q;
      const int kk = mb.b_nfast ? (t >> 6) + 4 * q : (t & 15);
      dst[kk * LDB + n] = v[q];
    }
  };

  T va[4], vb[4];
  if (steps > 0) {
    const GettMember &mb = a.mem[S.m0];
    Stage sa, sb;
    stage_a(mb, kb * BK, sa);
    stage_b(mb, kb * BK, sb);
    gather<T>((const T *)mb.A, sa, (T)mb.a_alpha, (T)mb.a_beta, va);
    gather<T>((const T *)mb.B, sb, (T)mb.b_alpha, (T)mb.b_beta, vb);
    put_a(As[0], mb, va);
    put_b(Bs[0], mb, vb);
  }
  __syncthreads();
  for (int64_t s = 0; s < steps; ++s) {
    const int buf = (int)(s & 1);
    const bool more = s + 1 < steps;
    int nm = 0;
    if (more) {
      nm = S.m0 + (int)((s + 1) / kt);
      const int64_t nk0 = (kb + (s + 1) % kt) * BK;
      const GettMember &mb = a.mem[nm];
      Stage sa, sb;
      stage_a(mb, nk0, sa);
      stage_b(mb, nk0, sb);
      gather<T>((const T *)mb.A, sa, (T)mb.a_alpha, (T)mb.a_beta, va);
      gather<T>((const T *)mb.B, sb, (T)mb.b_alpha, (T)mb.b_beta, vb);
    }
    const T *__restrict__ as = As[buf];
    const T *__restrict__ bs = Bs[buf];
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      T fa[2], fb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) fa[i] = as[kr * LDA + wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) fb[j] = bs[kr * LDB + wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = MC::mma(fa[i], fb[j], acc[i][j]);
    }
    if (more) {
      put_a(As[buf ^ 1], a.mem[nm], va);
      put_b(Bs[buf ^ 1], a.mem[nm], vb);
    }
    __syncthreads();
  }
  T *__restrict__ C = (T *)S.C;
  const int64_t *rowC = tab + S.rowC, *colC = tab + S.colC;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int64_t n = n0 + wn * 32 + j * 16 + (lane & 15);
    if (n >= N) continue;
    const int64_t cn = colC[n];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = m0 + wm * 32 + i * 16 + MC::row(v, lane);
        if (m >= M) continue;
        T *p = C + rowC[m] + cn;
        if (a.ksplit > 1) atomicAdd(p, acc[i][j][v]);   // into zeroed or caller's C
        else *p = S.acc ? *p + acc[i][j][v] : acc[i][j][v];
      }
  }
}

}  // namespace

hipError_t launch_gett(bool f64, const GettArgs &args, int ksplit, hipStream_t stream) {
  if (args.M <= 0 || args.N <= 0 || args.n_slots <= 0) return hipSuccess;
  GettArgs a = args;
  const int64_t tm = (a.M + BM - 1) / BM, tn = (a.N + BN - 1) / BN;
  const int64_t base = tm * tn * a.n_slots;
  const int64_t ktot = (a.K + BK - 1) / BK;
  // Split K when the output tiles alone cannot fill the chip: enough ranges
  // for about four blocks per compute unit, each at least four K stages.
  if (ksplit <= 0) {
    const int64_t want = (4 * (int64_t)device_cu_count() + base - 1) / base;
    ksplit = (int)std::max<int64_t>(1, std::min<int64_t>({want, ktot / 4, 256}));
  }
  a.ksplit = std::max(1, std::min<int>(ksplit, (int)std::max<int64_t>(ktot, 1)));
  const int64_t blocks = base * a.ksplit;
  if (tm * tn > (1 << 24) || blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (a.ksplit > 1) {
    const int64_t n = a.M * a.N * a.n_slots;
    const unsigned g = (unsigned)std::min<int64_t>((n + kThreads - 1) / kThreads, 8192);
    if (f64)
      hipLaunchKernelGGL(gett_zero_kernel<double>, dim3(g), dim3(kThreads), 0, stream, a);
    else
      hipLaunchKernelGGL(gett_zero_kernel<float>, dim3(g), dim3(kThreads), 0, stream, a);
  }
  if (f64)
    hipLaunchKernelGGL(gett_kernel<double>, dim3((unsigned)blocks), dim3(kThreads), 0, stream,
                       a, (int)tm, (int)tn);
  else
    hipLaunchKernelGGL(gett_kernel<float>, dim3((unsigned)blocks), dim3(kThreads), 0, stream,
                       a, (int)tm, (int)tn);
  return hipGetLastError();
}

}  // namespace bes
