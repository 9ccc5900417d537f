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
// Tiling: an output tile per block of four waves (64 x 64, 64 x 64 with K
// staged 32 deep, 128 x 64, or a skinny 16 x 128, 32 x 128, 128 x 32 or
// 128 x 16 when the output has few rows or columns), each wave a grid of 16 x 16 MFMA tiles, K staged 8 or 16 deep
// through double-buffered LDS with register prefetch of the next stage.  FP64 runs v_mfma_f64_16x16x4f64,
// FP32 v_mfma_f32_16x16x4f32.  Each operand's tile is read along whichever
// of its two groups is contiguous in memory (host flag), so that neighbouring
// lanes read neighbouring addresses.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace bes {

namespace {

constexpr int kThreads = 256;
constexpr int kBM0 = 64, kBN0 = 64, kBK0 = 16;   // the square tile shape

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
template <int E>
struct Stage {
  int64_t o[E];      // element offsets (row + column), or -1 when out of range
};

template <typename T, int E>
__device__ __forceinline__ void gather(const T *__restrict__ base, const Stage<E> &s, T alpha,
                                       T beta, T (&v)[E]) {
#pragma unroll
  for (int q = 0; q < E; ++q) v[q] = s.o[q] >= 0 ? fma(alpha, base[s.o[q]], beta) : (T)0;
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

// Sum of the K ranges' partial tiles into C (overwriting, or adding into an
// accumulating slot); grid-stride over (slot, m, n).
template <typename T>
__global__ void __launch_bounds__(kThreads) gett_reduce_kernel(const GettArgs a) {
  const int64_t per = a.M * a.N, total = per * a.n_slots;
  const T *__restrict__ part = (const T *)a.partial;
  for (int64_t f = blockIdx.x * (int64_t)kThreads + threadIdx.x; f < total;
       f += (int64_t)gridDim.x * kThreads) {
    const int sl = (int)(f / per);
    const int64_t r = f - sl * per, m = r / a.N, n = r - m * a.N;
    T sum = 0;
    for (int k = 0; k < a.ksplit; ++k) sum += part[(int64_t)k * total + f];
    T *p = (T *)a.slot[sl].C + a.tab[a.slot[sl].rowC + m] + a.tab[a.slot[sl].colC + n];
    *p = a.slot[sl].acc ? *p + sum : sum;
  }
}

// Tile shapes: BM x BN outputs per block of four waves laid out WM x WN,
// each wave 16 TI x 16 TJ; K staged BK deep.  The skinny shapes serve
// contractions with few rows or columns (TCCG-like cases often have one
// small free side), where a square tile would be mostly padding.
template <int BM_, int BN_, int BK_, int WM_>
struct Tile {
  static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = 4 / WM_;
  static constexpr int TI = BM / (16 * WM), TJ = BN / (16 * WN);
  static constexpr int EA = BM * BK / kThreads, EB = BN * BK / kThreads;   // per thread
  static_assert(TI >= 1 && TJ >= 1 && EA >= 1 && EB >= 1, "tile shape");
};

template <typename T, typename TL>
__global__ void __launch_bounds__(kThreads) gett_kernel(const GettArgs a, int tiles_m,
                                                        int tiles_n) {
  typedef MatrixCore<T> MC;
  constexpr int BM = TL::BM, BN = TL::BN, BK = TL::BK, TI = TL::TI, TJ = TL::TJ;
  constexpr int EA = TL::EA, EB = TL::EB;
  constexpr int LDA = BM + 1, LDB = BN + 1;
  __shared__ T As[2][BK * LDA];
  __shared__ T Bs[2][BK * LDB];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave / TL::WN, wn = wave - wm * TL::WN;
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

  typename MC::acc_t acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = typename MC::acc_t{0, 0, 0, 0};

  // K stages [kb, ke) of every member of the slot belong to this block
  const int64_t ktot = (K + BK - 1) / BK;
  const int64_t kb = ktot * ks / a.ksplit, ke = ktot * (ks + 1) / a.ksplit;
  const int64_t kt = ke - kb;
  const int64_t steps = kt * (S.m1 - S.m0);

  // Element (row, kk) of this thread's q-th A value: along K (k-fast:
  // kk = t % BK, row = t / BK + (256 / BK) q) or along M (m-fast:
  // row = t % BM, kk = t / BM + (256 / BM) q); B likewise with N.
  auto a_row = [&](const GettMember &mb, int q) {
    return mb.a_kfast ? t / BK + (kThreads / BK) * q : t % BM;
  };
  auto a_kk = [&](const GettMember &mb, int q) {
    return mb.a_kfast ? t % BK : t / BM + (kThreads / BM) * q;
  };
  auto b_col = [&](const GettMember &mb, int q) {
    return mb.b_nfast ? t % BN : t / BK + (kThreads / BK) * q;
  };
  auto b_kk = [&](const GettMember &mb, int q) {
    return mb.b_nfast ? t / BN + (kThreads / BN) * q : t % BK;
  };
  // The M offsets of A's rows and the N offsets of B's columns that this
  // thread gathers do not change along K: looked up once per member (-1:
  // outside the output).  Only the K offsets are looked up per stage.
  int64_t rowoff[EA], coloff[EB];
  int cur = -1;
  auto member_offsets = [&](int mi) {
    if (mi == cur) return;
    cur = mi;
    const GettMember &mb = a.mem[mi];
#pragma unroll
    for (int q = 0; q < EA; ++q) {
      const int64_t m = m0 + a_row(mb, q);
      rowoff[q] = m < M ? tab[mb.rowA + m] : -1;
    }
#pragma unroll
    for (int q = 0; q < EB; ++q) {
      const int64_t n = n0 + b_col(mb, q);
      coloff[q] = n < N ? tab[mb.colB + n] : -1;
    }
  };
  auto stage_a = [&](const GettMember &mb, int64_t k0, Stage<EA> &s) {
    const int64_t *colA = tab + mb.colA;
#pragma unroll
    for (int q = 0; q < EA; ++q) {
      const int64_t k = k0 + a_kk(mb, q);
      s.o[q] = (k < K && rowoff[q] >= 0) ? rowoff[q] + colA[k] : -1;
    }
  };
  auto stage_b = [&](const GettMember &mb, int64_t k0, Stage<EB> &s) {
    const int64_t *rowB = tab + mb.rowB;
#pragma unroll
    for (int q = 0; q < EB; ++q) {
      const int64_t k = k0 + b_kk(mb, q);
      s.o[q] = (k < K && coloff[q] >= 0) ? rowB[k] + coloff[q] : -1;
    }
  };
  auto put_a = [&](T *__restrict__ dst, const GettMember &mb, const T (&v)[EA]) {
#pragma unroll
    for (int q = 0; q < EA; ++q) dst[a_kk(mb, q) * LDA + a_row(mb, q)] = v[q];
  };
  auto put_b = [&](T *__restrict__ dst, const GettMember &mb, const T (&v)[EB]) {
#pragma unroll
    for (int q = 0; q < EB; ++q) dst[b_kk(mb, q) * LDB + b_col(mb, q)] = v[q];
  };

  T va[EA], vb[EB];
  if (steps > 0) {
    member_offsets(S.m0);
    const GettMember &mb = a.mem[S.m0];
    Stage<EA> sa;
    Stage<EB> sb;
    stage_a(mb, kb * BK, sa);
    stage_b(mb, kb * BK, sb);
    gather<T, EA>((const T *)mb.A, sa, (T)mb.a_alpha, (T)mb.a_beta, va);
    gather<T, EB>((const T *)mb.B, sb, (T)mb.b_alpha, (T)mb.b_beta, vb);
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
      member_offsets(nm);
      const GettMember &mb = a.mem[nm];
      Stage<EA> sa;
      Stage<EB> sb;
      stage_a(mb, nk0, sa);
      stage_b(mb, nk0, sb);
      gather<T, EA>((const T *)mb.A, sa, (T)mb.a_alpha, (T)mb.a_beta, va);
      gather<T, EB>((const T *)mb.B, sb, (T)mb.b_alpha, (T)mb.b_beta, vb);
    }
    const T *__restrict__ as = As[buf];
    const T *__restrict__ bs = Bs[buf];
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      T fa[TI], fb[TJ];
#pragma unroll
      for (int i = 0; i < TI; ++i) fa[i] = as[kr * LDA + (wm * TI + i) * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < TJ; ++j) fb[j] = bs[kr * LDB + (wn * TJ + j) * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) acc[i][j] = MC::mma(fa[i], fb[j], acc[i][j]);
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
  for (int j = 0; j < TJ; ++j) {
    const int64_t n = n0 + (wn * TJ + j) * 16 + (lane & 15);
    if (n >= N) continue;
    const int64_t cn = colC[n];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = m0 + (wm * TI + i) * 16 + MC::row(v, lane);
        if (m >= M) continue;
        if (a.partial) {          // K split, summed by gett_reduce_kernel
          ((T *)a.partial)[((int64_t)ks * a.n_slots + sl) * M * N + m * N + n] = acc[i][j][v];
          continue;
        }
        T *p = C + rowC[m] + cn;
        if (a.ksplit > 1) atomicAdd(p, acc[i][j][v]);   // into zeroed or caller's C
        else *p = S.acc ? *p + acc[i][j][v] : acc[i][j][v];
      }
  }
}

template <typename T, typename TL>
hipError_t launch_tile(const GettArgs &args, int ksplit, void *ws, size_t ws_bytes,
                       hipStream_t stream) {
  GettArgs a = args;
  a.partial = nullptr;
  const int64_t tm = (a.M + TL::BM - 1) / TL::BM, tn = (a.N + TL::BN - 1) / TL::BN;
  const int64_t base = tm * tn * a.n_slots;
  const int64_t ktot = (a.K + TL::BK - 1) / TL::BK;
  // Split K when the output tiles alone cannot fill the chip: enough ranges
  // for about four blocks per compute unit, each at least eight K stages
  // (every range adds its partial tile atomically).  Skinny contractions
  // (a few dozen outputs along M or N, K in the tens of thousands) need
  // hundreds of ranges to stream their operands at full rate.
  if (ksplit <= 0) {
    const int64_t want = (4 * (int64_t)device_cu_count() + base - 1) / base;
    ksplit = (int)std::max<int64_t>(1, std::min<int64_t>({want, ktot / 8, 1024}));
  }
  a.ksplit = std::max(1, std::min<int>(ksplit, (int)std::max<int64_t>(ktot, 1)));
  const int64_t blocks = base * a.ksplit;
  if (tm * tn > (1 << 24) || blocks > 0x7fffffff) return hipErrorInvalidValue;
  const int64_t n = a.M * a.N * a.n_slots;
  const unsigned g = (unsigned)std::min<int64_t>((n + kThreads - 1) / kThreads, 8192);
  // Many ranges of few outputs: partial tiles to the workspace and a second
  // kernel sums them (atomic adds of hundreds of ranges into the same few
  // addresses serialize); otherwise they add atomically into the output.
  if (a.ksplit >= 8 && ws && (size_t)a.ksplit * (size_t)n * sizeof(T) <= ws_bytes)
    a.partial = ws;
  if (a.ksplit > 1 && !a.partial)
    hipLaunchKernelGGL(gett_zero_kernel<T>, dim3(g), dim3(kThreads), 0, stream, a);
  hipLaunchKernelGGL((gett_kernel<T, TL>), dim3((unsigned)blocks), dim3(kThreads), 0, stream, a,
                     (int)tm, (int)tn);
  if (a.partial) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gett_reduce_kernel<T>, dim3(g), dim3(kThreads), 0, stream, a);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_shape(const GettArgs &a, int shape, int ksplit, void *ws, size_t wsb,
                        hipStream_t stream) {
  switch (shape) {
    case 1: return launch_tile<T, Tile<16, 128, 16, 1>>(a, ksplit, ws, wsb, stream);
    case 2: return launch_tile<T, Tile<32, 128, 8, 1>>(a, ksplit, ws, wsb, stream);
    case 3: return launch_tile<T, Tile<128, 32, 8, 4>>(a, ksplit, ws, wsb, stream);
    case 4: return launch_tile<T, Tile<128, 16, 16, 4>>(a, ksplit, ws, wsb, stream);
    case 6: return launch_tile<T, Tile<64, 64, 32, 2>>(a, ksplit, ws, wsb, stream);
    case 7: return launch_tile<T, Tile<128, 64, 16, 2>>(a, ksplit, ws, wsb, stream);
    default: return launch_tile<T, Tile<kBM0, kBN0, kBK0, 2>>(a, ksplit, ws, wsb, stream);
  }
}

}  // namespace

hipError_t launch_gett(bool f64, const GettArgs &a, int shape, int ksplit, void *workspace,
                       size_t workspace_bytes, hipStream_t stream) {
  if (a.M <= 0 || a.N <= 0 || a.n_slots <= 0) return hipSuccess;
  // shape 0: by the output's extents -- skinny tiles for few rows or columns
  if (shape <= 0)
    shape = a.M <= 16 ? 1 : a.M <= 32 ? 2 : a.N <= 16 ? 4 : a.N <= 32 ? 3 : 5;
  return f64 ? launch_shape<double>(a, shape, ksplit, workspace, workspace_bytes, stream)
             : launch_shape<float>(a, shape, ksplit, workspace, workspace_bytes, stream);
}

}  // namespace bes
