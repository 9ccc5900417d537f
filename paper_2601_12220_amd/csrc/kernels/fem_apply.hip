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


// ---------------------------------------------------------------------------
// FP64 matrix-core variant (plain U): out[i, e] = sum_k S[i, k] W[k, e] with
// k = (c, j) runs as v_mfma_f64_16x16x4f64 blocks, M = 16 values of i, N = 16
// elements, K = 4 values of k; lane group q' = lane / 16 of the K side takes
// k in [q' KQ, (q' + 1) KQ).  S sits in LDS once per block as A fragments.
// Per unit of 16 elements a wave stages the geometry terms G[x, c, e] (once
// per unit, shared by the members) and, per member, U's NP planes (each a
// contiguous block of 16 x NJ values) through its LDS area with 16-byte
// loads, forms W[k][n] there (one value per lane and pass, all 64 lanes
// busy), reads its B fragments, runs the MB x KQ matrix instructions and
// writes the unit's output block [n][i] through LDS.  A partial last unit
// takes guarded scalar accesses.
// ---------------------------------------------------------------------------
typedef double d4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

template <int NI, int NJ, int NC, int NX, bool DIAG>
struct ApplyMfma {
  static constexpr int kU = 16;                            // elements per unit
  static constexpr int kNP = DIAG ? NC : NX;               // planes of U
  static constexpr int kNG = DIAG ? NC : NX * NC;          // geometry values per element
  static constexpr int kK = NC * NJ;                       // contracted (c, j)
  static constexpr int kKQ = (kK + 3) / 4;                 // K blocks
  static constexpr int kMB = (NI + 15) / 16;               // 16-row M blocks
  static constexpr int kFrags = kMB * kKQ;
  static constexpr int kUB = kU * NJ;                      // values of one plane block
  static constexpr int kUArea = kNP * kUB;                 // >= kU * kK
  static constexpr int kArea1 = kUArea > kU * kK ? kUArea : kU * kK;   // U, then W
  static constexpr int kArea0 = kArea1 > kU * NI ? kArea1 : kU * NI;     // then out
  static constexpr int kArea = (kArea0 + 1) & ~1;          // 16-byte multiple
  static constexpr int kGArea = kNG * kU;
  static constexpr int kPerWave = kArea + ((kGArea + 1) & ~1);
  static constexpr int kLdsMax = 160 * 1024;
  static constexpr int kW0 = (kLdsMax - kFrags * 64 * 8) / (kPerWave * 8);
  static constexpr int kWaves = kW0 >= 8 ? 8 : (kW0 >= 4 ? 4 : (kW0 >= 2 ? 2 : 1));
  static constexpr int kWT = (kU * kK + 63) / 64;          // W values per lane
};

template <int NI, int NJ, int NC, int NX, bool DIAG>
__global__ void __launch_bounds__(512)
    fem_apply_mfma_kernel(const FemApplyArgs a, int64_t n_units) {
  using M = ApplyMfma<NI, NJ, NC, NX, DIAG>;
  __shared__ double Sf[M::kFrags * 64];
  __shared__ d2v Area2[M::kWaves * M::kPerWave / 2];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  double *const X = (double *)Area2 + wave * M::kPerWave;    // U planes, then W, then out
  d2v *const XV = Area2 + wave * (M::kPerWave / 2);
  double *const Gl = X + M::kArea;                            // [g][n]
  // S as A fragments: fragment (mb, kb), lane l holds S[i][k] for
  // i = 16 mb + l % 16 and k = (l / 16) KQ + kb, k = (c, j).
  {
    const double *__restrict__ S = (const double *)a.S;
    for (int f = threadIdx.x; f < M::kFrags * 64; f += 64 * M::kWaves) {
      const int frag = f >> 6, l = f & 63;
      const int mb = frag / M::kKQ, kb = frag - mb * M::kKQ;
      const int i = 16 * mb + (l & 15), k = (l >> 4) * M::kKQ + kb;
      const int c = k / NJ, j = k - c * NJ;
      Sf[f] = (i < NI && k < M::kK) ? S[c * a.ss[0] + i * a.ss[1] + j * a.ss[2]] : 0.0;
    }
    __syncthreads();
  }
  const int n = lane & 15, q = lane >> 4;
  const double *__restrict__ Gp = (const double *)a.G;
  for (int64_t un = (int64_t)blockIdx.x * M::kWaves + wave; un < n_units;
       un += (int64_t)gridDim.x * M::kWaves) {
    const int64_t e0 = un * M::kU;
    const int n_el = (int)min((int64_t)M::kU, a.E - e0);
    const bool full = n_el == M::kU;
    // ---- geometry terms of the unit's elements: Gl[g][n] -------------------
#pragma unroll
    for (int t = 0; t < (M::kGArea + 63) / 64; ++t) {
      const int f = lane + 64 * t;
      const int g = f >> 4, el = f & 15;
      if (f < M::kGArea) {
        const int x = DIAG ? 0 : g / NC, c = DIAG ? g : g - (g / NC) * NC;
        Gl[f] = el < n_el ? Gp[x * a.gs[0] + c * a.gs[1] + (e0 + el) * a.gs[2]] : 0.0;
      }
    }
    // U planes of the next member of the unit, loaded into registers while
    // the current member computes (shapes whose planes take at most twelve
    // 16-byte values per lane)
    constexpr int kUT = (M::kUB / 2 + 63) / 64;
    constexpr bool PF = M::kNP * kUT <= 12;
    d2v pre[PF ? M::kNP : 1][PF ? kUT : 1];
    auto load_planes = [&](const FemApplyMember &Mn, d2v (&dst)[PF ? M::kNP : 1][PF ? kUT : 1]) {
      const double *__restrict__ Un = (const double *)Mn.u0 + Mn.uoff0 + e0 * NJ;
#pragma unroll
      for (int p = 0; p < (PF ? M::kNP : 1); ++p) {
        const d2v *__restrict__ pu = (const d2v *)(Un + p * Mn.us0[0]);
#pragma unroll
        for (int t = 0; t < (PF ? kUT : 1); ++t) {
          int qv = lane + 64 * t;
          if ((t + 1) * 64 > M::kUB / 2) qv = qv < M::kUB / 2 ? qv : M::kUB / 2 - 1;
          dst[p][t] = __builtin_nontemporal_load(&pu[qv]);
        }
      }
    };
    bool have_pre = false;
    for (int m = 0; m < a.n_members; ++m) {
      const FemApplyMember &Mb = a.mem[m];
      const double *__restrict__ U0 = (const double *)Mb.u0 + Mb.uoff0 + e0 * NJ;
      // ---- U planes into X[p][el * NJ + j] ---------------------------------
      if (full && PF && have_pre) {
#pragma unroll
        for (int p = 0; p < (PF ? M::kNP : 1); ++p)
#pragma unroll
          for (int t = 0; t < (PF ? kUT : 1); ++t) {
            const int qv = lane + 64 * t;
            if ((t + 1) * 64 <= M::kUB / 2 || qv < M::kUB / 2) XV[(p * M::kUB) / 2 + qv] = pre[p][t];
          }
      } else if (full) {
#pragma unroll
        for (int p = 0; p < M::kNP; ++p) {
          const d2v *__restrict__ pu = (const d2v *)(U0 + p * Mb.us0[0]);
#pragma unroll
          for (int t = 0; t < (M::kUB / 2 + 63) / 64; ++t) {
            const int qv = lane + 64 * t;
            if ((t + 1) * 64 <= M::kUB / 2 || qv < M::kUB / 2)
              XV[(p * M::kUB) / 2 + qv] = __builtin_nontemporal_load(&pu[qv]);
          }
        }
      } else {
#pragma unroll
        for (int p = 0; p < M::kNP; ++p)
          for (int f = lane; f < M::kUB; f += 64)
            X[p * M::kUB + f] = f < n_el * NJ ? U0[p * Mb.us0[0] + f] : 0.0;
      }
      wave_sync();
      have_pre = false;
      if constexpr (PF) {
        if (full && m + 1 < a.n_members) {
          load_planes(a.mem[m + 1], pre);
          have_pre = true;
        }
      }
      // ---- W[k][n] = sum_x G[x][c][n] U[x][n][j] (face mass: G[c][n] U[c][n][j])
      double wv[M::kWT];
#pragma unroll
      for (int t = 0; t < M::kWT; ++t) {
        const int f = lane + 64 * t;
        const int k = f >> 4, el = f & 15;
        const int c = k / NJ, j = k - c * NJ;
        double w = 0.0;
        if (f < M::kU * M::kK) {
          if constexpr (DIAG) {
            w = Gl[c * M::kU + el] * X[c * M::kUB + el * NJ + j];
          } else {
#pragma unroll
            for (int x = 0; x < NX; ++x)
              w = fma(Gl[(x * NC + c) * M::kU + el], X[x * M::kUB + el * NJ + j], w);
          }
        }
        wv[t] = w;
      }
      wave_sync();
#pragma unroll
      for (int t = 0; t < M::kWT; ++t) {
        const int f = lane + 64 * t;
        if (f < M::kU * M::kK) X[f] = wv[t];
      }
      wave_sync();
      double bf[M::kKQ];
#pragma unroll
      for (int kb = 0; kb < M::kKQ; ++kb) {
        const int k = q * M::kKQ + kb;
        bf[kb] = k < M::kK ? X[k * M::kU + n] : 0.0;
      }
      wave_sync();
      // ---- out[i][n] on the matrix cores ----------------------------------
      d4v acc[M::kMB];
#pragma unroll
      for (int mb = 0; mb < M::kMB; ++mb) acc[mb] = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kb = 0; kb < M::kKQ; ++kb)
#pragma unroll
        for (int mb = 0; mb < M::kMB; ++mb)
          acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(Sf[(mb * M::kKQ + kb) * 64 + lane],
                                                         bf[kb], acc[mb], 0, 0, 0);
      // ---- output block: item v of block mb is i = 16 mb + 4 v + q --------
      double *__restrict__ out = (double *)Mb.out;
      if (full && Mb.oe == NI && Mb.oi == 1 && ((uintptr_t)out & 15) == 0) {
#pragma unroll
        for (int mb = 0; mb < M::kMB; ++mb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = 16 * mb + 4 * v + q;
            if (i < NI) X[n * NI + i] = acc[mb][v];
          }
        wave_sync();
        d2v *__restrict__ ov = (d2v *)(out + e0 * NI);
#pragma unroll
        for (int t = 0; t < (M::kU * NI / 2 + 63) / 64; ++t) {
          const int qv = lane + 64 * t;
          if ((t + 1) * 64 <= M::kU * NI / 2 || qv < M::kU * NI / 2) {
            const d2v vv = XV[qv];
            __builtin_nontemporal_store(vv, &ov[qv]);
          }
        }
      } else {
#pragma unroll
        for (int mb = 0; mb < M::kMB; ++mb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = 16 * mb + 4 * v + q;
            if (i < NI && n < n_el) out[(e0 + n) * Mb.oe + i * Mb.oi] = acc[mb][v];
          }
      }
      wave_sync();
    }
  }
}

// The matrix-core variant takes plain U whose element rows are contiguous
// (j stride 1, element stride NJ) and 16-byte aligned per plane.
bool apply_mfma_ok(const FemApplyArgs &a, int NJ) {
  if (a.u_kind != FEM_SRC_ARRAY) return false;
  for (int m = 0; m < a.n_members; ++m) {
    const FemApplyMember &M = a.mem[m];
    if (M.us0[2] != 1 || M.us0[1] != NJ || (M.us0[0] & 1)) return false;
    if ((((uintptr_t)M.u0 + (uintptr_t)(M.uoff0 * 8)) & 15) != 0) return false;
  }
  return true;
}

template <int NI, int NJ, int NC, int NX, bool DIAG>
hipError_t launch_apply_mfma_shape(const FemApplyArgs &a, int blocks_per_cu, hipStream_t stream) {
  using M = ApplyMfma<NI, NJ, NC, NX, DIAG>;
  const int64_t units = (a.E + M::kU - 1) / M::kU;
  const int64_t cap = (int64_t)device_cu_count() * std::max(1, blocks_per_cu);
  const int64_t blocks = std::min<int64_t>((units + M::kWaves - 1) / M::kWaves, cap);
  hipLaunchKernelGGL((fem_apply_mfma_kernel<NI, NJ, NC, NX, DIAG>), dim3((unsigned)blocks),
                     dim3(64 * M::kWaves), 0, stream, a, units);
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
  // most shapes; the tuner picks per shape); 3: S W on the FP64 matrix cores
  const bool sreg = variant == 2;
  if (variant == 3 && f64 && apply_mfma_ok(a, NJ)) {
    hipError_t em = hipSuccess;
    if (ev_start && (em = hipEventRecord(ev_start, stream)) != hipSuccess) return em;
    em = hipErrorInvalidValue;
#define BES_APPLY_MFMA_DISPATCH(ni, nj, nc, nx, dg)                                          \
    if (NI == ni && NJ == nj && NC == nc && NX == nx && diag == dg)                          \
      em = launch_apply_mfma_shape<ni, nj, nc, nx, dg>(a, blocks_per_cu, stream);
    BES_FEM_APPLY_SHAPES(BES_APPLY_MFMA_DISPATCH)
#undef BES_APPLY_MFMA_DISPATCH
    if (em != hipSuccess) return em;
    if (ev_stop && (em = hipEventRecord(ev_stop, stream)) != hipSuccess) return em;
    return hipSuccess;
  }
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
