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
// Mapping: one wave per block, a tile of 64 consecutive elements per wave,
// one element per lane.  Occupancy, not arithmetic, decides the speed of this
// HBM-bound stream, so every choice below keeps the per-wave footprint small:
//   * one LDS staging region X of max(NJ, 12, IC) rows x 65 (odd pitch) per
//     wave, reused in turn for the G row, the U rows and the output rows;
//   * per-element sources are read with coalesced loads (lane k reads flat
//     position k, k+64, ... of the tile's rows); the G loads and the U loads
//     of a tile are issued together so their HBM latencies overlap, and with
//     PF the raw loads of the next tile are issued before the current tile's
//     arithmetic (register double buffering);
//   * element-wise functional operands (alpha*op(S0)+beta+S1) are evaluated
//     in registers during the coalesced pass; the tetrahedron Jacobian is
//     formed from the staged vertex row, once per tile when every member
//     reads the same one;
//   * stage 1 runs over i-chunks of IC outputs: T[r][0..IC) lives in
//     registers, S is packed [r][j][i] so a chunk row S[r][j][i0..i0+IC) is a
//     contiguous wave-uniform run (scalar loads, scalar FMA operand);
//     u comes from LDS (IC == NI) or from registers (UREG, several chunks);
//   * stage 2 writes each (member, x, chunk) block to X and then to HBM as
//     runs of IC contiguous values per element.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../fem_shapes.h"
#include "kernels.h"
#include "../../../include/bes.h"

namespace bes {

namespace {

constexpr int kTile = 64;      // elements per wave tile = lanes per wave
constexpr int kPitch = kTile + 1;
constexpr int kMaxRow = 12;    // staged G row width (TET: 4 x 3 vertex coords)

// FP64 sin (shift 0) or cos (shift 1) for |x| < 2^20 with one polynomial:
// Cody-Waite reduction by pi, x = (k + shift/2) pi + r with |r| <= pi/2 (pi
// split in three parts, the first two with 33 significant bits, so that
// (k + 1/2) times them is exact for |k| < 2^19), then
// op(x) = (-1)^(k + shift) sin(r), sin(r) by its Taylor series to degree 21
// (truncation below 2e-18 on |r| <= pi/2): about 22 operations, every one
// of them on every lane (no data-dependent choice between two series).
// Callers check the range for the whole wave first.
__device__ __forceinline__ double sincos_small(double x, int shift) {
  const double h = 0.5 * shift;
  const double k = rint(fma(x, 0x1.45f306dc9c883p-2, -h));   // x / pi - h
  const double m = k + h;
  double r = fma(-m, 0x1.921fb54400000p+1, x);
  r = fma(-m, 0x1.0b4611a600000p-33, r);
  r = fma(-m, 0x1.3198a2e037073p-68, r);
  const double r2 = r * r;
  double p = 1.0 / 51090942171709440000.0;            //  1/21!
  p = fma(p, r2, -1.0 / 121645100408832000.0);        // -1/19!
  p = fma(p, r2, 1.0 / 355687428096000.0);            //  1/17!
  p = fma(p, r2, -1.0 / 1307674368000.0);             // -1/15!
  p = fma(p, r2, 1.0 / 6227020800.0);                 //  1/13!
  p = fma(p, r2, -1.0 / 39916800.0);                  // -1/11!
  p = fma(p, r2, 1.0 / 362880.0);                     //  1/9!
  p = fma(p, r2, -1.0 / 5040.0);                      // -1/7!
  p = fma(p, r2, 1.0 / 120.0);                        //  1/5!
  p = fma(p, r2, -1.0 / 6.0);                         // -1/3!
  const double sr = fma(r2 * p, r, r);
  const unsigned odd = (unsigned)((int)k + shift) & 1u;
  return __hiloint2double(__double2hiint(sr) ^ (int)(odd << 31), __double2loint(sr));
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

// Element-wise functional operand value alpha * op(v) + beta + w (inline: a
// call would make the caller save its live registers to scratch).
template <typename T>
__device__ __forceinline__ T elementwise_call(int op, T v, T alpha, T beta, T w) {
  return alpha * apply_op<T>(op, v) + beta + w;
}

// Position of component c (of W) of element el in a source whose element
// stride is se and whose component c = ca * DIV + cb sits at ca*sa + cb*sb.
template <int W, int DIV>
__device__ __forceinline__ int src_pos(int f, int se, int sa, int sb, int &el, int &c) {
  el = f / W;
  c = f - el * W;
  const int ca = c / DIV, cb = c - ca * DIV;
  return el * se + ca * sa + cb * sb;
}

// Raw coalesced loads of W components for the 64 elements of a full tile:
// v[k] holds flat position lane + 64 k of the tile's (element, component)
// block.  In-tile offsets are 32-bit element counts from a wave-uniform base
// (the planner guarantees they fit).
template <typename T, int W, int DIV>
__device__ __forceinline__ void load_rows(T (&v)[W], const T *__restrict__ p, int se, int sa,
                                          int sb, int lane) {
#pragma unroll
  for (int k = 0; k < W; ++k) {
    int el, c;
    v[k] = p[src_pos<W, DIV>(lane + kTile * k, se, sa, sb, el, c)];
  }
}

// Write raw loads (full tile) into X as [component][element].
template <typename T, int W>
__device__ __forceinline__ void put_rows(T *__restrict__ X, const T (&v)[W], int lane) {
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const int f = lane + kTile * k;
    const int el = f / W, c = f - el * W;
    X[c * kPitch + el] = v[k];
  }
}

// Partial tile (n < 64 elements) or a source that needs two buffers: rolled
// loop with the element-wise prologue applied per value.
template <typename T, int W, int DIV, bool EW>
__device__ __forceinline__ void stage_rows_rolled(T *__restrict__ X, const FemSrc &s, int64_t e0,
                                                  int n, int lane) {
  const T *__restrict__ p0 = (const T *)s.p0 + s.off0 + e0 * s.s0[0];
  const int se0 = (int)s.s0[0], a0 = (int)s.s0[1], b0 = (int)s.s0[2];
  const bool ew = EW && s.kind == FEM_SRC_ELEMENTWISE;
  const bool two = ew && s.p1 != nullptr;
  const T *__restrict__ p1 = two ? (const T *)s.p1 + s.off1 + e0 * s.s1[0] : p0;
  const int se1 = (int)s.s1[0], a1 = (int)s.s1[1], b1 = (int)s.s1[2];
  for (int f = lane; f < n * W; f += kTile) {
    int el, c;
    T v = p0[src_pos<W, DIV>(f, se0, a0, b0, el, c)];
    if constexpr (EW) {
      if (ew) {
        T w = (T)0;
        if (two) w = p1[src_pos<W, DIV>(f, se1, a1, b1, el, c)];
        v = elementwise_call<T>(s.op, v, (T)s.alpha, (T)s.beta, w);
      }
    }
    X[c * kPitch + el] = v;
  }
}

// Tetrahedron Jacobian of this lane's element from its staged vertex row
// (components vertex * 3 + coordinate): J[x][r] = V[r+1][x] - V[0][x]; the
// kernel's (x, r) may be the operand's (r, x).  NX = NR = 3 on this path.
// Staged rows are P apart.
template <typename T, int NX, int NR, int P = kPitch>
__device__ __forceinline__ void tet_from_lds(const T *__restrict__ X, int lane, bool swapped,
                                             T (&g)[NX][NR]) {
  T v[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) v[k][c] = X[(k * 3 + c) * P + lane];
#pragma unroll
  for (int x = 0; x < NX; ++x)
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const T jxr = v[(r + 1) & 3][x % 3] - v[0][x % 3];
      const T jrx = v[(x + 1) & 3][r % 3] - v[0][r % 3];
      g[x][r] = swapped ? jrx : jxr;
    }
}

template <int NX, int NR>
constexpr bool kTetCapable = NX == 3 && NR == 3;

// G components of member descriptor s from the staged row in X:
// views read (off0 + x*sx + r*sr) of the row, tetrahedra the 12 vertex
// coordinates.
template <typename T, int NX, int NR, int P = kPitch>
__device__ __forceinline__ void g_from_row(const T *__restrict__ X, const FemSrc &s, int lane,
                                           T (&g)[NX][NR]) {
  if (kTetCapable<NX, NR> && s.kind == FEM_SRC_TET) {
    if constexpr (kTetCapable<NX, NR>) tet_from_lds<T, NX, NR, P>(X, lane, s.s1[0] != 0, g);
  } else {
    const int off = (int)s.off0, sx = (int)s.s0[1], sr = (int)s.s0[2];
#pragma unroll
    for (int x = 0; x < NX; ++x)
#pragma unroll
      for (int r = 0; r < NR; ++r) g[x][r] = X[(off + x * sx + r * sr) * P + lane];
  }
}

struct Unit {
  int64_t tile;
  int g;
};

// A fresh copy of the lane id that the compiler cannot see through: address
// arithmetic derived from it is recomputed per work unit instead of being
// hoisted out of the tile loop and held in VGPRs for the whole kernel (which
// would cap occupancy at one wave per SIMD).
__device__ __forceinline__ int fresh_lane() {
  int l = (int)threadIdx.x & (kTile - 1);
  asm volatile("" : "+v"(l));
  return l;
}

// Coalesced raw loads of W components of the 64 elements of a full tile:
// v[k] = component c of element el for the flat position f = lane + 64 k,
// el = f / W, c = f % W.  Only components c < w are meaningful; the others
// re-read the tile's last meaningful value (clamped address) so the loads
// stay branch-free and in bounds.
//   dense: the tile's block is contiguous (element stride W, unit component
//   stride): base + f, immediate offsets.
template <typename T, int W>
__device__ __forceinline__ void load_block(T (&v)[W], const T *__restrict__ p, bool dense, int se,
                                           int sc, int w, int lane) {
  if (dense) {
#pragma unroll
    for (int k = 0; k < W; ++k) v[k] = p[lane + kTile * k];
  } else {
    const int lim = (kTile - 1) * se + (w - 1) * sc;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const int f = lane + kTile * k;
      const int el = f / W, c = f - el * W;
      const int pos = el * se + c * sc;
      v[k] = p[pos < lim ? pos : lim];
    }
  }
}

// Raw loads of a full tile into X as [component][element]; rows c >= w get
// the meaningless values (X always has at least W rows).
template <typename T, int W>
__device__ __forceinline__ void put_block(T *__restrict__ X, const T (&v)[W], int lane) {
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const int f = lane + kTile * k;
    const int el = f / W, c = f - el * W;
    X[c * kPitch + el] = v[k];
  }
}

// 16-byte vector accesses of a dense tile block of W values per element:
// lane k moves the kV consecutive values at flat positions
// kV * (k + 64 t) + s, s < kV, for t < kVT<W> (the last t may be partly past
// the block: those lanes re-read the block's last vector and are not used).
template <typename T, int W>
struct Dense {
  static constexpr int kV = 16 / (int)sizeof(T);                 // values per vector
  static constexpr int kN = W * kTile / kV;                       // vectors in the block
  static constexpr int kVT = (kN + kTile - 1) / kTile;            // vectors per lane
  static constexpr int kLen = kVT * kV;                           // values per lane
};

template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
  typedef double __attribute__((ext_vector_type(2))) type;
};
template <>
struct Vec16<float> {
  typedef float __attribute__((ext_vector_type(4))) type;
};

template <typename T, int W>
__device__ __forceinline__ void load_dense(T *v, const T *__restrict__ p,
                                           int lane) {
  using D = Dense<T, W>;
  using V = typename Vec16<T>::type;
  const V *__restrict__ pv = (const V *)p;
#pragma unroll
  for (int t = 0; t < D::kVT; ++t) {
    int q = lane + kTile * t;
    if ((t + 1) * kTile > D::kN) q = q < D::kN ? q : D::kN - 1;
    const V x = __builtin_nontemporal_load(&pv[q]);   // streamed once
#pragma unroll
    for (int s = 0; s < D::kV; ++s) v[t * D::kV + s] = x[s];
  }
}

template <typename T, int W>
__device__ __forceinline__ void put_dense(T *__restrict__ X, const T *v,
                                          int lane) {
  using D = Dense<T, W>;
#pragma unroll
  for (int t = 0; t < D::kVT; ++t)
#pragma unroll
    for (int s = 0; s < D::kV; ++s) {
      const int f = D::kV * (lane + kTile * t) + s;
      const int el = f / W, c = f - el * W;
      if ((t + 1) * kTile <= D::kN || f < W * kTile) X[c * kPitch + el] = v[t * D::kV + s];
    }
}

template <typename T, int NI, int NJ, int NR, int NX, int MPG, int IC, bool EW, bool FAST>
struct Fem {
  static constexpr int kRows = (NJ > kMaxRow ? (NJ > IC ? NJ : IC) : (kMaxRow > IC ? kMaxRow : IC));
  static constexpr int kChunks = (NI + IC - 1) / IC;
};

// Waves per SIMD the register allocation of an instantiation must allow
// (the compiler otherwise spreads a kernel over VGPRs and AGPRs and ends at
// one wave per SIMD): accumulators T[NR][IC], G of MPG members and u, in
// 32-bit registers, plus a margin.
template <typename T, int NI, int NJ, int NR, int NX, int MPG, int IC>
constexpr int kWaves() {
  constexpr int w = (int)sizeof(T) / 4;
  constexpr int live = w * (NR * IC + MPG * NX * NR + (IC < NI ? NJ : 0)) + 48;
  constexpr int waves = 512 / live;
  return waves < 1 ? 1 : (waves > 8 ? 8 : waves);
}

// The stream kernel.  FAST instantiations contain only the straight-line
// full-tile code: every tile they visit holds 64 elements, U rows are dense,
// G arrives through a shared row (or is absent) and outputs are dense -- the
// launcher checks all of it and sends the rest (the last partial tile, other
// layouts) to the general instantiation.  Keeping the rolled paths out of the
// FAST code matters for more than size: the compiler's memory-counter waits
// merge over all paths of the loop, and with them present it made each tile
// wait for the previous tile's stores before loading.
//
// WPB > 1 (shapes whose S outgrows the scalar data cache): a block of WPB
// waves, one 64-element tile each, with its own staging region.  The waves of
// a block pass the same barriers, so they walk S together and share each
// chunk of it in the scalar cache instead of each thrashing its own.
template <typename T, int NI, int NJ, int NR, int NX, int MPG, int IC, bool EW, bool FAST,
          int WPB>
__global__ void __launch_bounds__(kTile * WPB)
    __attribute__((amdgpu_waves_per_eu(kWaves<T, NI, NJ, NR, NX, MPG, IC>())))
    fem_stream_kernel(const FemArgs a, const T *__restrict__ Spack) {
  using F = Fem<T, NI, NJ, NR, NX, MPG, IC, EW, FAST>;
  static_assert(FAST || WPB == 1, "partial tiles run one wave per block");
  __shared__ T Xall[WPB * F::kRows * kPitch];
  const int wave = WPB > 1 ? __builtin_amdgcn_readfirstlane((int)threadIdx.x / kTile) : 0;
  T *const X = Xall + wave * F::kRows * kPitch;
  const int64_t tile_end = a.tile1;
  const int n_groups = a.n_groups;

  // Shared-row width of a unit: g_same plans stage one row per tile (at the
  // tile's first group), other plans one row per group.
  auto row_of = [&](int g) -> int {
    if (a.g_same) return g == 0 ? a.grp[0].g_row : 0;
    return a.grp[g].g_row;
  };

  T gm[MPG][NX][NR];   // G of the group's members (or of the plan, g_same)

  Unit cur{a.tile0 + (int64_t)blockIdx.x * WPB, 0};
  while (cur.tile < tile_end) {
    int lane = fresh_lane();
    // This wave's tile; a wave past the end repeats the last tile's work
    // (valid addresses, same barriers) and stores nothing.
    const int64_t mine = cur.tile + wave;
    const bool live = WPB == 1 || mine < tile_end;
    const int64_t e0 = (live ? mine : tile_end - 1) * kTile;
    const int n = FAST ? kTile : (int)(a.E - e0 < kTile ? a.E - e0 : kTile);
    const bool full = FAST || n == kTile;
    const FemGroup &G = a.grp[cur.g];
    const int m0 = G.m0, nm = G.m1 - G.m0;
    const bool has_g = a.mem[m0].g.kind != FEM_SRC_NONE;
    const int grow = has_g ? row_of(cur.g) : 0;
    const bool g_each = !FAST && has_g && G.g_row == 0 && !(a.g_same && cur.g > 0);
    const bool u_ew = EW && G.u.kind == FEM_SRC_ELEMENTWISE;

    // ---- raw loads: G row and U rows, all issued before any is used --------
    constexpr int kRU = FAST ? Dense<T, NJ>::kLen : NJ;
    T ru[kRU];
    T rg[kMaxRow];
    T rw[EW ? kRU : 1];
    if (full && grow > 0) {
      const FemSrc &s0 = a.mem[m0].g;
      const T *__restrict__ pb = (const T *)s0.p0 + G.g_off + e0 * s0.s0[0];
      load_block<T, kMaxRow>(rg, pb, false, (int)s0.s0[0], 1, grow, lane);
    }
    const bool u_fast = full && (FAST || G.u_dense);
    if (u_fast) {
      const T *__restrict__ p0 = (const T *)G.u.p0 + G.u.off0 + e0 * NJ;
      if constexpr (FAST) load_dense<T, NJ>(ru, p0, lane);
      else load_block<T, NJ>(ru, p0, true, NJ, 1, NJ, lane);
      if constexpr (EW) {
        if (u_ew && G.u.p1) {
          const T *__restrict__ p1 = (const T *)G.u.p1 + G.u.off1 + e0 * NJ;
          if constexpr (FAST) load_dense<T, NJ>(rw, p1, lane);
          else load_block<T, NJ>(rw, p1, true, NJ, 1, NJ, lane);
        } else {
#pragma unroll
          for (int k = 0; k < kRU; ++k) rw[k] = (T)0;
        }
      }
    }

    // ---- G to registers ---------------------------------------------------
    if (grow > 0) {
      if (full) {
        put_block<T, kMaxRow>(X, rg, lane);
      } else if constexpr (!FAST) {
        const FemSrc &s0 = a.mem[m0].g;
        const T *__restrict__ pb = (const T *)s0.p0 + G.g_off + e0 * s0.s0[0];
        const int se = (int)s0.s0[0];
        for (int f = lane; f < n * grow; f += kTile) {
          const int el = f / grow, c = f - el * grow;
          X[c * kPitch + el] = pb[el * se + c];
        }
      }
      __syncthreads();
      if (a.g_same) {
        g_from_row<T, NX, NR>(X, a.mem[0].g, lane, gm[0]);
      } else {
#pragma unroll
        for (int q = 0; q < MPG; ++q)
          if (q < nm) g_from_row<T, NX, NR>(X, a.mem[m0 + q].g, lane, gm[q]);
      }
      __syncthreads();
    } else if constexpr (!FAST) {
      if (g_each) {
        for (int q = 0; q < nm && q < MPG; ++q) {
          const FemSrc &s = a.mem[m0 + q].g;
          const bool tet = s.kind == FEM_SRC_TET;
          if (tet) {
            stage_rows_rolled<T, 12, 3, false>(X, s, e0, n, lane);
          } else {
            stage_rows_rolled<T, NX * NR, NR, EW>(X, s, e0, n, lane);
          }
          __syncthreads();
#pragma unroll
          for (int qq = 0; qq < MPG; ++qq) {
            if (qq != q) continue;
            if (kTetCapable<NX, NR> && tet) {
              if constexpr (kTetCapable<NX, NR>)
                tet_from_lds<T, NX, NR>(X, lane, s.s1[0] != 0, gm[qq]);
            } else {
#pragma unroll
              for (int x = 0; x < NX; ++x)
#pragma unroll
                for (int r = 0; r < NR; ++r) gm[qq][x][r] = X[(x * NR + r) * kPitch + lane];
            }
          }
          __syncthreads();
        }
      }
    }

    // ---- U rows into X (prologue applied) ---------------------------------
    if (u_fast) {
      if constexpr (EW) {
        if (u_ew) {
          const T alpha = (T)G.u.alpha, beta = (T)G.u.beta;
          const int op = G.u.op;
#pragma unroll
          for (int k = 0; k < kRU; ++k) ru[k] = alpha * apply_op<T>(op, ru[k]) + beta + rw[k];
        }
      }
      if constexpr (FAST) put_dense<T, NJ>(X, ru, lane);
      else put_block<T, NJ>(X, ru, lane);
    } else if constexpr (!FAST) {
      stage_rows_rolled<T, NJ, 1, EW>(X, G.u, e0, n, lane);  // U strides (e, j)
    }
    __syncthreads();

    // ---- next unit --------------------------------------------------------
    Unit nxt = cur;
    if (++nxt.g >= n_groups) {
      nxt.g = 0;
      nxt.tile += (int64_t)gridDim.x * WPB;
    }

    // ---- u into registers (chunked shapes); X is then free for outputs ----
    constexpr bool NAT = F::kChunks > 1;
    T ur[NAT ? NJ : 1];
    if constexpr (NAT) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) ur[j] = X[j * kPitch + lane];
      __syncthreads();
    }

    // S: chunked shapes read it in its natural [r][i][j] layout (the caller's
    // buffer when dense, else the packed copy); the others read the packed
    // [r][j][i] copy.
    const T *__restrict__ S = (NAT && G.s_dense) ? (const T *)G.S
                                                 : Spack + (int64_t)cur.g * NR * NI * NJ;
    bool o_fast = full;
    if constexpr (!FAST) {
#pragma unroll
      for (int q = 0; q < MPG; ++q)
        if (q < nm) o_fast = o_fast && a.mem[m0 + q].o_dense;
    }
    // Stage 2 and stores of one chunk [i0, i0 + cn) of T (cn <= IC), one
    // (member, x) block at a time through X.
    auto stage2_store = [&](const auto &t, int i0, int cn) {
      constexpr int W = sizeof(t[0]) / sizeof(T);
#pragma unroll
      for (int q = 0; q < MPG; ++q) {
        if (q >= nm) break;
        const FemMember &M = a.mem[m0 + q];
        const int gq = a.g_same ? 0 : q;
#pragma unroll
        for (int x = 0; x < NX; ++x) {
#pragma unroll
          for (int ic = 0; ic < W; ++ic) {
            T acc;
            if (has_g) {
              acc = gm[gq][x][0] * t[0][ic];
#pragma unroll
              for (int r = 1; r < NR; ++r) acc = fma(gm[gq][x][r], t[r][ic], acc);
            } else {
              acc = t[0][ic];
            }
            X[ic * kPitch + lane] = acc;
          }
          __syncthreads();
          if (FAST && NX == 1 && W == NI) {
            // Contiguous output block of 64 * NI values: 16-byte stores.
            using V = typename Vec16<T>::type;
            using D = Dense<T, NI>;
            V *__restrict__ ov = (V *)((T *)M.out + e0 * NI);
#pragma unroll
            for (int t = 0; t < D::kVT; ++t) {
              const int q = lane + kTile * t;
              V vv;
#pragma unroll
              for (int sv = 0; sv < D::kV; ++sv) {
                const int f = D::kV * q + sv;
                const int el = f / NI, ic = f - el * NI;
                vv[sv] = X[ic * kPitch + (el < kTile ? el : 0)];
              }
              // written once, never re-read here: streaming store
              if (live && ((t + 1) * kTile <= D::kN || q < D::kN))
                __builtin_nontemporal_store(vv, &ov[q]);
            }
          } else if (FAST || o_fast) {
            // Dense output [E][NX][NI]: the block is 64 runs of cn values,
            // one element every NX*NI (contiguous when cn == NI, NX == 1).
            T *__restrict__ ox = (T *)M.out + e0 * (NX * NI) + x * NI + i0;
#pragma unroll
            for (int k = 0; k < W; ++k) {
              const int f = lane + kTile * k;
              const int el = f / W, ic = f - el * W;
              const T val = X[ic * kPitch + el];
              if (live && (W == NI || ic < cn)) ox[el * (NX * NI) + ic] = val;
            }
          } else if constexpr (!FAST) {
            T *__restrict__ ox = (T *)M.out + e0 * M.oe + x * M.ox + (int64_t)i0 * M.oi;
            const int oe = (int)M.oe, oi = (int)M.oi;
            const int total = n * cn;
            for (int f = lane; f < total; f += kTile) {
              const int el = f / cn, ic = f - el * cn;
              ox[el * oe + ic * oi] = X[ic * kPitch + el];
            }
          }
          __syncthreads();
        }
      }
    };
    // Stage 1 over chunks of IC outputs (one chunk when T[NR][NI] fits):
    //   T[r][ic] = sum_j S[r][i0 + ic][j] u[j]
    // S in its natural [r][i][j] layout: a group of four accumulators walks
    // four contiguous S rows together, 8 values of each per scalar load, with
    // u in registers.  Rows past NI (the last chunk's padding) re-read row
    // NI - 1; their results are never stored.  One loop body for all chunks,
    // so nothing is hoisted from one chunk into the next.
    if constexpr (NAT) {
#pragma unroll 1
    for (int ch = 0; ch < F::kChunks; ++ch) {
      const int i0 = ch * IC;
      if (F::kChunks > 1) lane = fresh_lane();
      T t[NR][IC];
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int ic = 0; ic < IC; ++ic) t[r][ic] = 0;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
#pragma unroll
        for (int g4 = 0; g4 < (IC + 3) / 4; ++g4) {
          const T *__restrict__ rows[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            int i = i0 + g4 * 4 + q;
            i = i < NI ? i : NI - 1;
            rows[q] = S + ((int64_t)r * NI + i) * NJ;
          }
#pragma unroll
          for (int jb = 0; jb < NJ; jb += 8)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int ic = g4 * 4 + q;
              if (ic < IC) {
#pragma unroll
                for (int jj = 0; jj < 8; ++jj)
                  if (jb + jj < NJ) t[r][ic] = fma(rows[q][jb + jj], ur[NAT ? jb + jj : 0], t[r][ic]);
              }
            }
        }
      }
      const int ic_n = NI - i0 < IC ? NI - i0 : IC;
      stage2_store(t, i0, ic_n);
    }
    } else {
      // One chunk: T[r][i] = sum_j S[r][j][i] u[j] with S packed [r][j][i],
      // a row of NI wave-uniform values per (r, j), u read from LDS.
      T t[NR][NI];
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int ic = 0; ic < NI; ++ic) t[r][ic] = 0;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        // u is re-read from LDS for every r: a fresh address keeps the
        // compiler from caching all NJ values in registers across r.
        const int xl = fresh_lane();
#pragma unroll 2
        for (int j = 0; j < NJ; ++j) {
          const T uj = X[j * kPitch + xl];
          const T *__restrict__ Srow = S + ((int64_t)r * NJ + j) * NI;
#pragma unroll
          for (int ic = 0; ic < NI; ++ic) t[r][ic] = fma(Srow[ic], uj, t[r][ic]);
        }
      }
      __syncthreads();
      stage2_store(t, 0, NI);
    }
    cur = nxt;
  }
}

// S packed from the caller's strides into the layout the kernel reads:
// [group][r][j][i] (one-chunk shapes) or [group][r][i][j] (chunked shapes,
// only for groups whose S is not already dense in that order).
struct PackArgs {
  const void *S[BES_FEM_MAX_GROUPS];
  int64_t sr[BES_FEM_MAX_GROUPS], si[BES_FEM_MAX_GROUPS], sj[BES_FEM_MAX_GROUPS];
  int n_groups, NR, NI, NJ;
  int transposed;   // 1: [group][r][j][i]; 0: [group][r][i][j]
};

template <typename T>
__global__ void __launch_bounds__(256) pack_s_kernel(const PackArgs a, T *__restrict__ dst) {
  const int per = a.NR * a.NI * a.NJ;
  const int total = per * a.n_groups;
  for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < total; f += gridDim.x * blockDim.x) {
    const int g = f / per;
    int rem = f - g * per;
    const int r = rem / (a.NI * a.NJ);
    rem -= r * a.NI * a.NJ;
    int i, j;
    if (a.transposed) {
      j = rem / a.NI;
      i = rem - j * a.NI;
    } else {
      i = rem / a.NJ;
      j = rem - i * a.NJ;
    }
    if (a.S[g]) dst[f] = ((const T *)a.S[g])[r * a.sr[g] + i * a.si[g] + j * a.sj[g]];
  }
}

// i-chunk of the stage-1 accumulator: the whole T[NR][NI] when it fits in
// 120 VGPRs (u then stays in LDS), else as few equal chunks as keep each
// within 64 VGPRs (u and G are in registers too).
template <typename T, int NI, int NR>
constexpr int kChunksOf = (NR * NI * (int)sizeof(T) / 4 <= 120)
                              ? 1
                              : (NR * NI * (int)sizeof(T) / 4 + 63) / 64;
template <typename T, int NI, int NR>
constexpr int kIC = (NI + kChunksOf<T, NI, NR> - 1) / kChunksOf<T, NI, NR>;

// Stage-1 chunks of a shape (1: T in registers whole, u read from LDS).
int chunks_of(bool f64, int NI, int NR) {
  return f64 ? (NR * NI * 2 <= 120 ? 1 : (NR * NI * 2 + 63) / 64)
             : (NR * NI <= 120 ? 1 : (NR * NI + 63) / 64);
}

// Waves per block: one, unless S (read through the scalar data cache by every
// FMA of stage 1) is larger than about 12 KB; then eight waves (one block per
// compute unit at two waves per SIMD) share it.
template <typename T, int NI, int NJ, int NR>
constexpr int kWPB = (NR * NI * NJ * (int)sizeof(T) > 12 * 1024) ? 8 : 1;

// ---------------------------------------------------------------------------
// Lean instantiation for the plain FEM batch: one stage-1 group (all members
// share u and S), one output component per member, G absent or read by every
// member from one staged row per element (views of one buffer, such as the
// rows of a Jacobian), dense 16-byte-aligned operands, full tiles, T[NR][NI]
// in registers and S packed [r][j][i] within the scalar data cache.
//
// A 64-element tile is shared by WPT waves (one block): each wave loads and
// stores 1/WPT of the tile's rows and owns NI/WPT of the outputs i, so it
// keeps 1/WPT of T in registers.  Two waves per tile halve each wave's
// arithmetic phase and raise the waves resident per SIMD; while one of them
// computes, the others' loads and stores keep HBM busy (measured on the P3
// gradient batch: about 1.2x the bandwidth of one wave per tile).
//
// All that the tile loop addresses besides the tile index is fixed for the
// launch and arrives in a small argument block held in scalar registers: no
// descriptor reads sit between one tile's stores and the next tile's loads.
// S is a kernel argument of its own, restrict-qualified, so the compiler may
// read it with scalar loads across the kernel's stores (through a struct
// field it falls back to one vector load per lane).
// ---------------------------------------------------------------------------
struct LeanArgs {
  const void *u;        // dense [E][NJ], offset applied
  const void *grow;     // start of element 0's G row (null: no G)
  void *out[3];         // member outputs, dense [E][NI]
  int64_t tile0, tile1; // 64-element tiles [tile0, tile1), all full
  int32_t n_mem;        // members (<= MPG)
  int32_t g_w;          // G row width (<= kMaxRow; 0: no G)
  int32_t g_stride;     // element stride of the G row source
  int32_t g_off[3][3];  // row position of G[member][r] (unused members: 0)
};

template <typename T, int NI, int NJ, int NR>
constexpr bool kLeanShape = kChunksOf<T, NI, NR> == 1 && kWPB<T, NI, NJ, NR> == 1;

// Rows of S per scalar round trip of stage 1: 320 bytes of a wave's slice.
template <typename T, int IH, int NJ>
constexpr int kLeanUnrollJ = (320 / (IH * (int)sizeof(T))) < 1 ? 1
                             : (320 / (IH * (int)sizeof(T))) > NJ ? NJ
                                                                  : 320 / (IH * (int)sizeof(T));

// No occupancy attribute here: with one, the scheduler keeps SGPR use low and
// walks S through a single 16-SGPR window, one scalar round trip per 64 bytes
// of S; without, it batches 320 bytes per round trip.
template <typename T, int NI, int NJ, int NR, int MPG, int WPT>
__global__ void __launch_bounds__(kTile * WPT)
    fem_lean_kernel(const LeanArgs a, const T *__restrict__ S) {
  static_assert(kMaxRow % WPT == 0, "G row loads split evenly");
  constexpr int kR0 = NJ > NI ? NJ : NI;
  __shared__ T X[kR0 * kPitch];        // u rows, then one member's output rows
  __shared__ T GX[kMaxRow * kPitch];   // the staged G rows
  using V = typename Vec16<T>::type;
  using DU = Dense<T, NJ>;
  using DI = Dense<T, NI>;
  constexpr int kIH = (NI + WPT - 1) / WPT;        // outputs i per wave
  constexpr int kGK = kMaxRow / WPT;               // G-row loads per lane
  constexpr int kUK = (DU::kVT + WPT - 1) / WPT;   // u vectors per lane
  constexpr int kOK = (DI::kVT + WPT - 1) / WPT;   // output vectors per lane
  // shares that divide evenly need no per-wave bounds (kept compile-time)
  constexpr bool kUEven = DU::kVT % WPT == 0, kOEven = DI::kVT % WPT == 0;
  constexpr bool kIEven = NI % WPT == 0;
  const int w = WPT > 1 ? __builtin_amdgcn_readfirstlane((int)threadIdx.x / kTile) : 0;
  const bool has_g = a.g_w > 0;
  const int i0 = w * kIH;                          // this wave's first output i
  for (int64_t tile = a.tile0 + blockIdx.x; tile < a.tile1; tile += gridDim.x) {
    const int lane = fresh_lane();
    const int64_t e0 = tile * kTile;
    // raw loads, this wave's share: G rows (clamped, branch-free), u rows
    T rg[kGK];
    if (has_g) {
      const T *__restrict__ pg = (const T *)a.grow + e0 * a.g_stride;
      const int lim = (kTile - 1) * a.g_stride + a.g_w - 1;
#pragma unroll
      for (int k = 0; k < kGK; ++k) {
        const int f = lane + kTile * (k + w * kGK);
        const int el = f / kMaxRow, c = f - el * kMaxRow;
        const int pos = el * a.g_stride + c;
        rg[k] = pg[pos < lim ? pos : lim];
      }
    }
    T ru[kUK * DU::kV];
    {
      const V *__restrict__ pu = (const V *)((const T *)a.u + e0 * NJ);
#pragma unroll
      for (int k = 0; k < kUK; ++k) {
        const int t = k + w * kUK;
        int q = lane + kTile * t;
        if (!kUEven && t >= DU::kVT) q = DU::kN - 1;   // past the last share
        else if ((t + 1) * kTile > DU::kN) q = q < DU::kN ? q : DU::kN - 1;
        const V x = __builtin_nontemporal_load(&pu[q]);   // streamed once
#pragma unroll
        for (int sv = 0; sv < DU::kV; ++sv) ru[k * DU::kV + sv] = x[sv];
      }
    }
    // transposes into [component][element]
    if (has_g) {
#pragma unroll
      for (int k = 0; k < kGK; ++k) {
        const int f = lane + kTile * (k + w * kGK);
        const int el = f / kMaxRow, c = f - el * kMaxRow;
        GX[c * kPitch + el] = rg[k];
      }
    }
#pragma unroll
    for (int k = 0; k < kUK; ++k) {
      const int t = k + w * kUK;
#pragma unroll
      for (int sv = 0; sv < DU::kV; ++sv) {
        const int f = DU::kV * (lane + kTile * t) + sv;
        const int el = f / NJ, c = f - el * NJ;
        if ((kUEven || t < DU::kVT) && ((t + 1) * kTile <= DU::kN || f < NJ * kTile))
          X[c * kPitch + el] = ru[k * DU::kV + sv];
      }
    }
    __syncthreads();
    // G of this lane's element for every member
    T gm[MPG][NR];
    if (has_g) {
#pragma unroll
      for (int q = 0; q < MPG; ++q)
#pragma unroll
        for (int r = 0; r < NR; ++r) gm[q][r] = GX[a.g_off[q][r] * kPitch + lane];
    }
    // stage 1, this wave's outputs: T[r][ii] = sum_j S[r][j][i0 + ii] u[j]
    T t[NR][kIH];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int ii = 0; ii < kIH; ++ii) t[r][ii] = 0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int xl = fresh_lane();   // u re-read per r instead of pinned in VGPRs
#pragma unroll(kLeanUnrollJ<T, kIH, NJ>)
      for (int j = 0; j < NJ; ++j) {
        const T uj = X[j * kPitch + xl];
        const T *__restrict__ Srow = S + (r * NJ + j) * NI;
#pragma unroll
        for (int ii = 0; ii < kIH; ++ii) {
          // NI not a multiple of WPT: the last wave's extra output re-reads
          // the row's last value (never stored)
          const int i = kIEven ? i0 + ii : (i0 + ii < NI ? i0 + ii : NI - 1);
          t[r][ii] = fma(Srow[i], uj, t[r][ii]);
        }
      }
    }
    __syncthreads();
    // stage 2 per member, through X to 16-byte streaming stores
#pragma unroll
    for (int q = 0; q < MPG; ++q) {
      if (q >= a.n_mem) break;
#pragma unroll
      for (int ii = 0; ii < kIH; ++ii) {
        T acc = t[0][ii];
        if (has_g) {
          acc = gm[q][0] * t[0][ii];
#pragma unroll
          for (int r = 1; r < NR; ++r) acc = fma(gm[q][r], t[r][ii], acc);
        }
        if (kIEven || i0 + ii < NI) X[(i0 + ii) * kPitch + lane] = acc;
      }
      __syncthreads();
      V *__restrict__ ov = (V *)((T *)a.out[q] + e0 * NI);
#pragma unroll
      for (int k = 0; k < kOK; ++k) {
        const int tt = k + w * kOK;
        const int v = lane + kTile * tt;
        V vv;
#pragma unroll
        for (int sv = 0; sv < DI::kV; ++sv) {
          const int f = DI::kV * v + sv;
          const int el = f / NI, ic = f - el * NI;
          vv[sv] = X[ic * kPitch + (el < kTile ? el : 0)];
        }
        if ((kOEven || tt < DI::kVT) && ((tt + 1) * kTile <= DI::kN || v < DI::kN))
          __builtin_nontemporal_store(vv, &ov[v]);
      }
      __syncthreads();
    }
  }
}

template <typename T, int NI, int NJ, int NR>
hipError_t launch_lean(const LeanArgs &a, const T *spack, int mpg, int wpt, dim3 grid,
                       hipStream_t s) {
  if constexpr (kLeanShape<T, NI, NJ, NR>) {
#define BES_LEAN_LAUNCH(MPG, WPT)                                                         \
  hipLaunchKernelGGL((fem_lean_kernel<T, NI, NJ, NR, MPG, WPT>), grid, dim3(kTile * WPT), 0, s, \
                     a, spack)
    if (mpg == 1) {
      if (wpt == 2) BES_LEAN_LAUNCH(1, 2);
      else BES_LEAN_LAUNCH(1, 1);
    } else {
      if (wpt == 2) BES_LEAN_LAUNCH(3, 2);
      else BES_LEAN_LAUNCH(3, 1);
    }
#undef BES_LEAN_LAUNCH
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

bool lean_shape(bool f64, int NI, int NJ, int NR) {
  const int w = f64 ? 2 : 1;
  const bool one_chunk = NR * NI * w <= 120;
  const bool small_s = NR * NI * NJ * 4 * w <= 12 * 1024;
  return one_chunk && small_s;
}

template <typename T, int NI, int NJ, int NR, int NX>
hipError_t launch_shape(const FemArgs &a, const T *spack, int mpg, bool ew, bool fast, dim3 grid,
                        hipStream_t s) {
  constexpr int IC = kIC<T, NI, NR>;
  constexpr int WPB = kWPB<T, NI, NJ, NR>;
  // FAST launches of multi-wave blocks cover WPB tiles per block.
  dim3 g = grid;
  if (fast && WPB > 1) g.x = (unsigned)std::max<int64_t>(1, ((int64_t)grid.x + WPB - 1) / WPB);
  // Functional (element-wise) operands get their own instantiations, so the
  // plain kernels carry no prologue code; those keep one member per group.
#define BES_FEM_LAUNCH(MPG, EW, FAST)                                                            \
  hipLaunchKernelGGL((fem_stream_kernel<T, NI, NJ, NR, NX, MPG, IC, EW, FAST,                    \
                                        FAST ? WPB : 1>),                                        \
                     FAST ? g : grid, dim3(kTile * (FAST ? WPB : 1)), 0, s, a, spack)
  if (ew) {
    if (fast) BES_FEM_LAUNCH(1, true, true);
    else BES_FEM_LAUNCH(1, true, false);
  } else if (mpg == 1) {
    if (fast) BES_FEM_LAUNCH(1, false, true);
    else BES_FEM_LAUNCH(1, false, false);
  } else {
    if (fast) BES_FEM_LAUNCH(3, false, true);
    else BES_FEM_LAUNCH(3, false, false);
  }
#undef BES_FEM_LAUNCH
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// FP64 matrix-core variant for shapes whose S outgrows the scalar data cache
// (P4: S = 3 x 35 x 35 doubles).  Stage 1 of a tile is a dense contraction,
//   T[e, (r, i)] = sum_j u[e, j] S[r, i, j]      (64 x 35 times 35 x 105),
// run as v_mfma_f64_16x16x4f64 blocks: M = 16 elements, N = 16 values of i for
// one r, K = 4 values of j.  S is staged once per block in LDS in fragment
// order (B operand, one double per lane, so every LDS read feeds 16
// elements), u of the tile in registers (A operand); the waves of a block
// share S and nothing else, and run unsynchronized.  Stage 2 runs in the
// accumulator layout -- lane l, item v of block mb holds element
// 16 mb + 4 v + l / 16 and i = 16 ib + l % 16 -- reading the per-element G from
// LDS, and each store writes four 16-value runs of one output row.
// Operand layouts (checked on gfx950): A[i][k] in lane i + 16 k,
// B[k][j] in lane j + 16 k, D[i][j] item v of lane l with i = 4 v + l / 16,
// j = l % 16.
// ---------------------------------------------------------------------------
typedef double d4v __attribute__((ext_vector_type(4)));

// True for the FP64 shapes that take the matrix-core variant.
constexpr bool mfma_shape(int NI, int NJ, int NR) {
  return NI >= 16 && NJ >= 4 && NR * NI * NJ * 8 > 12 * 1024;
}

constexpr int kMW = 8;       // waves per block (one block per CU, 2 per SIMD)

// Ordering of one wave's own LDS accesses (its staging regions are private):
// LDS executes a wave's instructions in order, so only the compiler must be
// kept from moving accesses across this point; waves never wait for each
// other, so their load and matrix phases interleave.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}
constexpr int kUPass = 12;   // u rows staged per pass (3 K-blocks)

template <int NI, int NJ, int NR, int NX>
struct MfmaFem {
  static constexpr int kIB = (NI + 15) / 16;           // 16-wide i blocks
  static constexpr int kKB = (NJ + 3) / 4;             // 4-deep j blocks
  static constexpr int kFrags = NR * kIB * kKB;        // B fragments of S
  static constexpr int kPasses = (kKB * 4 + kUPass - 1) / kUPass;
  static constexpr int kGRows = NX * NR > kMaxRow ? NX * NR : kMaxRow;
};

template <int NI, int NJ, int NR, int NX, bool EW>
__global__ void __launch_bounds__(kTile * kMW) __attribute__((amdgpu_waves_per_eu(2)))
    fem_mfma_kernel(const FemArgs a) {
  using M = MfmaFem<NI, NJ, NR, NX>;
  using D = Dense<double, NJ>;
  __shared__ double Sf[M::kFrags * kTile];
  __shared__ double Xall[kMW * kUPass * kPitch];
  __shared__ double Jall[kMW * M::kGRows * kPitch];
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kTile);
  double *const X = Xall + wave * kUPass * kPitch;
  double *const Jb = Jall + wave * M::kGRows * kPitch;

  // S of every group (the launcher checks they are one buffer) as fragments:
  // fragment (r, ib, kb), lane l = S[r][16 ib + l % 16][4 kb + l / 16].
  {
    const FemGroup &G0 = a.grp[0];
    const double *__restrict__ S = (const double *)G0.S;
    for (int f = threadIdx.x; f < M::kFrags * kTile; f += kTile * kMW) {
      const int frag = f / kTile, l = f - frag * kTile;
      const int r = frag / (M::kIB * M::kKB), rem = frag - r * (M::kIB * M::kKB);
      const int ib = rem / M::kKB, kb = rem - ib * M::kKB;
      const int i = 16 * ib + l % 16, j = 4 * kb + l / 16;
      Sf[f] = (i < NI && j < NJ) ? S[r * G0.ss[0] + i * G0.ss[1] + j * G0.ss[2]] : 0.0;
    }
    __syncthreads();
  }

  for (int64_t base = a.tile0 + (int64_t)blockIdx.x * kMW; base < a.tile1;
       base += (int64_t)gridDim.x * kMW) {
    const int64_t mine = base + wave;
    const bool live = mine < a.tile1;          // idle waves repeat the last tile
    const int64_t e0 = (live ? mine : a.tile1 - 1) * kTile;
    for (int g = 0; g < a.n_groups; ++g) {
      int lane = fresh_lane();
      const FemGroup &G = a.grp[g];
      // ---- raw loads: the shared G row (first group of the tile), U ------
      double rg[kMaxRow];
      const int grow = a.grp[0].g_row;
      if (g == 0) {
        const FemSrc &s0 = a.mem[0].g;
        const double *__restrict__ pb = (const double *)s0.p0 + a.grp[0].g_off + e0 * s0.s0[0];
        load_block<double, kMaxRow>(rg, pb, false, (int)s0.s0[0], 1, grow, lane);
      }
      double ru[D::kLen], rw[EW ? D::kLen : 1];
      load_dense<double, NJ>(ru, (const double *)G.u.p0 + G.u.off0 + e0 * NJ, lane);
      if constexpr (EW) {
        if (G.u.kind == FEM_SRC_ELEMENTWISE && G.u.p1) {
          load_dense<double, NJ>(rw, (const double *)G.u.p1 + G.u.off1 + e0 * NJ, lane);
        } else {
#pragma unroll
          for (int k = 0; k < D::kLen; ++k) rw[k] = 0.0;
        }
      }
      // ---- G of this lane's element into Jb[x * NR + r][element] ---------
      if (g == 0) {
        put_block<double, kMaxRow>(X, rg, lane);
        wave_sync();
        double gm[NX][NR];
        g_from_row<double, NX, NR>(X, a.mem[0].g, lane, gm);
#pragma unroll
        for (int x = 0; x < NX; ++x)
#pragma unroll
          for (int r = 0; r < NR; ++r) Jb[(x * NR + r) * kPitch + lane] = gm[x][r];
        wave_sync();
      }
      // ---- prologue, then u in passes of kUPass rows into A fragments -------
      if constexpr (EW) {
        if (G.u.kind == FEM_SRC_ELEMENTWISE) {
          const double alpha = G.u.alpha, beta = G.u.beta;
          const int op = G.u.op;
          // sin / cos: the short reduction when every value of the wave is
          // below 2^20 in magnitude (a wave-uniform branch), else the library
          bool small = true;
#pragma unroll
          for (int k = 0; k < D::kLen; ++k) small = small && fabs(ru[k]) < 0x1p20;
          const bool trig = op == BES_OP_SIN || op == BES_OP_COS;
          if (trig && __builtin_amdgcn_ballot_w64(!small) == 0) {
            const int shift = op == BES_OP_COS ? 1 : 0;
#pragma unroll
            for (int k = 0; k < D::kLen; ++k) ru[k] = alpha * sincos_small(ru[k], shift) + beta + rw[k];
          } else {
#pragma unroll
            for (int k = 0; k < D::kLen; ++k) ru[k] = alpha * apply_op<double>(op, ru[k]) + beta + rw[k];
          }
        }
      }
      double af[4][M::kKB];
#pragma unroll
      for (int p = 0; p < M::kPasses; ++p) {
#pragma unroll
        for (int t = 0; t < D::kVT; ++t)
#pragma unroll
          for (int sv = 0; sv < D::kV; ++sv) {
            const int f = D::kV * (lane + kTile * t) + sv;
            const int el = f / NJ, c = f - el * NJ;
            if (f < NJ * kTile && c >= p * kUPass && c < (p + 1) * kUPass)
              X[(c - p * kUPass) * kPitch + el] = ru[t * D::kV + sv];
          }
        wave_sync();
#pragma unroll
        for (int kl = 0; kl < kUPass / 4; ++kl) {
          const int kb = p * (kUPass / 4) + kl;
          if (kb < M::kKB) {
            const int j = 4 * kb + lane / 16;
#pragma unroll
            for (int mb = 0; mb < 4; ++mb)
              af[mb][kb] = j < NJ ? X[(4 * kl + lane / 16) * kPitch + 16 * mb + lane % 16] : 0.0;
          }
        }
        wave_sync();
      }
      // ---- stage 1 on the matrix cores, stage 2 in the accumulator layout --
      // One 16-element block at a time through every i-block, so that the
      // block's output rows (contiguous) are completed within a short span
      // and leave L2 as whole lines.
      double *__restrict__ outp = (double *)a.mem[G.m0].out;   // one member per group
#pragma unroll 1
      for (int mb = 0; mb < 4; ++mb) {
        lane = fresh_lane();
        d4v acc[NR][M::kIB];
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
          for (int ib = 0; ib < M::kIB; ++ib) acc[r][ib] = d4v{0.0, 0.0, 0.0, 0.0};
        double am[M::kKB];
#pragma unroll
        for (int kb = 0; kb < M::kKB; ++kb) am[kb] = mb == 0 ? af[0][kb] : mb == 1 ? af[1][kb]
                                                  : mb == 2 ? af[2][kb] : af[3][kb];
#pragma unroll
        for (int kb = 0; kb < M::kKB; ++kb)
#pragma unroll
          for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int ib = 0; ib < M::kIB; ++ib) {
              const double b = Sf[((r * M::kIB + ib) * M::kKB + kb) * kTile + lane];
              acc[r][ib] = __builtin_amdgcn_mfma_f64_16x16x4f64(am[kb], b, acc[r][ib], 0, 0, 0);
            }
#pragma unroll
        for (int ib = 0; ib < M::kIB; ++ib) {
          const int i = 16 * ib + lane % 16;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int el = 16 * mb + 4 * v + lane / 16;
#pragma unroll
            for (int x = 0; x < NX; ++x) {
              double o = 0.0;
#pragma unroll
              for (int r = 0; r < NR; ++r) o = fma(Jb[(x * NR + r) * kPitch + el], acc[r][ib][v], o);
              // plain store: L2 merges the 16-value runs of neighbouring
              // stores into whole lines (a streaming hint would send them
              // to HBM as partial writes)
              if (live && i < NI) outp[(e0 + el) * (NX * NI) + x * NI + i] = o;
            }
          }
        }
      }
    }
  }
}

template <int NI, int NJ, int NR, int NX>
hipError_t launch_mfma_shape(const FemArgs &a, bool ew, int grid, hipStream_t s) {
  if constexpr (mfma_shape(NI, NJ, NR)) {
    if (ew)
      hipLaunchKernelGGL((fem_mfma_kernel<NI, NJ, NR, NX, true>), dim3(grid), dim3(kTile * kMW), 0,
                         s, a);
    else
      hipLaunchKernelGGL((fem_mfma_kernel<NI, NJ, NR, NX, false>), dim3(grid), dim3(kTile * kMW), 0,
                         s, a);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// FP64 matrix-core variant with (r, i) on the M side and the elements on N.
// Stage 1 of a unit of 16 elements, T[(r, i), e] = sum_j S[r, i, j] u[e, j],
// runs as v_mfma_f64_16x16x4f64 blocks (M = 16 (r, i) pairs, N = 16
// elements, K = 4 values of j).  The rows are ordered so that the
// accumulator layout hands every lane all NR values of T it needs: item v of
// lane l holds row 4 v + l / 16 of each M block, so lane group q = l / 16
// takes the i values [q IQ, (q + 1) IQ), IQ = ceil(NI / 4), and slot
// s = 4 mb + v of the group holds (i = q IQ + s / NR, r = s % NR).  For P4
// that is 105 useful rows of 112 (with i on the N side: 144 columns).  The j
// axis is split the same way (lane group q' of the K side takes j in
// [q' KQ, (q' + 1) KQ)), so one u value per lane and K block.  S is staged
// once per block in LDS as A fragments.  Per unit a wave
//   * stages the G row of its 16 elements (once per unit; the members share
//     G) and forms G[x][r] of its lane's element in registers;
//   * per member: u (and the second source of an element-wise u) arrive
//     through coalesced 16-byte loads issued one work item ahead; the
//     element-wise prologue runs on them, and LDS turns them into B
//     fragments;
//   * stage 2, out[e, x, i] = sum_r G[x][r] T[r, i], runs in registers; the
//     unit's output block (contiguous: 16 x NX x NI values) goes through LDS
//     to HBM as 16-byte streaming stores of whole lines.
// ---------------------------------------------------------------------------
template <int NI, int NJ, int NR, int NX>
struct MfmaRI {
  static constexpr int kU = 16;                             // elements per unit
  static constexpr int kIQ = (NI + 3) / 4;                  // i values per lane group
  static constexpr int kSlots = kIQ * NR;                   // (i, r) slots per lane group
  static constexpr int kMB = (kSlots + 3) / 4;              // 16-row M blocks
  static constexpr int kKQ = (NJ + 3) / 4;                  // K blocks
  static constexpr int kFrags = kMB * kKQ;                  // A fragments of S
  static constexpr int kOut = kU * NX * NI;                 // output values of a unit
  static constexpr int kUVec = kU * NJ / 2;                 // 16-byte vectors of u per unit
  static constexpr int kUT = (kUVec + kTile - 1) / kTile;   // u vectors per lane
  static constexpr int kOVec = kOut / 2;
  static constexpr int kOT = (kOVec + kTile - 1) / kTile;
  static constexpr int kGP = kU + 1;                        // pitch of the staged G row
  static constexpr int kGT = (kU * kMaxRow + kTile - 1) / kTile;
  static constexpr int kStage0 = kOut > kU * NJ ? kOut : kU * NJ;
  static constexpr int kStage1 = kStage0 > kMaxRow * kGP ? kStage0 : kMaxRow * kGP;
  static constexpr int kStage = (kStage1 + 1) & ~1;         // 16-byte multiple
};

// UK: 0 plain u; 1 element-wise prologue on the groups that have one, one
// source; 2 every group element-wise with two sources.
template <int NI, int NJ, int NR, int NX, int UK>
__global__ void __launch_bounds__(kTile * kMW) __attribute__((amdgpu_waves_per_eu(2)))
    fem_mfma_ri_kernel(const FemArgs a) {
  constexpr bool EW = UK > 0, TWO = UK == 2;
  using M = MfmaRI<NI, NJ, NR, NX>;
  using V2 = typename Vec16<double>::type;
  __shared__ double Sf[M::kFrags * kTile];
  __shared__ V2 Stage2[kMW * M::kStage / 2];
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kTile);
  double *const X = (double *)Stage2 + wave * M::kStage;
  V2 *const XV = Stage2 + wave * (M::kStage / 2);

  // S as A fragments: fragment (mb, kb), lane l holds row m = 16 mb + l % 16
  // (lane group q = m % 4, slot s = 4 mb + (l % 16) / 4) and j = (l / 16) KQ + kb.
  {
    const FemGroup &G0 = a.grp[0];
    const double *__restrict__ S = (const double *)G0.S;
    for (int f = threadIdx.x; f < M::kFrags * kTile; f += kTile * kMW) {
      const int frag = f / kTile, l = f - frag * kTile;
      const int mb = frag / M::kKQ, kb = frag - mb * M::kKQ;
      const int ml = l % 16;
      const int s = 4 * mb + ml / 4, q = ml % 4;
      const int k = s / NR, r = s - k * NR;
      const int i = q * M::kIQ + k, j = (l / 16) * M::kKQ + kb;
      Sf[f] = (s < M::kSlots && i < NI && j < NJ)
                  ? S[r * G0.ss[0] + i * G0.ss[1] + j * G0.ss[2]] : 0.0;
    }
    __syncthreads();
  }

  const int64_t u0 = a.tile0 * (kTile / M::kU), u1 = a.tile1 * (kTile / M::kU);
  const int64_t nw = (int64_t)gridDim.x * kMW;
  int64_t unit = u0 + (int64_t)blockIdx.x * kMW + wave;
  if (unit >= u1) return;
  const int ng = a.n_groups;
  const FemSrc &gs = a.mem[0].g;
  const int grow = a.grp[0].g_row;
  const int gse = (int)gs.s0[0];

  // Raw loads of one work item (unit, member group g): u, the second source
  // of an element-wise u, and the unit's G row when g == 0.  Two sets
  // alternate: the loads of item t + 2 are issued while item t computes.
  struct Raw {
    double u[2 * M::kUT];
    double w[TWO ? 2 * M::kUT : 1];
    double g[M::kGT];
  };
  auto load_item = [&](Raw &R, int64_t un, int g) {
    const int lane = fresh_lane();
    const FemGroup &G = a.grp[g];
    const int64_t e0 = un * M::kU;
    const V2 *__restrict__ pu = (const V2 *)((const double *)G.u.p0 + G.u.off0 + e0 * NJ);
#pragma unroll
    for (int t = 0; t < M::kUT; ++t) {
      int qv = lane + kTile * t;
      if ((t + 1) * kTile > M::kUVec) qv = qv < M::kUVec ? qv : M::kUVec - 1;
      const V2 x = __builtin_nontemporal_load(&pu[qv]);
      R.u[2 * t] = x[0];
      R.u[2 * t + 1] = x[1];
    }
    if constexpr (TWO) {
      const V2 *__restrict__ pw = (const V2 *)((const double *)G.u.p1 + G.u.off1 + e0 * NJ);
#pragma unroll
      for (int t = 0; t < M::kUT; ++t) {
        int qv = lane + kTile * t;
        if ((t + 1) * kTile > M::kUVec) qv = qv < M::kUVec ? qv : M::kUVec - 1;
        const V2 x = __builtin_nontemporal_load(&pw[qv]);
        R.w[2 * t] = x[0];
        R.w[2 * t + 1] = x[1];
      }
    }
    if (g == 0) {
      const double *__restrict__ pg = (const double *)gs.p0 + a.grp[0].g_off + e0 * gse;
      const int lim = (M::kU - 1) * gse + grow - 1;
#pragma unroll
      for (int t = 0; t < M::kGT; ++t) {
        const int f = lane + kTile * t;
        const int el = f / kMaxRow, c = f - el * kMaxRow;
        const int pos = el * gse + c;
        R.g[t] = pg[pos < lim ? pos : lim];
      }
    }
  };

  double gm[NX][NR];
  // G[x][r] of this lane's element from the G row in R (first member of a unit).
  auto stage_g = [&](const Raw &R) {
    const int lane = fresh_lane();
#pragma unroll
    for (int t = 0; t < M::kGT; ++t) {
      const int f = lane + kTile * t;
      const int el = f / kMaxRow, c = f - el * kMaxRow;
      if (f < M::kU * kMaxRow) X[c * M::kGP + el] = R.g[t];
    }
    wave_sync();
    g_from_row<double, NX, NR, M::kGP>(X, gs, lane % 16, gm);
    wave_sync();
  };
  // u values through LDS into B fragments: lane (n, q) takes u[n][q KQ + kb].
  auto to_bf = [&](const double (&uv)[2 * M::kUT], double (&bf)[M::kKQ]) {
    const int lane = fresh_lane();
#pragma unroll
    for (int t = 0; t < M::kUT; ++t) {
      const int qv = lane + kTile * t;
      if ((t + 1) * kTile <= M::kUVec || qv < M::kUVec) XV[qv] = V2{uv[2 * t], uv[2 * t + 1]};
    }
    wave_sync();
    const int n = lane % 16, q = lane / 16;
#pragma unroll
    for (int kb = 0; kb < M::kKQ; ++kb) {
      const int j = q * M::kKQ + kb;
      bf[kb] = j < NJ ? X[n * NJ + j] : 0.0;
    }
    wave_sync();
  };
  auto mfma = [&](const double (&bf)[M::kKQ], d4v (&acc)[M::kMB]) {
    const int lane = fresh_lane();
#pragma unroll
    for (int mb = 0; mb < M::kMB; ++mb) acc[mb] = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kb = 0; kb < M::kKQ; ++kb)
#pragma unroll
      for (int mb = 0; mb < M::kMB; ++mb)
        acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(Sf[(mb * M::kKQ + kb) * kTile + lane],
                                                       bf[kb], acc[mb], 0, 0, 0);
  };
  // Stage 1 of the current item on the matrix cores; meanwhile the next
  // item's u values (uv, from R) get their element-wise prologue on the
  // vector ALUs: the two share one basic block so the scheduler interleaves
  // them.
  auto mfma_and_prologue = [&](const double (&bf)[M::kKQ], d4v (&acc)[M::kMB], bool next,
                               const Raw &R, int gn, double (&uv)[2 * M::kUT]) {
#pragma unroll
    for (int k = 0; k < 2 * M::kUT; ++k) uv[k] = R.u[k];
    if (!next) {
      mfma(bf, acc);
      return;
    }
    if constexpr (EW) {
      const FemSrc &u = a.grp[gn].u;
      if (u.kind == FEM_SRC_ELEMENTWISE) {
        const double alpha = u.alpha, beta = u.beta;
        const int op = u.op;
        bool small = true;
#pragma unroll
        for (int k = 0; k < 2 * M::kUT; ++k) small = small && fabs(uv[k]) < 0x1p20;
        const bool trig = op == BES_OP_SIN || op == BES_OP_COS;
        if (trig && __builtin_amdgcn_ballot_w64(!small) == 0) {
          // sin / cos: the short reduction (every value of the wave below 2^20)
          const int shift = op == BES_OP_COS ? 1 : 0;
          mfma(bf, acc);
#pragma unroll
          for (int k = 0; k < 2 * M::kUT; ++k)
            uv[k] = alpha * sincos_small(uv[k], shift) + beta + (TWO ? R.w[k] : 0.0);
          // issue order: each matrix instruction followed by a run of the
          // prologue's vector instructions, which execute in its shadow
#pragma unroll
          for (int k = 0; k < M::kFrags; ++k) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, 6, 0);   // VALU
          }
        } else {
          mfma(bf, acc);
#pragma unroll
          for (int k = 0; k < 2 * M::kUT; ++k)
            uv[k] = alpha * apply_op<double>(op, uv[k]) + beta + (TWO ? R.w[k] : 0.0);
        }
        return;
      }
    }
    mfma(bf, acc);
  };
  // Stage 2 of item (un, g) in the accumulator layout; the unit's output
  // block goes through LDS to HBM.
  auto stage2 = [&](const d4v (&acc)[M::kMB], int64_t un, int g) {
    const int lane = fresh_lane();
    const int n = lane % 16, q = lane / 16;
#pragma unroll
    for (int k = 0; k < M::kIQ; ++k) {
      const int i = q * M::kIQ + k;
#pragma unroll
      for (int x = 0; x < NX; ++x) {
        double o = 0.0;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const int s = k * NR + r;
          o = fma(gm[x][r], acc[s / 4][s % 4], o);
        }
        if (i < NI) X[n * (NX * NI) + x * NI + i] = o;
      }
    }
    wave_sync();
    V2 *__restrict__ ov = (V2 *)((double *)a.mem[a.grp[g].m0].out + un * M::kU * (NX * NI));
#pragma unroll
    for (int t = 0; t < M::kOT; ++t) {
      const int qv = lane + kTile * t;
      if ((t + 1) * kTile <= M::kOVec || qv < M::kOVec) {
        const V2 vv = XV[qv];
        __builtin_nontemporal_store(vv, &ov[qv]);
      }
    }
    wave_sync();
  };
  // One item k: its G row (first member of a unit) from Rk, the loads of
  // item k + 2 into Rk, stage 1 of k with the prologue of k + 1 (raw in Rn),
  // the B fragments of k + 1, stage 2 of k.
  double bf[M::kKQ];
  auto step = [&](Raw &Rk, const Raw &Rn, int64_t uk, int gk, bool v1, int g1, bool v2,
                  int64_t u2, int g2) {
    if (gk == 0) stage_g(Rk);
    if (v2) load_item(Rk, u2, g2);
    d4v acc[M::kMB];
    double uv[2 * M::kUT];
    mfma_and_prologue(bf, acc, v1, Rn, g1, uv);
    if (v1) to_bf(uv, bf);
    stage2(acc, uk, gk);
  };

  // items in order: (unit, 0..ng-1), then the wave's next unit
  auto advance = [&](int64_t &un, int &g) {
    if (++g == ng) {
      g = 0;
      un += nw;
    }
  };
  Raw A, B;
  int64_t ua = unit, ub = unit, uc;
  int ga = 0, gb = 0, gc;
  advance(ub, gb);
  load_item(A, ua, ga);
  if (ub < u1) load_item(B, ub, gb);
  {
    // the first item's prologue and B fragments, not overlapped
    d4v acc[M::kMB];
    double uv[2 * M::kUT];
    (void)acc;
#pragma unroll
    for (int k = 0; k < 2 * M::kUT; ++k) uv[k] = A.u[k];
    if constexpr (EW) {
      const FemSrc &u = a.grp[ga].u;
      if (u.kind == FEM_SRC_ELEMENTWISE) {
#pragma unroll
        for (int k = 0; k < 2 * M::kUT; ++k)
          uv[k] = u.alpha * apply_op<double>(u.op, uv[k]) + u.beta + (TWO ? A.w[k] : 0.0);
      }
    }
    to_bf(uv, bf);
  }
  while (true) {
    // A: item a (G row pending), B: item b = a + 1; item c = b + 1 into A
    uc = ub;
    gc = gb;
    advance(uc, gc);
    step(A, B, ua, ga, ub < u1, gb, uc < u1, uc, gc);
    if (ub >= u1) break;
    ua = uc;
    ga = gc;
    // B: item b (G row pending), A: item a = b + 1; the item after into B
    uc = ua;
    gc = ga;
    advance(uc, gc);
    step(B, A, ub, gb, ua < u1, ga, uc < u1, uc, gc);
    if (ua >= u1) break;
    ub = uc;
    gb = gc;
  }
}

// Source kind of the groups' u for fem_mfma_ri_kernel (its UK), or -1 when
// the groups mix one- and two-source element-wise operands.
int ri_u_kind(const FemArgs &a) {
  bool any_ew = false, any_two = false, all_two = true;
  for (int g = 0; g < a.n_groups; ++g) {
    const FemSrc &u = a.grp[g].u;
    const bool ew = u.kind == FEM_SRC_ELEMENTWISE;
    any_ew |= ew;
    any_two |= ew && u.p1 != nullptr;
    all_two &= ew && u.p1 != nullptr;
  }
  if (!any_ew) return 0;
  if (all_two) return 2;
  return any_two ? -1 : 1;
}

template <int NI, int NJ, int NR, int NX>
hipError_t launch_mfma_ri_shape(const FemArgs &a, int uk, int grid, hipStream_t s) {
  if constexpr (mfma_shape(NI, NJ, NR)) {
    const dim3 block(kTile * kMW);
    if (uk == 2)
      hipLaunchKernelGGL((fem_mfma_ri_kernel<NI, NJ, NR, NX, 2>), dim3(grid), block, 0, s, a);
    else if (uk == 1)
      hipLaunchKernelGGL((fem_mfma_ri_kernel<NI, NJ, NR, NX, 1>), dim3(grid), block, 0, s, a);
    else if (uk == 0)
      hipLaunchKernelGGL((fem_mfma_ri_kernel<NI, NJ, NR, NX, 0>), dim3(grid), block, 0, s, a);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// FP32 matrix-core variant of the gradient class for one stage-1 group (its
// members share S and u; each has its own G view and output).  Stage 1 of 16
// elements runs on v_mfma_f32_16x16x4f32 with (r, i) on the M side, laid out
// so that each lane ends with all NR values of T for its i values: the FP32
// accumulator holds row 4 (lane / 16) + v of each block in item v, so lane
// group q takes slots s = 4 mb + v with i = q IQ + s / NR, r = s % NR (for
// P3: 60 useful rows of 64, K = 20 exactly).  Stage 2 runs per member in
// registers.  u comes in and each member's output block goes out through a
// small per-wave LDS area with 16-byte accesses; units of 16 elements are
// dealt to the grid's waves in turn, the next unit's loads in flight while
// the current one computes.
// ---------------------------------------------------------------------------
typedef float f4v __attribute__((ext_vector_type(4)));

template <int NI, int NJ, int NR, int NX>
struct Mfma32 {
  static constexpr int kU = 16;                             // elements per unit
  static constexpr int kIQ = (NI + 3) / 4;                  // i values per lane group
  static constexpr int kSlots = kIQ * NR;                   // (i, r) slots per lane group
  static constexpr int kMB = (kSlots + 3) / 4;              // 16-row M blocks
  static constexpr int kKQ = (NJ + 3) / 4;                  // K blocks
  static constexpr int kFrags = kMB * kKQ;                  // A fragments of S
  static constexpr int kOut = kU * NX * NI;                 // output values of a member
  static constexpr int kUVec = kU * NJ / 4;                 // 16-byte vectors of u
  static constexpr int kUT = (kUVec + kTile - 1) / kTile;
  static constexpr int kOVec = kOut / 4;
  static constexpr int kOT = (kOVec + kTile - 1) / kTile;
  static constexpr int kGP = kU + 1;                        // pitch of the staged G row
  static constexpr int kGT = (kU * kMaxRow + kTile - 1) / kTile;
  static constexpr int kStage0 = kOut > kU * NJ ? kOut : kU * NJ;
  static constexpr int kStage1 = kStage0 > kMaxRow * kGP ? kStage0 : kMaxRow * kGP;
  static constexpr int kStage = (kStage1 + 3) & ~3;         // 16-byte multiple
};
constexpr int kMW32 = 4;        // waves per block
constexpr int kMaxMem32 = 3;    // members of the group

template <int NI, int NJ, int NR, int NX>
__global__ void __launch_bounds__(kTile * kMW32) fem_mfma32_kernel(const FemArgs a) {
  using M = Mfma32<NI, NJ, NR, NX>;
  using V4 = typename Vec16<float>::type;
  __shared__ float Sf[M::kFrags * kTile];
  __shared__ V4 Stage4[kMW32 * M::kStage / 4];
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kTile);
  float *const X = (float *)Stage4 + wave * M::kStage;
  V4 *const XV = Stage4 + wave * (M::kStage / 4);
  const FemGroup &G = a.grp[0];

  // S as A fragments: fragment (mb, kb), lane l holds row m = 16 mb + l % 16
  // (lane group q = (l % 16) / 4, slot s = 4 mb + l % 4) and j = (l / 16) KQ + kb.
  {
    const float *__restrict__ S = (const float *)G.S;
    for (int f = threadIdx.x; f < M::kFrags * kTile; f += kTile * kMW32) {
      const int frag = f / kTile, l = f - frag * kTile;
      const int mb = frag / M::kKQ, kb = frag - mb * M::kKQ;
      const int ml = l % 16;
      const int s = 4 * mb + ml % 4, q = ml / 4;
      const int k = s / NR, r = s - k * NR;
      const int i = q * M::kIQ + k, j = (l / 16) * M::kKQ + kb;
      Sf[f] = (s < M::kSlots && i < NI && j < NJ)
                  ? S[r * G.ss[0] + i * G.ss[1] + j * G.ss[2]] : 0.0f;
    }
    __syncthreads();
  }

  const int64_t u0 = a.tile0 * (kTile / M::kU), u1 = a.tile1 * (kTile / M::kU);
  const int64_t nw = (int64_t)gridDim.x * kMW32;
  int64_t unit = u0 + (int64_t)blockIdx.x * kMW32 + wave;
  if (unit >= u1) return;
  const int nm = a.n_members;
  const FemSrc &gs = a.mem[0].g;
  const int grow = G.g_row;
  const int gse = (int)gs.s0[0];

  V4 ru[M::kUT];
  float rg[M::kGT];
  auto load = [&](int64_t un) {
    const int lane = fresh_lane();
    const int64_t e0 = un * M::kU;
    const V4 *__restrict__ pu = (const V4 *)((const float *)G.u.p0 + G.u.off0 + e0 * NJ);
#pragma unroll
    for (int t = 0; t < M::kUT; ++t) {
      int qv = lane + kTile * t;
      if ((t + 1) * kTile > M::kUVec) qv = qv < M::kUVec ? qv : M::kUVec - 1;
      ru[t] = __builtin_nontemporal_load(&pu[qv]);
    }
    const float *__restrict__ pg = (const float *)gs.p0 + G.g_off + e0 * gse;
    const int lim = (M::kU - 1) * gse + grow - 1;
#pragma unroll
    for (int t = 0; t < M::kGT; ++t) {
      const int f = lane + kTile * t;
      const int el = f / kMaxRow, c = f - el * kMaxRow;
      const int pos = el * gse + c;
      rg[t] = pg[pos < lim ? pos : lim];
    }
  };
  load(unit);
  while (true) {
    const int lane = fresh_lane();
    const int n = lane % 16, q = lane / 16;
    const int64_t e0 = unit * M::kU;
    // ---- G of this lane's element for every member, from the staged row --
#pragma unroll
    for (int t = 0; t < M::kGT; ++t) {
      const int f = lane + kTile * t;
      const int el = f / kMaxRow, c = f - el * kMaxRow;
      if (f < M::kU * kMaxRow) X[c * M::kGP + el] = rg[t];
    }
    wave_sync();
    float gm[kMaxMem32][NX][NR];
#pragma unroll
    for (int m = 0; m < kMaxMem32; ++m)
      if (m < nm) g_from_row<float, NX, NR, M::kGP>(X, a.mem[m].g, n, gm[m]);
    wave_sync();
    // ---- u through LDS into B fragments -----------------------------------
#pragma unroll
    for (int t = 0; t < M::kUT; ++t) {
      const int qv = lane + kTile * t;
      if ((t + 1) * kTile <= M::kUVec || qv < M::kUVec) XV[qv] = ru[t];
    }
    wave_sync();
    float bf[M::kKQ];
#pragma unroll
    for (int kb = 0; kb < M::kKQ; ++kb) {
      const int j = q * M::kKQ + kb;
      bf[kb] = j < NJ ? X[n * NJ + j] : 0.0f;
    }
    wave_sync();
    // ---- the next unit's loads, in flight during this one -----------------
    const int64_t next = unit + nw;
    const bool more = next < u1;
    if (more) load(next);
    // ---- stage 1 on the matrix cores -------------------------------------
    f4v acc[M::kMB];
#pragma unroll
    for (int mb = 0; mb < M::kMB; ++mb) acc[mb] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kb = 0; kb < M::kKQ; ++kb)
#pragma unroll
      for (int mb = 0; mb < M::kMB; ++mb)
        acc[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(Sf[(mb * M::kKQ + kb) * kTile + lane],
                                                       bf[kb], acc[mb], 0, 0, 0);
    // ---- stage 2 per member, output block through LDS ---------------------
#pragma unroll
    for (int m = 0; m < kMaxMem32; ++m) {
      if (m >= nm) break;
#pragma unroll
      for (int k = 0; k < M::kIQ; ++k) {
        const int i = q * M::kIQ + k;
#pragma unroll
        for (int x = 0; x < NX; ++x) {
          float o = 0.0f;
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const int s = k * NR + r;
            o = fmaf(gm[m][x][r], acc[s / 4][s % 4], o);
          }
          if (i < NI) X[n * (NX * NI) + x * NI + i] = o;
        }
      }
      wave_sync();
      V4 *__restrict__ ov = (V4 *)((float *)a.mem[m].out + e0 * (NX * NI));
#pragma unroll
      for (int t = 0; t < M::kOT; ++t) {
        const int qv = lane + kTile * t;
        if ((t + 1) * kTile <= M::kOVec || qv < M::kOVec) {
          const V4 vv = XV[qv];
          __builtin_nontemporal_store(vv, &ov[qv]);
        }
      }
      wave_sync();
    }
    if (!more) break;
    unit = next;
  }
}

template <int NI, int NJ, int NR, int NX>
hipError_t launch_mfma32_shape(const FemArgs &a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((fem_mfma32_kernel<NI, NJ, NR, NX>), dim3(grid), dim3(kTile * kMW32), 0, s,
                     a);
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

bool same_src(const FemSrc &x, const FemSrc &y) {
  if (x.kind != y.kind || x.p0 != y.p0 || x.p1 != y.p1 || x.off0 != y.off0 || x.off1 != y.off1 ||
      x.op != y.op || x.alpha != y.alpha || x.beta != y.beta)
    return false;
  for (int k = 0; k < 3; ++k)
    if (x.s0[k] != y.s0[k] || x.s1[k] != y.s1[k]) return false;
  return true;
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
                      int blocks_per_cu, int variant, hipStream_t stream, hipEvent_t ev_start,
                      hipEvent_t ev_stop) {
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
  // Every member reads the same G through one shared row: stage it once per
  // tile (the Jacobian of all members of a functional batch, for example).
  bool g_same = a.n_members > 0 && a.mem[0].g.kind != FEM_SRC_NONE;
  for (int m = 1; m < a.n_members && g_same; ++m) g_same = same_src(a.mem[m].g, a.mem[0].g);
  for (int g = 0; g < a.n_groups && g_same; ++g) g_same = a.grp[g].g_row > 0;
  const int mpg = (maxm <= 1 || ew) ? 1 : 3;
  int chunk_src[BES_FEM_MAX_GROUPS + 1];
  FemArgs c = chunk_groups(a, mpg, chunk_src);
  if (c.n_groups > BES_FEM_MAX_GROUPS) return hipErrorInvalidValue;
  c.g_same = g_same ? 1 : 0;
  (void)tet;
  for (int g = 0; g < c.n_groups; ++g) {
    const FemSrc &u = c.grp[g].u;
    bool d = u.s0[0] == NJ && u.s0[1] == 1;
    if (u.kind == FEM_SRC_ELEMENTWISE && u.p1) d = d && u.s1[0] == NJ && u.s1[1] == 1;
    c.grp[g].u_dense = d ? 1 : 0;
  }
  for (int m = 0; m < c.n_members; ++m) {
    FemMember &M = c.mem[m];
    M.o_dense = (M.oe == (int64_t)NX * NI && (NX == 1 || M.ox == NI) && M.oi == 1) ? 1 : 0;
  }
  // Full dense tiles go to the straight-line FAST instantiation; the last
  // partial tile and any other layout to the general one.
  bool fast_ok = true;
  for (int g = 0; g < c.n_groups && fast_ok; ++g) {
    const FemGroup &G = c.grp[g];
    fast_ok = G.u_dense != 0;
    const bool has_g = c.mem[G.m0].g.kind != FEM_SRC_NONE;
    const int row = c.g_same ? (g == 0 ? c.grp[0].g_row : 1) : G.g_row;
    if (has_g && row <= 0) fast_ok = false;
  }
  for (int m = 0; m < c.n_members && fast_ok; ++m) fast_ok = c.mem[m].o_dense != 0;
  // The FAST code moves dense U rows and contiguous outputs 16 bytes at a time.
  const size_t esz = f64 ? 8 : 4;
  auto al16 = [](const void *p, int64_t off, size_t esz) {
    return (((uintptr_t)p + (uintptr_t)(off * (int64_t)esz)) & 15u) == 0;
  };
  for (int g = 0; g < c.n_groups && fast_ok; ++g) {
    const FemSrc &u = c.grp[g].u;
    fast_ok = al16(u.p0, u.off0, esz) && (!u.p1 || u.kind != FEM_SRC_ELEMENTWISE || al16(u.p1, u.off1, esz));
  }
  for (int m = 0; m < c.n_members && fast_ok; ++m) fast_ok = al16(c.mem[m].out, 0, esz);
  const int64_t tiles = (a.E + kTile - 1) / kTile;
  const int64_t full_tiles = fast_ok ? a.E / kTile : 0;
  // FP32 matrix-core variant (p[2] = 3): one stage-1 group of at most three
  // members, plain u, every member's G a view of one staged row (or the
  // tetrahedron rows), full dense tiles.  It reads S in place.
  bool use_mfma32 = variant == 3 && !f64 && fast_ok && full_tiles > 0 && !ew &&
                    c.n_groups == 1 && c.grp[0].m0 == 0 && c.grp[0].m1 == c.n_members &&
                    c.n_members >= 1 && c.n_members <= kMaxMem32 && c.grp[0].g_row > 0 &&
                    c.grp[0].g_row <= kMaxRow && c.mem[0].g.s0[0] > 0 &&
                    c.mem[0].g.s0[0] <= INT32_MAX;
  for (int m = 0; m < c.n_members && use_mfma32; ++m) {
    const FemSrc &g = c.mem[m].g;
    if (g.kind == FEM_SRC_TET) {
      use_mfma32 = NX == 3 && NR == 3;
      continue;
    }
    use_mfma32 = g.kind == FEM_SRC_ARRAY;   // a view of the group's staged row
    for (int x = 0; x < NX && use_mfma32; ++x)
      for (int r = 0; r < NR && use_mfma32; ++r) {
        const int64_t pos = g.off0 + x * g.s0[1] + r * g.s0[2];
        use_mfma32 = pos >= 0 && pos < c.grp[0].g_row;
      }
  }
  // S is read in place when it is dense [r][i][j]; other layouts are packed
  // into that layout first (one small kernel, only when needed).
  PackArgs pk;
  pk.n_groups = c.n_groups;
  pk.NR = NR;
  pk.NI = NI;
  pk.NJ = NJ;
  bool need_pack = false;
  pk.transposed = chunks_of(f64, NI, NR) == 1 ? 1 : 0;
  for (int k = 0; k < c.n_groups; ++k) {
    FemGroup &G = c.grp[k];
    const bool dense = !pk.transposed && G.ss[2] == 1 && (NI == 1 || G.ss[1] == NJ) &&
                       (NR == 1 || G.ss[0] == (int64_t)NI * NJ);
    G.s_dense = dense ? 1 : 0;
    pk.S[k] = dense ? nullptr : G.S;
    pk.sr[k] = G.ss[0];
    pk.si[k] = G.ss[1];
    pk.sj[k] = G.ss[2];
    // the matrix-core variant reads S in place; a partial last tile still
    // goes to the general kernel, which reads the packed layout
    need_pack |= !dense && !(use_mfma32 && full_tiles == tiles);
  }
  hipError_t e = hipSuccess;
  if (need_pack) {
    const int pack_total = NR * NI * NJ * c.n_groups;
    dim3 pgrid((pack_total + 255) / 256);
    if (f64)
      hipLaunchKernelGGL(pack_s_kernel<double>, pgrid, dim3(256), 0, stream, pk,
                         (double *)workspace);
    else
      hipLaunchKernelGGL(pack_s_kernel<float>, pgrid, dim3(256), 0, stream, pk,
                         (float *)workspace);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (blocks_per_cu < 1) blocks_per_cu = 1;
  const int64_t cap = (int64_t)device_cu_count() * blocks_per_cu;
  auto launch = [&](bool fast, int64_t t0, int64_t t1) -> hipError_t {
    FemArgs d = c;
    d.tile0 = t0;
    d.tile1 = t1;
    dim3 grid((unsigned)std::min<int64_t>(t1 - t0, cap));
#define BES_FEM_DISPATCH(ni, nj, nr, nx)                                                      \
    if (NI == ni && NJ == nj && NR == nr && NX == nx)                                         \
      return f64 ? launch_shape<double, ni, nj, nr, nx>(d, (const double *)workspace, mpg, ew, \
                                                        fast, grid, stream)                   \
                 : launch_shape<float, ni, nj, nr, nx>(d, (const float *)workspace, mpg, ew,   \
                                                       fast, grid, stream);
    BES_FEM_SHAPES(BES_FEM_DISPATCH)
#undef BES_FEM_DISPATCH
    return hipErrorInvalidValue;
  };
  // Matrix-core variant: FP64, large S shared by every group, one G shared
  // by every member through one row (or none), full dense tiles.
  bool use_mfma = f64 && fast_ok && full_tiles > 0 && mfma_shape(NI, NJ, NR) && c.g_same &&
                  c.grp[0].g_row > 0 && NX * NR <= kMaxRow;
  for (int g = 0; g < c.n_groups && use_mfma; ++g) use_mfma = c.grp[g].m1 - c.grp[g].m0 == 1;
  for (int g = 1; g < c.n_groups && use_mfma; ++g)
    use_mfma = c.grp[g].S == c.grp[0].S && c.grp[g].ss[0] == c.grp[0].ss[0] &&
               c.grp[g].ss[1] == c.grp[0].ss[1] && c.grp[g].ss[2] == c.grp[0].ss[2];
  // Lean variant: one group, one output component per member, G absent or
  // one shared row of plain views.
  bool use_lean = variant != 1 && !use_mfma && !use_mfma32 && fast_ok && full_tiles > 0 && NX == 1 && !ew &&
                  c.n_groups == 1 &&
                  pk.transposed && c.n_members <= 3 && c.grp[0].m0 == 0 &&
                  c.grp[0].m1 == c.n_members && lean_shape(f64, NI, NJ, NR);
  LeanArgs la{};
  if (use_lean) {
    const FemGroup &G = c.grp[0];
    bool no_g = true, row_g = G.g_row > 0 && G.g_row <= kMaxRow;
    for (int m = 0; m < c.n_members; ++m) {
      no_g = no_g && c.mem[m].g.kind == FEM_SRC_NONE;
      row_g = row_g && c.mem[m].g.kind == FEM_SRC_ARRAY;
    }
    use_lean = no_g || row_g;
    if (use_lean) {
      const size_t esz_ = f64 ? 8 : 4;
      la.u = (const char *)G.u.p0 + G.u.off0 * (int64_t)esz_;
      la.tile0 = 0;
      la.tile1 = full_tiles;
      la.n_mem = c.n_members;
      if (row_g) {
        const FemSrc &s0 = c.mem[0].g;
        la.grow = (const char *)s0.p0 + G.g_off * (int64_t)esz_;
        la.g_w = G.g_row;
        la.g_stride = (int32_t)s0.s0[0];
      }
      for (int m = 0; m < c.n_members; ++m) {
        la.out[m] = c.mem[m].out;
        for (int r = 0; r < NR && row_g; ++r) {
          const int64_t pos = c.mem[m].g.off0 + r * c.mem[m].g.s0[2];
          if (pos < 0 || pos >= G.g_row) use_lean = false;   // outside the staged row
          else la.g_off[m][r] = (int32_t)pos;
        }
      }
      if (row_g && (c.mem[0].g.s0[0] <= 0 || c.mem[0].g.s0[0] > INT32_MAX)) use_lean = false;
    }
  }
  if (ev_start && (e = hipEventRecord(ev_start, stream)) != hipSuccess) return e;
  if (use_mfma32) {
    const int64_t units = full_tiles * (kTile / 16);
    const int64_t blocks = std::min<int64_t>((units + kMW32 - 1) / kMW32,
                                             (int64_t)device_cu_count() * blocks_per_cu);
    FemArgs d = c;
    d.tile0 = 0;
    d.tile1 = full_tiles;
    e = hipErrorInvalidValue;
#define BES_FEM_MFMA32_DISPATCH(ni, nj, nr, nx)                                           \
    if (NI == ni && NJ == nj && NR == nr && NX == nx) e = launch_mfma32_shape<ni, nj, nr, nx>(d, (int)blocks, stream);
    BES_FEM_SHAPES(BES_FEM_MFMA32_DISPATCH)
#undef BES_FEM_MFMA32_DISPATCH
    if (e != hipSuccess) return e;
  } else if (use_lean) {
    const int wpt = variant == 2 ? 1 : 2;       // waves per tile
    dim3 lgrid((unsigned)std::min<int64_t>(full_tiles, cap));
    e = hipErrorInvalidValue;
#define BES_FEM_LEAN_DISPATCH(ni, nj, nr, nx)                                                  \
    if (NI == ni && NJ == nj && NR == nr && nx == 1)                                          \
      e = f64 ? launch_lean<double, ni, nj, nr>(la, (const double *)workspace, mpg, wpt, lgrid, \
                                                stream)                                        \
              : launch_lean<float, ni, nj, nr>(la, (const float *)workspace, mpg, wpt, lgrid,  \
                                               stream);
    BES_FEM_SHAPES(BES_FEM_LEAN_DISPATCH)
#undef BES_FEM_LEAN_DISPATCH
    if (e != hipSuccess) return e;
  } else if (use_mfma) {
    FemArgs d = c;
    d.tile0 = 0;
    d.tile1 = full_tiles;
    const int64_t blocks = std::min<int64_t>((full_tiles + kMW - 1) / kMW,
                                             (int64_t)device_cu_count() * std::max(1, blocks_per_cu / kMW));
    // variant 1, or groups that mix one- and two-source element-wise u: i
    // on the N side; otherwise (r, i) on the M side
    const int uk = ri_u_kind(d);
    const bool ri = variant != 1 && uk >= 0;
#define BES_FEM_MFMA_DISPATCH(ni, nj, nr, nx)                                              \
    if (NI == ni && NJ == nj && NR == nr && NX == nx)                                      \
      e = ri ? launch_mfma_ri_shape<ni, nj, nr, nx>(d, uk, (int)blocks, stream)            \
             : launch_mfma_shape<ni, nj, nr, nx>(d, ew, (int)blocks, stream);
    e = hipErrorInvalidValue;
    BES_FEM_SHAPES(BES_FEM_MFMA_DISPATCH)
#undef BES_FEM_MFMA_DISPATCH
    if (e != hipSuccess) return e;
  } else if (full_tiles > 0) {
    e = launch(true, 0, full_tiles);
    if (e != hipSuccess) return e;
  }
  if (full_tiles < tiles && (e = launch(false, full_tiles, tiles)) != hipSuccess) return e;
  if (ev_stop && (e = hipEventRecord(ev_stop, stream)) != hipSuccess) return e;
  return hipSuccess;
}

}  // namespace bes
