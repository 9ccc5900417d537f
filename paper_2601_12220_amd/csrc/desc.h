// Plain-old-data launch descriptors shared by the host planner and the HIP
// kernels.  Host code fills them after binding the caller's buffers to the
// canonical operand slots; kernels read them from kernel arguments or from a
// device-resident table.
#pragma once

#include <stdint.h>

// ---------------------------------------------------------------------------
// FEM-stream template: per-element ("stream") operands U and G, a small
// operand S that carries no stream index.  Per element e and member m:
//   T_g[r, i]        = sum_j S_g[r, i, j] * U_g[e, j]        (stage 1)
//   out_m[e, x, i]   = sum_r G_m[e, x, r] * T_g[r, i]        (stage 2)
// where g is the stage-1 group of member m (members whose S and U are the
// same argument share T: the batch-level hoisting of a shared product).
// Without G (two-operand einsums) out_m[e, i] = T_g[0, i].
// ---------------------------------------------------------------------------
#define BES_FEM_MAX_MEMBERS 8
#define BES_FEM_MAX_GROUPS 8

enum { FEM_SRC_ARRAY = 0, FEM_SRC_ELEMENTWISE = 1, FEM_SRC_TET = 2, FEM_SRC_NONE = 3 };

typedef struct FemSrc {
  const void *p0;
  const void *p1;   // second source of ELEMENTWISE (S1) or NULL
  int64_t off0, off1;
  int64_t s0[3];    // strides of source 0 along (e, x, r) for G, (e, j) for U;
                    // for TET: (e, vertex, coordinate) strides of V[e, 4, 3]
  int64_t s1[3];    // for TET, s1[0] = 1 when the einsum reads the Jacobian
                    // operand with its last two axes swapped, (e, r, x)
  int32_t kind;     // FEM_SRC_*
  int32_t op;       // BES_OP_*
  double alpha, beta;
} FemSrc;

typedef struct FemMember {
  FemSrc g;         // kind FEM_SRC_NONE when the einsum has no G operand
  void *out;
  int64_t oe, ox, oi;  // output strides along (e, x, i)
  int32_t group;
  int32_t o_dense;     // set by the launcher: oe == NX*NI, ox == NI, oi == 1
} FemMember;

typedef struct FemGroup {
  const void *S;    // the caller's S (offset applied)
  int64_t ss[3];    // S strides along (r, i, j); S that is not dense in that
                    // order is packed into it by the launcher
  FemSrc u;
  int32_t m0, m1;   // members [m0, m1) use this group
  int32_t g_row;    // > 0: the G operands of all members of the group read
                    // one row of g_row (<= 12) contiguous components per
                    // element, p0 + g_off + e * s0[0] + c, from one source
                    // (views of one buffer, or dense tetrahedron vertex rows);
                    // the row is staged once per tile and shared
  int32_t u_dense;  // set by the launcher: U's source rows are dense
                    // (s0 = (NJ, 1), and s1 likewise for a second source)
  int64_t g_off;
  int32_t s_dense;  // set by the launcher: S is dense [r][i][j] (read in place)
  int32_t pad2;
} FemGroup;

typedef struct FemArgs {
  int64_t E;                 // number of stream elements
  int64_t tile0, tile1;      // 64-element tiles [tile0, tile1) of this launch
  int32_t n_groups, n_members;
  int32_t g_same;            // every member reads the same G through one shared
                             // row: the row is staged once per tile
  int32_t pad;
  FemGroup grp[BES_FEM_MAX_GROUPS];
  FemMember mem[BES_FEM_MAX_MEMBERS];
} FemArgs;

// ---------------------------------------------------------------------------
// FEM-stream "apply" class (face mass and local divergence of Section
// "Batched einsums in DG-FEM Operators"): per element e and member m,
//   W_m[c, j]   = sum_x G[x, c, e] U_m[x, e, j]   (DIAG: G[c, e] U_m[c, e, j])
//   out_m[e, i] = sum_{c, j} S[c, i, j] W_m[c, j]
// with one S and one G shared by every member (the reference face-mass or
// derivative matrix and the geometry terms) and a streamed operand U_m per
// member (flux or vector-field components).  Strides are in elements.
// ---------------------------------------------------------------------------
#define BES_FEM_APPLY_MAX_MEMBERS 16

typedef struct FemApplyMember {
  const void *u0;       // U source 0 (offset applied by the kernel)
  const void *u1;       // second source of an ELEMENTWISE U, or NULL
  int64_t uoff0, uoff1;
  int64_t us0[3];       // U source 0 strides along (x, e, j)
  int64_t us1[3];       // U source 1 strides along (x, e, j)
  void *out;
  int64_t oe, oi;       // output strides along (e, i)
} FemApplyMember;

typedef struct FemApplyArgs {
  int64_t E;
  const void *S;        // offset applied
  int64_t ss[3];        // S strides along (c, i, j)
  const void *G;        // offset applied
  int64_t gs[3];        // G strides along (x, c, e); DIAG: (unused, c, e)
  int32_t n_members;
  int32_t u_kind;       // FEM_SRC_ARRAY or FEM_SRC_ELEMENTWISE (all members)
  int32_t op;           // BES_OP_* of an ELEMENTWISE U
  int32_t pad;
  double alpha, beta;
  FemApplyMember mem[BES_FEM_APPLY_MAX_MEMBERS];
} FemApplyArgs;

// ---------------------------------------------------------------------------
// Generic template: any batched einsum with up to 4 operands, 8 output and 8
// contracted indices.  Output element o of slot s is
//   sum over members m of slot s, sum over contracted c, prod_k M(A^{m,k})[...]
// (a slot is one output; regular plans have one member per slot, adjoint
// plans may sum several).
// ---------------------------------------------------------------------------
#define BES_GEN_MAX_OPS 4
#define BES_GEN_MAX_IDX 8
#define BES_GEN_MAX_B 16

// GEN_ELEMENTWISE reads one source, GEN_ELEMENTWISE2 adds a second source;
// GEN_TET is S0[pos0] - S0[pos1] (both positions in the first source);
// GEN_EXPR is expression body `op` of the plan at (S0[pos0], S1[pos1]).
enum { GEN_ARRAY = 0, GEN_ELEMENTWISE = 1, GEN_TET = 2, GEN_ELEMENTWISE2 = 3, GEN_EXPR = 4 };

typedef struct GenLayout {
  int32_t kind, op;
  double alpha, beta;
  int64_t off0, off1;
  int64_t so0[BES_GEN_MAX_IDX], sc0[BES_GEN_MAX_IDX];  // source 0 strides per
  int64_t so1[BES_GEN_MAX_IDX], sc1[BES_GEN_MAX_IDX];  // output / contracted idx
} GenLayout;

// The contracted indices are ordered: first the n_sh "shared" ones (each in
// at least two operands), then, for each operand k, the ex_n[k] indices that
// only operand k carries (positions ex_off[k] ...).  An exclusive index is
// summed inside its operand before the product is taken,
//   sum_{shared} prod_k ( sum_{exclusive of k} M(A^k)[...] ),
// the same value as Eq. (1) in a factored order; an operand without shared
// indices (row_dep bit clear) is summed once per output.
typedef struct GenEinsum {
  int32_t n_ops, n_out, n_con, b, n_slots;
  int32_t lanes;             // lanes cooperating on one output (1..64)
  int32_t tile;              // outputs per work item
  int32_t n_sh;              // shared contracted indices (first in con order)
  int64_t out_ext[BES_GEN_MAX_IDX], con_ext[BES_GEN_MAX_IDX];
  int64_t out_size, con_size;
  int64_t sh_size;                       // product of the shared extents
  int32_t ex_off[BES_GEN_MAX_OPS], ex_n[BES_GEN_MAX_OPS];
  int64_t ex_size[BES_GEN_MAX_OPS];      // product of operand k's exclusive extents
  int32_t row_dep;                       // bit k: operand k carries a shared index
  int32_t split;                         // chunks of the shared space per output
                                         // (> 1: chunks add into zeroed outputs)
  // Output slot s is written at o_off[s] + sum_d idx_d * o_str[s][d] (dense
  // row-major unless the caller set a layout); o_acc[s] != 0 adds into it
  // (atomically: slots may share memory).
  int64_t o_off[BES_GEN_MAX_B];
  int64_t o_str[BES_GEN_MAX_B][BES_GEN_MAX_IDX];
  int32_t o_acc[BES_GEN_MAX_B];
  int32_t o_dense;                       // every slot dense, offset 0, overwrite
  // Division by the extents with precomputed multipliers: for a dividend
  // x < 2^31, x / ext = (umulhi(x, mul) + x) >> shift (round-up method of
  // Granlund and Montgomery).  `narrow`: every linear index of the
  // descriptor is below 2^31, so the kernels decode with these 32-bit
  // multiplications instead of 64-bit divisions.
  int32_t narrow;
  uint32_t out_mul[BES_GEN_MAX_IDX], con_mul[BES_GEN_MAX_IDX];
  int32_t out_shift[BES_GEN_MAX_IDX], con_shift[BES_GEN_MAX_IDX];
  int32_t layout[BES_GEN_MAX_B][BES_GEN_MAX_OPS];  // layout id per (member, op)
  int32_t slot_of[BES_GEN_MAX_B];                  // member -> output slot
  int32_t slot_m0[BES_GEN_MAX_B], slot_m1[BES_GEN_MAX_B];  // members of slot,
  int32_t slot_members[BES_GEN_MAX_B];             // listed contiguously
  int32_t n_layouts;
  int32_t pad2;
  GenLayout lay[BES_GEN_MAX_B * BES_GEN_MAX_OPS];
} GenEinsum;

typedef struct GenPtrs {
  const void *src[BES_GEN_MAX_B][BES_GEN_MAX_OPS][2];
  void *out[BES_GEN_MAX_B];
} GenPtrs;

// Work item of the persistent batched launch: one tile of one slot of one
// einsum.
typedef struct GenItem {
  int32_t einsum;   // index into the descriptor table
  int32_t slot;
  int64_t first;    // first output element of the tile
  int64_t count;    // outputs in the tile
  int32_t chunk;    // chunk of the shared contracted space (0..split-1)
  int32_t pad;
} GenItem;

// ---------------------------------------------------------------------------
// MFMA template: C_m[M, N] (+)= sum_{members m of the slot} A_m[M, K] B_m[K, N]
// where each of M, N, K is a group of indices that merges into one strided
// axis in every operand.  FP32 in, FP32 accumulate.
// ---------------------------------------------------------------------------
#define BES_MFMA_MAX_B 8

typedef struct MfmaMember {
  const float *A;
  const float *B;
  int64_t sam, sak;   // A strides (M, K)
  int64_t sbk, sbn;   // B strides (K, N)
} MfmaMember;

typedef struct MfmaSlot {
  float *C;
  int64_t scm, scn;
  int32_t m0, m1;     // members [m0, m1) are summed into C
  int32_t acc;        // add into C instead of overwriting it
  int32_t pad;
} MfmaSlot;

typedef struct MfmaArgs {
  int64_t M, N, K;
  int32_t n_members, n_slots;
  MfmaMember mem[BES_MFMA_MAX_B];
  MfmaSlot slot[BES_MFMA_MAX_B];
} MfmaArgs;

// ---------------------------------------------------------------------------
// GETT template: a general binary contraction on the matrix cores,
//   C_s[M, N] (+)= sum over members m of slot s of
//                  sum_K (alpha_A A_m[M, K] + beta_A) (alpha_B B_m[K, N] + beta_B)
// where M, N and K are arbitrary groups of indices with arbitrary strides:
// operand addresses come from offset tables, row and column offsets added
// (address of A[m, k] = rowA[m] + colA[k]).  The affine operands are the
// linear polynomials of arrays of Section "TCCG Benchmark suite with
// Unmaterialized Operands".
// ---------------------------------------------------------------------------
#define BES_GETT_MAX_B 8

typedef struct GettMember {
  const void *A;
  const void *B;
  int64_t rowA, colA, rowB, colB;   // table offsets (int64 entries) in `tab`
  double a_alpha, a_beta, b_alpha, b_beta;
  int32_t a_kfast;                  // A's tile is read along K (else along M)
  int32_t b_nfast;                  // B's tile is read along N (else along K)
} GettMember;

typedef struct GettSlot {
  void *C;
  int64_t rowC, colC;               // table offsets in `tab`
  int32_t m0, m1;                   // members [m0, m1) are summed into C
  int32_t acc;                      // add into C instead of overwriting it
  int32_t pad;
} GettSlot;

typedef struct GettArgs {
  int64_t M, N, K;
  const int64_t *tab;               // device offset tables
  int32_t n_members, n_slots;
  int32_t ksplit;                   // K ranges per output tile (> 1: partial
                                    // tiles add atomically into C, or go to
                                    // `partial` and a second kernel sums them)
  int32_t pad;
  void *partial;                    // [ksplit][n_slots][M][N] partial tiles, or NULL
  GettMember mem[BES_GETT_MAX_B];
  GettSlot slot[BES_GETT_MAX_B];
} GettArgs;
