// Launchers of the HIP kernel templates (gfx950).  Each returns hipSuccess or
// the HIP error of the failed call; none synchronizes.
#pragma once

#include <hip/hip_runtime.h>

#include "../desc.h"
#include "../fem_shapes.h"

namespace bes {

// Compute units of the current device (cached per device).
int device_cu_count();

// FEM-stream template: a pack of S into `workspace` (at least
// fem_workspace_bytes) followed by the stream kernel with `blocks_per_cu`
// blocks per compute unit walking 64-element tiles.  `variant`: 0 runs plain
// batches (one stage-1 group, one output component per member) on the lean
// kernel with two waves per tile, 2 on the lean kernel with one wave per
// tile, 1 always on the descriptor-driven kernel.
size_t fem_workspace_bytes(bool f64, int NI, int NJ, int NR);
// `ev_start` / `ev_stop` (may be NULL) are recorded on `stream` right before
// and after the stream kernel(s), after the re-layout of S.
hipError_t launch_fem(bool f64, int NI, int NJ, int NR, int NX, const FemArgs &a, void *workspace,
                      int blocks_per_cu, int variant, hipStream_t stream,
                      hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);

// FEM-stream "apply" class (face mass, local divergence): one launch over
// (64-element tile, member) work items; a grid of at most `blocks_per_cu`
// blocks of four waves per compute unit.  `variant` 0 or 1 keeps S in LDS,
// 2 reads it as scalar operands from a copy re-laid into `workspace` (at
// least fem_apply_workspace_bytes).  Events as for launch_fem.
size_t fem_apply_workspace_bytes(bool f64, int NI, int NJ, int NC);
hipError_t launch_fem_apply(bool f64, int NI, int NJ, int NC, int NX, bool diag,
                            const FemApplyArgs &a, void *workspace, int blocks_per_cu,
                            int variant, hipStream_t stream, hipEvent_t ev_start = nullptr,
                            hipEvent_t ev_stop = nullptr);

// Generic template: one launch over (slot, tile) pairs.  `dev` is the device
// copy of `host`.
hipError_t launch_generic(bool f64, const GenEinsum *dev, const GenEinsum &host,
                          const GenPtrs &ptrs, hipStream_t stream);

// Persistent batched launch: blocks pull GenItems off a device counter.
// `table`/`ptrs` are device arrays indexed by einsum; counters[2] must be zero
// before the first launch and are left zero by every launch.
// Einsums with split > 1 get their outputs zeroed by a kernel first
// (`any_split`), then their chunks add into them.
// `narrow`: every descriptor of the table is narrow (32-bit decoding).
hipError_t launch_persistent(bool f64, const GenEinsum *table, const GenPtrs *ptrs,
                             const GenItem *items, int n_items, unsigned *counters,
                             int grid, hipStream_t stream, int n_einsums, bool any_split,
                             bool narrow);

// Zero n elements of 4 or 8 bytes at p (a fill kernel: no memset node, so a
// captured graph replays it correctly).
hipError_t launch_fill_zero(void *p, int64_t n, int elem_bytes, hipStream_t stream);

// GETT template (FP32 / FP64 matrix cores): `a.tab` points to the device
// offset tables the host built for the plan.  `shape` = tile shape (1: 16 x
// 128, 2: 32 x 128, 3: 128 x 32, 4: 128 x 16, 5: 64 x 64; 0: by the output's
// extents).  `ksplit` = K ranges per output tile (0: chosen from the tile
// count and K; > 1 zeroes the overwritten outputs first, then adds partial
// tiles atomically).
hipError_t launch_gett(bool f64, const GettArgs &a, int shape, int ksplit, void *workspace,
                       size_t workspace_bytes, hipStream_t stream);

// MFMA dense-contraction template (FP32).  mfma_args_ok: the shape and the
// alignment of every operand fit the template's vector tile loads.
bool mfma_args_ok(const MfmaArgs &a);
hipError_t launch_mfma(const MfmaArgs &a, int tile_m, int tile_n, hipStream_t stream);

}  // namespace bes
