// Plans: a registered batched einsum with its canonical form, tuning config,
// and the analysis each kernel template needs (roles of the canonical indices
// and operand positions).  Binding turns a plan plus the caller's pointers
// into a launch descriptor.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../desc.h"
#include "canon.h"
#include "spec.h"

namespace bes {

// FEM-stream roles, on the canonical form (see desc.h for the computation).
// cls 0, the local-gradient class: T = S.U then out = G.T (desc.h FemArgs).
// cls 1, the "apply" class (face mass, local divergence): W = G.U per
// element, then out = S.W (desc.h FemApplyArgs); r is the index c that S and
// G share, x the component index of U and G (the same index as c when
// `diag`, the face-mass case).
struct FemRoles {
  int cls = 0;
  bool diag = false;
  int e = -1, i = -1, j = -1, r = -1, x = -1;  // canonical index ordinals
  int NI = 1, NJ = 1, NR = 1, NX = 1;
  int posS = -1, posU = -1, posG = -1;         // canonical positions
};

// MFMA roles: C[M, N] = A[M, K] B[K, N] with merged index groups.
struct MfmaRoles {
  std::vector<int> Mi, Ni, Ki;  // canonical index ordinals, in merge order
  int posA = -1, posB = -1;
  bool c_mn = true;             // output order is (M group, N group)
  int64_t M = 0, N = 0, K = 0;
};

// Where a launch writes output slot s: element offset and strides along the
// output indices in the notation's output order, and whether it adds into the
// existing values.  Default: offset 0, dense row-major, overwrite.
struct OutLayout {
  bool custom = false;      // false: dense row-major, offset 0
  int64_t offset = 0;
  int64_t stride[BES_MAX_DIM] = {0};
  bool accumulate = false;
};

inline bool same_layout(const OutLayout &a, const OutLayout &b) {
  if (a.custom != b.custom || a.accumulate != b.accumulate) return false;
  if (!a.custom) return true;
  if (a.offset != b.offset) return false;
  for (int d = 0; d < BES_MAX_DIM; ++d)
    if (a.stride[d] != b.stride[d]) return false;
  return true;
}

inline bool same_layouts(const std::vector<OutLayout> &a, const std::vector<OutLayout> &b) {
  if (a.size() != b.size()) return false;
  for (size_t k = 0; k < a.size(); ++k)
    if (!same_layout(a[k], b[k])) return false;
  return true;
}

// GETT roles: C[M, N] = sum_K A[M, K] B[K, N] with index groups of any
// strides (M and N in output order, K in A's axis order).
struct GettRoles {
  std::vector<int> Mi, Ni, Ki;  // canonical index ordinals
  int posA = -1, posB = -1;
  int64_t M = 1, N = 1, K = 1;
};

struct Plan {
  Spec spec;
  Canonical canon;
  std::string key, tuple;
  bes_config cfg{};
  bool cfg_from_db = false;

  bool fem_ok = false;
  std::string fem_why;
  FemRoles fem;
  bool mfma_ok = false;
  std::string mfma_why;
  MfmaRoles mf;
  bool gett_ok = false;
  std::string gett_why;
  GettRoles gt;

  // Output slots: member (user order) -> slot.  Regular plans: identity.
  // Adjoint plans sum the members of a slot.
  std::vector<int> slot_of_member;
  int n_slots = 0;
  // Flattened source pointers: arg a's sources start at src_base[a].
  std::vector<int> src_base;
  int n_src = 0;
  // For adjoint plans: this plan's flat source k is the caller's src_from[k].
  std::vector<int> src_from;
  bool adjoint = false;
  // Output layouts per slot (bes_plan_set_output).
  std::vector<OutLayout> out_layout;
  // Distinct expression bodies of BES_EXPR arguments (GenLayout::op indexes
  // this list); such plans run the generic template built at run time.
  std::vector<std::string> exprs;

  // FEM-stream workspace for the packed shared operand (first FEM launch).
  mutable void *fem_ws = nullptr;
  mutable int fem_ws_device = -1;
  // GETT workspace for the partial tiles of a K-split launch (first GETT
  // launch; fixed size, never regrown while launches may read it).
  mutable void *gett_ws = nullptr;
  mutable size_t gett_ws_bytes = 0;
  mutable int gett_ws_device = -1;
  // Generic descriptors bound so far, one per (config, output layouts,
  // device): a pinned host copy and the device copy uploaded from it.  Kept
  // until the plan is destroyed, so a launch never waits for or frees a
  // descriptor an earlier launch may still read.
  struct GenCopy {
    bes_config cfg{};
    std::vector<OutLayout> layouts;
    int device = -1;
    GenEinsum *host = nullptr;   // pinned
    GenEinsum *dev = nullptr;
  };
  mutable std::vector<GenCopy> gen_cache;
  // GETT offset tables, one device copy per (output layouts, device).
  struct GettCopy {
    std::vector<OutLayout> layouts;
    int device = -1;
    GettArgs args{};            // table offsets, flags and scalars; no pointers
    int64_t *dev = nullptr;
  };
  mutable std::vector<GettCopy> gett_cache;
  // Profiling hook (bes_plan_set_timing): events recorded around the main
  // evaluation kernel(s) of every launch; caller-owned hipEvent_t handles.
  void *time_start = nullptr;
  void *time_stop = nullptr;
};

// Analyse a registered spec: canonicalize, fill roles, default config.
int build_plan(Plan &p, std::string &err);

// Templates able to evaluate the plan.
bool template_supported(const Plan &p, int template_id);
bes_config default_config(const Plan &p);

// Binders.  `src` are the plan's flat source pointers (after src_from
// remapping), `out` one pointer per slot.
int bind_fem(const Plan &p, const void *const *src, void *const *out, FemArgs &a,
             std::string &err);
int bind_fem_apply(const Plan &p, const void *const *src, void *const *out, FemApplyArgs &a,
                   std::string &err);
int bind_generic_static(const Plan &p, const bes_config &cfg, GenEinsum &g, std::string &err);
int bind_generic_ptrs(const Plan &p, const void *const *src, void *const *out, GenPtrs &ptrs);
int bind_mfma(const Plan &p, const void *const *src, void *const *out, MfmaArgs &a,
              std::string &err);
// GETT: the offset tables (host copy) and the pointer-free part of the
// arguments; then the caller's pointers.
int bind_gett_static(const Plan &p, std::vector<int64_t> &tables, GettArgs &a,
                     std::string &err);
void bind_gett_ptrs(const Plan &p, const void *const *src, void *const *out, GettArgs &a);

// Dense row-major strides of the output in the notation's order.
std::vector<int64_t> dense_out_strides(const Plan &p);
// Strides of slot `slot` along the user's output indices (custom or dense).
std::vector<int64_t> out_strides(const Plan &p, int slot);
// True when no slot has a custom layout or accumulates.
bool outputs_plain(const Plan &p);
bool any_accumulate(const Plan &p);

// Build the adjoint plan of position `pos` (see bes_adjoint in bes.h).
int build_adjoint(const Plan &fwd, int pos, Plan &adj, int &n_out, std::string &err);

}  // namespace bes
