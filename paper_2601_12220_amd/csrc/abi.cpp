// C ABI of the batched-einsum library (declared in include/bes.h).
//
// Registration, canonicalization, tuning lookup and binding are host-only and
// make no HIP call, so they run on machines without a GPU.  Launch entry
// points enqueue hand-written HIP kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/bes.h"
#include "host/canon.h"
#include "host/db.h"
#include "host/graph.h"
#include "host/plan.h"
#include "host/spec.h"
#include "jit.h"
#include "kernels/kernels.h"

struct bes_ctx {
  bes::TuningDB db;
};

struct bes_plan {
  bes::Plan p;
};

struct bes_batch {
  std::vector<const bes::Plan *> plans;
  bool f64 = false;
  int n_items = 0;
  int grid = 0;
  int device = -1;
  GenEinsum *d_table = nullptr;
  GenPtrs *d_ptrs = nullptr;
  GenItem *d_items = nullptr;
  unsigned *d_counters = nullptr;
  GenPtrs *h_ptrs = nullptr;  // pinned staging for pointer updates
  std::vector<GenPtrs> last;
  bool have_last = false;
  hipEvent_t staged = nullptr;
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool use_graph = true;
  bool any_split = false;
  bool narrow = true;   // every plan's descriptor decodes in 32 bits
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

int copy_out(const std::string &s, char *buf, size_t cap, size_t *len) {
  if (len) *len = s.size();
  if (!buf) return cap == 0 ? BES_OK : fail(BES_E_INVALID, "NULL buffer with non-zero capacity");
  if (cap < s.size() + 1) return fail(BES_E_BUFFER, "buffer too small");
  std::memcpy(buf, s.c_str(), s.size() + 1);
  return BES_OK;
}

const char *kDefaultArch = "gfx950";

int apply_lookup(bes_ctx *ctx, bes::Plan &p, const std::string &arch) {
  p.cfg = bes::default_config(p);
  p.cfg_from_db = false;
  if (!ctx) return BES_W_NOTFOUND;
  const bes::TuningRecord *r = ctx->db.find(p.key, arch);
  if (r && bes::template_supported(p, r->cfg.template_id)) {
    p.cfg = r->cfg;
    p.cfg_from_db = true;
    ++ctx->db.hits;
    return BES_OK;
  }
  ++ctx->db.misses;
  return BES_W_NOTFOUND;
}

bool env_flag(const char *name) {
  const char *s = std::getenv(name);
  return s && *s && std::strcmp(s, "0") != 0;
}

// The plan's generic descriptor for `cfg` and its current output layouts on
// the current device: bound once into pinned host memory and uploaded with an
// asynchronous copy on `stream` (ordered before the kernel that reads it).
// Entries live until the plan is destroyed.
int generic_descriptor(const bes::Plan &p, const bes_config &cfg, hipStream_t stream,
                       const bes::Plan::GenCopy **out, std::string &err) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    err = std::string("hipGetDevice: ") + hipGetErrorString(e);
    return BES_E_HIP;
  }
  for (const auto &c : p.gen_cache)
    if (c.device == dev && bes::same_layouts(c.layouts, p.out_layout) &&
        std::memcmp(&c.cfg, &cfg, sizeof cfg) == 0) {
      *out = &c;
      return BES_OK;
    }
  bes::Plan::GenCopy c;
  c.cfg = cfg;
  c.layouts = p.out_layout;
  c.device = dev;
  if ((e = hipHostMalloc((void **)&c.host, sizeof(GenEinsum))) != hipSuccess) {
    err = std::string("pinned descriptor: ") + hipGetErrorString(e);
    return BES_E_NOMEM;
  }
  int rc = bes::bind_generic_static(p, cfg, *c.host, err);
  if (rc) {
    (void)hipHostFree(c.host);
    return rc;
  }
  if ((e = hipMalloc((void **)&c.dev, sizeof(GenEinsum))) != hipSuccess ||
      (e = hipMemcpyAsync(c.dev, c.host, sizeof(GenEinsum), hipMemcpyHostToDevice, stream)) !=
          hipSuccess) {
    if (c.dev) (void)hipFree(c.dev);
    (void)hipHostFree(c.host);
    err = std::string("generic descriptor upload: ") + hipGetErrorString(e);
    return BES_E_HIP;
  }
  p.gen_cache.push_back(c);
  *out = &p.gen_cache.back();
  return BES_OK;
}

// The plan's GETT offset tables for its current output layouts on the
// current device: built on the host and uploaded once (the first launch of
// a layout allocates and copies synchronously; later launches reuse them).
int gett_tables(const bes::Plan &p, const bes::Plan::GettCopy **out, std::string &err) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    err = std::string("hipGetDevice: ") + hipGetErrorString(e);
    return BES_E_HIP;
  }
  for (const auto &c : p.gett_cache)
    if (c.device == dev && bes::same_layouts(c.layouts, p.out_layout)) {
      *out = &c;
      return BES_OK;
    }
  bes::Plan::GettCopy c;
  c.layouts = p.out_layout;
  c.device = dev;
  std::vector<int64_t> tab;
  int rc = bes::bind_gett_static(p, tab, c.args, err);
  if (rc) return rc;
  const size_t bytes = std::max<size_t>(tab.size(), 1) * sizeof(int64_t);
  if ((e = hipMalloc((void **)&c.dev, bytes)) != hipSuccess ||
      (e = hipMemcpy(c.dev, tab.data(), tab.size() * sizeof(int64_t), hipMemcpyHostToDevice)) !=
          hipSuccess) {
    if (c.dev) (void)hipFree(c.dev);
    err = std::string("GETT table upload: ") + hipGetErrorString(e);
    return BES_E_HIP;
  }
  p.gett_cache.push_back(c);
  *out = &p.gett_cache.back();
  return BES_OK;
}

void free_gen_cache(const bes::Plan &p) {
  for (auto &c : p.gett_cache)
    if (c.dev) (void)hipFree(c.dev);
  p.gett_cache.clear();
  for (auto &c : p.gen_cache) {
    if (c.dev) (void)hipFree(c.dev);
    if (c.host) (void)hipHostFree(c.host);
  }
  p.gen_cache.clear();
}

// Byte range [lo, hi) that output slot s of a launch touches.
void slot_range(const bes::Plan &p, int s, const void *base, uintptr_t &lo, uintptr_t &hi) {
  const int64_t item = p.spec.dtype == BES_FLOAT64 ? 8 : 4;
  const std::vector<int64_t> st = bes::out_strides(p, s);
  int64_t a = p.out_layout[s].custom ? p.out_layout[s].offset : 0, b = a;
  for (size_t d = 0; d < p.spec.out.size(); ++d) {
    const int64_t span = (p.spec.extent[p.spec.out[d]] - 1) * st[d];
    if (span < 0) a += span;
    else b += span;
  }
  lo = (uintptr_t)base + a * item;
  hi = (uintptr_t)base + (b + 1) * item;
}

// Do two accumulating slots of this launch address overlapping memory?
bool accumulating_slots_overlap(const bes::Plan &p, void *const *out) {
  if (!bes::any_accumulate(p) || p.n_slots < 2) return false;
  std::vector<uintptr_t> lo(p.n_slots), hi(p.n_slots);
  for (int s = 0; s < p.n_slots; ++s) slot_range(p, s, out[s], lo[s], hi[s]);
  for (int s = 0; s < p.n_slots; ++s)
    for (int t = s + 1; t < p.n_slots; ++t)
      if (lo[s] < hi[t] && lo[t] < hi[s]) return true;
  return false;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(BES_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Scratch of the entry point that allocates nothing (bes_launch_noalloc): a
// fixed device array per GPU holding the re-laid shared operand of the
// FEM-stream template.  In host code `scratch` names a host-side stand-in;
// kernels get the device address that hipGetSymbolAddress returns for the
// current device, looked up once per device.
constexpr size_t kScratchBytes = 256 * 1024;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {nullptr};

int scratch_of_current_device(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(BES_E_UNSUPPORTED, "device ordinal >= 64");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return BES_OK;
}

}  // namespace

extern "C" {

const char *bes_last_error(void) { return g_err.c_str(); }

int bes_ctx_create(bes_ctx **out, const char *tuning_db_path) {
  if (!out) return fail(BES_E_INVALID, "out is NULL");
  *out = nullptr;
  bes_ctx *c = new (std::nothrow) bes_ctx;
  if (!c) return fail(BES_E_NOMEM, "out of host memory");
  std::string err;
  int rc = c->db.open(tuning_db_path, err);
  if (rc) {
    delete c;
    return fail(rc, err);
  }
  *out = c;
  return BES_OK;
}

void bes_ctx_destroy(bes_ctx *ctx) { delete ctx; }

int bes_register(bes_ctx *ctx, const char *notation, int32_t b, int32_t n, int32_t n_args,
                 const bes_operand *args, const int32_t *table, bes_plan **out) {
  return bes_register_expr(ctx, notation, b, n, n_args, args, table, nullptr, out);
}

int bes_register_expr(bes_ctx *ctx, const char *notation, int32_t b, int32_t n,
                      int32_t n_args, const bes_operand *args, const int32_t *table,
                      const char *const *exprs, bes_plan **out) {
  if (!out) return fail(BES_E_INVALID, "out is NULL");
  *out = nullptr;
  try {
    bes_plan *P = new bes_plan;
    std::string err;
    int rc = bes::make_spec(notation, b, n, n_args, args, table, P->p.spec, err, exprs);
    if (rc == BES_OK) rc = bes::build_plan(P->p, err);
    if (rc != BES_OK) {
      delete P;
      return fail(rc, err);
    }
    rc = apply_lookup(ctx, P->p, kDefaultArch);
    *out = P;
    return rc;
  } catch (const std::bad_alloc &) {
    return fail(BES_E_NOMEM, "out of host memory");
  }
}

void bes_plan_destroy(bes_plan *plan) {
  if (!plan) return;
  free_gen_cache(plan->p);
  if (plan->p.fem_ws) (void)hipFree(plan->p.fem_ws);
  if (plan->p.gett_ws) (void)hipFree(plan->p.gett_ws);
  delete plan;
}

int bes_plan_key(const bes_plan *plan, char *buf, size_t cap, size_t *len) {
  if (!plan) return fail(BES_E_INVALID, "plan is NULL");
  return copy_out(plan->p.key, buf, cap, len);
}

int bes_plan_canonical(const bes_plan *plan, char *buf, size_t cap, size_t *len) {
  if (!plan) return fail(BES_E_INVALID, "plan is NULL");
  return copy_out(plan->p.tuple, buf, cap, len);
}

int bes_plan_maps(const bes_plan *plan, int32_t *member_map, int32_t *pos_map, int32_t *arg_map,
                  char *index_map, int32_t *n_index) {
  if (!plan) return fail(BES_E_INVALID, "plan is NULL");
  const bes::Canonical &c = plan->p.canon;
  if (member_map) std::copy(c.member_map.begin(), c.member_map.end(), member_map);
  if (pos_map) std::copy(c.pos_map.begin(), c.pos_map.end(), pos_map);
  if (arg_map) std::copy(c.arg_map.begin(), c.arg_map.end(), arg_map);
  if (index_map)
    for (size_t k = 0; k < c.index_map.size(); ++k) index_map[k] = (char)('a' + c.index_map[k]);
  if (n_index) *n_index = (int32_t)c.index_map.size();
  return BES_OK;
}

int bes_plan_graph(const bes_plan *plan, int32_t which, int32_t *n_nodes, uint8_t *adj,
                   int32_t *colors) {
  if (!plan) return fail(BES_E_INVALID, "plan is NULL");
  const bes::Digraph &g = which ? plan->p.canon.canon_graph : plan->p.canon.induced.g;
  if (n_nodes) *n_nodes = g.n;
  if (adj) {
    auto d = g.dense();
    std::memcpy(adj, d.data(), d.size());
  }
  if (colors) std::copy(g.color.begin(), g.color.end(), colors);
  return BES_OK;
}

int bes_check_compliance(int32_t n, const uint8_t *adj, const int32_t *colors) {
  if (n < 0 || (n > 0 && (!adj || !colors))) return fail(BES_E_INVALID, "bad graph");
  bes::Digraph g = bes::Digraph::from_dense(n, adj, colors);
  return bes::check_compliance(g);
}

int bes_canonical_labeling(int32_t n, const uint8_t *adj, const int32_t *colors, int32_t *label) {
  if (n < 0 || (n > 0 && (!adj || !colors || !label))) return fail(BES_E_INVALID, "bad graph");
  bes::Digraph g = bes::Digraph::from_dense(n, adj, colors);
  std::vector<int> lab = bes::canonical_labeling(g);
  std::copy(lab.begin(), lab.end(), label);
  return BES_OK;
}

int bes_plan_lookup(bes_ctx *ctx, bes_plan *plan, const char *arch) {
  if (!plan) return fail(BES_E_INVALID, "plan is NULL");
  return apply_lookup(ctx, plan->p, arch ? arch : kDefaultArch);
}

int bes_plan_get_config(const bes_plan *plan, bes_config *cfg) {
  if (!plan || !cfg) return fail(BES_E_INVALID, "NULL argument");
  *cfg = plan->p.cfg;
  return BES_OK;
}

int bes_plan_set_config(bes_plan *plan, const bes_config *cfg) {
  if (!plan || !cfg) return fail(BES_E_INVALID, "NULL argument");
  bes_config c = *cfg;
  if (c.template_id == BES_T_AUTO) c = bes::default_config(plan->p);
  if (!bes::template_supported(plan->p, c.template_id))
    return fail(BES_E_UNSUPPORTED, "template cannot evaluate this plan");
  if (c.template_id == BES_T_GENERIC) {
    int lanes = c.p[1] > 0 ? c.p[1] : 1;
    if (lanes > 64 || (lanes & (lanes - 1))) return fail(BES_E_INVALID, "lanes must be 2^k <= 64");
    if (c.p[0] < 0) return fail(BES_E_INVALID, "negative tile");
  }
  if (c.template_id == BES_T_FEM_STREAM) {
    if (c.p[1] < 0 || c.p[1] > 64) return fail(BES_E_INVALID, "blocks per CU must be 0..64");
    if (c.p[2] < 0 || c.p[2] > 3) return fail(BES_E_INVALID, "FEM kernel variant must be 0, 1, 2 or 3");
  }
  plan->p.cfg = c;
  return BES_OK;
}

int bes_db_record(bes_ctx *ctx, const char *key, const char *arch, const bes_config *cfg,
                  double seconds) {
  if (!ctx || !key || !arch || !cfg) return fail(BES_E_INVALID, "NULL argument");
  std::string err;
  int rc = ctx->db.record(key, arch, *cfg, seconds, err);
  return rc ? fail(rc, err) : BES_OK;
}

int bes_ctx_stats(const bes_ctx *ctx, int64_t *hits, int64_t *misses) {
  if (!ctx) return fail(BES_E_INVALID, "ctx is NULL");
  if (hits) *hits = ctx->db.hits;
  if (misses) *misses = ctx->db.misses;
  return BES_OK;
}

int bes_plan_set_timing(bes_plan *plan, void *start_event, void *stop_event) {
  if (!plan) return fail(BES_E_INVALID, "NULL plan");
  if ((start_event == nullptr) != (stop_event == nullptr))
    return fail(BES_E_INVALID, "give both events or neither");
  plan->p.time_start = start_event;
  plan->p.time_stop = stop_event;
  return BES_OK;
}

int bes_launch(const bes_plan *plan, const void *const *src_ptrs, void *const *out_ptrs,
               void *hip_stream) {
  if (!plan || !src_ptrs || !out_ptrs) return fail(BES_E_INVALID, "NULL argument");
  const bes::Plan &p = plan->p;
  hipStream_t stream = (hipStream_t)hip_stream;
  std::vector<const void *> src(p.n_src);
  for (int k = 0; k < p.n_src; ++k) src[k] = p.adjoint ? src_ptrs[p.src_from[k]] : src_ptrs[k];
  // NULL is accepted only for empty operands and outputs.
  for (size_t a = 0; a < p.spec.args.size(); ++a) {
    const bes::Operand &o = p.spec.args[a];
    int64_t sz = 1;
    for (int d = 0; d < o.ndim; ++d) sz *= o.shape[d];
    for (int s = 0; s < o.nsrc; ++s)
      if (!src[p.src_base[a] + s] && sz != 0) return fail(BES_E_INVALID, "NULL source pointer");
  }
  int64_t out_size = 1;
  for (int c : p.spec.out) out_size *= p.spec.extent[c];
  for (int s = 0; s < p.n_slots; ++s)
    if (!out_ptrs[s] && out_size != 0) return fail(BES_E_INVALID, "NULL output pointer");
  const bool f64 = p.spec.dtype == BES_FLOAT64;
  std::string err;
  hipError_t e;
  auto record = [&](void *ev) -> hipError_t {
    return ev ? hipEventRecord((hipEvent_t)ev, stream) : hipSuccess;
  };
  // The generic template evaluates every plan within its limits and honours
  // every output layout; the others hand over to it where they cannot.
  auto run_generic = [&](bes_config gc) -> int {
    if (gc.template_id != BES_T_GENERIC) {
      gc = bes_config{};
      gc.template_id = BES_T_GENERIC;
      gc.p[0] = 256;
      gc.p[1] = 1;
    }
    const bes::Plan::GenCopy *gd = nullptr;
    int rc = generic_descriptor(p, gc, stream, &gd, err);
    if (rc) return fail(rc, err);
    GenPtrs ptrs;
    bes::bind_generic_ptrs(p, src.data(), out_ptrs, ptrs);
    bes::JitKernels jk;
    if (!p.exprs.empty() && (rc = bes::jit_generic(f64, p.exprs, &jk, err)) != BES_OK)
      return fail(rc, err);
    if ((e = record(p.time_start)) != hipSuccess) return hip_fail(e, "timing event");
    e = p.exprs.empty() ? bes::launch_generic(f64, gd->dev, *gd->host, ptrs, stream)
                        : bes::launch_generic_jit(jk, gd->dev, *gd->host, ptrs, stream);
    if (e != hipSuccess) return hip_fail(e, "generic launch");
    if ((e = record(p.time_stop)) != hipSuccess) return hip_fail(e, "timing event");
    return BES_OK;
  };
  switch (p.cfg.template_id) {
    case BES_T_FEM_STREAM: {
      if (bes::any_accumulate(p)) return run_generic(p.cfg);
      int dev = 0;
      if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e, "hipGetDevice");
      if (p.fem_ws && p.fem_ws_device != dev) {
        (void)hipFree(p.fem_ws);
        p.fem_ws = nullptr;
      }
      if (!p.fem_ws) {   // re-laid S (both classes; sized for the larger need)
        size_t bytes = bes::fem_workspace_bytes(f64, p.fem.NI, p.fem.NJ, p.fem.NR);
        if ((e = hipMalloc(&p.fem_ws, bytes)) != hipSuccess) {
          p.fem_ws = nullptr;
          return hip_fail(e, "FEM workspace allocation");
        }
        p.fem_ws_device = dev;
      }
      if (p.fem.cls == 1) {
        FemApplyArgs a;
        int rc = bes::bind_fem_apply(p, src.data(), out_ptrs, a, err);
        if (rc) return fail(rc, err);
        e = bes::launch_fem_apply(f64, p.fem.NI, p.fem.NJ, p.fem.NR, p.fem.NX, p.fem.diag, a,
                                  p.fem_ws, p.cfg.p[1], p.cfg.p[2], stream,
                                  (hipEvent_t)p.time_start, (hipEvent_t)p.time_stop);
        if (e != hipSuccess) return hip_fail(e, "FEM-stream apply launch");
        return BES_OK;
      }
      FemArgs a;
      int rc = bes::bind_fem(p, src.data(), out_ptrs, a, err);
      if (rc) return fail(rc, err);
      e = bes::launch_fem(f64, p.fem.NI, p.fem.NJ, p.fem.NR, p.fem.NX, a, p.fem_ws, p.cfg.p[1],
                          p.cfg.p[2], stream, (hipEvent_t)p.time_start,
                          (hipEvent_t)p.time_stop);
      if (e != hipSuccess) return hip_fail(e, "FEM-stream launch");
      return BES_OK;
    }
    case BES_T_MFMA: {
      // accumulating slots that overlap in memory need the atomic adds of
      // the generic template
      if (accumulating_slots_overlap(p, out_ptrs)) return run_generic(p.cfg);
      MfmaArgs a;
      int rc = bes::bind_mfma(p, src.data(), out_ptrs, a, err);
      if (rc == BES_E_UNSUPPORTED) return run_generic(p.cfg);  // output layout
      if (rc) return fail(rc, err);
      if (!bes::mfma_args_ok(a)) return run_generic(p.cfg);  // unaligned rows
      if ((e = record(p.time_start)) != hipSuccess) return hip_fail(e, "timing event");
      e = bes::launch_mfma(a, p.cfg.p[0], p.cfg.p[1], stream);
      if (e != hipSuccess) return hip_fail(e, "MFMA launch");
      if ((e = record(p.time_stop)) != hipSuccess) return hip_fail(e, "timing event");
      return BES_OK;
    }
    case BES_T_GETT: {
      // overlapping accumulating outputs need the generic template's atomics
      if (accumulating_slots_overlap(p, out_ptrs)) return run_generic(p.cfg);
      const bes::Plan::GettCopy *gc = nullptr;
      int rc = gett_tables(p, &gc, err);
      if (rc) return fail(rc, err);
      GettArgs a = gc->args;
      a.tab = gc->dev;
      bes::bind_gett_ptrs(p, src.data(), out_ptrs, a);
      // partial tiles of a K split: up to 1024 ranges of every output, at
      // most 64 MiB (larger outputs split little and add atomically)
      {
        int dev = 0;
        if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e, "hipGetDevice");
        if (p.gett_ws && p.gett_ws_device != dev) {
          (void)hipFree(p.gett_ws);
          p.gett_ws = nullptr;
        }
        if (!p.gett_ws && p.cfg.p[4] == 1) {
          const size_t esz = f64 ? 8 : 4;
          const size_t one = (size_t)a.M * (size_t)a.N * (size_t)a.n_slots * esz;
          const size_t bytes = std::min<size_t>(one * 1024, (size_t)64 << 20);
          if (bytes >= one * 4) {
            if ((e = hipMalloc(&p.gett_ws, bytes)) != hipSuccess) {
              p.gett_ws = nullptr;
              return hip_fail(e, "GETT workspace allocation");
            }
            p.gett_ws_bytes = bytes;
            p.gett_ws_device = dev;
          }
        }
      }
      if ((e = record(p.time_start)) != hipSuccess) return hip_fail(e, "timing event");
      // p[4] = 1: a K split of eight or more ranges sums its partial tiles in
      // a second kernel (else they add atomically)
      const bool two_pass = p.cfg.p[4] == 1 && p.gett_ws;
      e = bes::launch_gett(f64, a, p.cfg.p[3], p.cfg.p[2], two_pass ? p.gett_ws : nullptr,
                           two_pass ? p.gett_ws_bytes : 0, stream);
      if (e != hipSuccess) return hip_fail(e, "GETT launch");
      if ((e = record(p.time_stop)) != hipSuccess) return hip_fail(e, "timing event");
      return BES_OK;
    }
    case BES_T_GENERIC:
      return run_generic(p.cfg);
    default:
      return fail(BES_E_UNSUPPORTED, "no kernel template evaluates this plan (dtype " +
                                         std::string(bes::dtype_name(p.spec.dtype)) + ")");
  }
}

int bes_launch_noalloc(const bes_plan *plan, const void *const *src_ptrs, void *const *out_ptrs,
                       void *hip_stream) {
  if (!plan || !src_ptrs || !out_ptrs) return fail(BES_E_INVALID, "NULL argument");
  const bes::Plan &p = plan->p;
  hipStream_t stream = (hipStream_t)hip_stream;
  std::vector<const void *> src(p.n_src);
  for (int k = 0; k < p.n_src; ++k) src[k] = p.adjoint ? src_ptrs[p.src_from[k]] : src_ptrs[k];
  const bool f64 = p.spec.dtype == BES_FLOAT64;
  std::string err;
  hipError_t e;
  auto record = [&](void *ev) -> hipError_t {
    return ev ? hipEventRecord((hipEvent_t)ev, stream) : hipSuccess;
  };
  switch (p.cfg.template_id) {
    case BES_T_FEM_STREAM: {
      if (bes::any_accumulate(p))
        return fail(BES_E_UNSUPPORTED, "no-alloc launch: the FEM-stream template overwrites");
      const size_t need = bes::fem_workspace_bytes(f64, p.fem.NI, p.fem.NJ, p.fem.NR);
      if (need > kScratchBytes)
        return fail(BES_E_UNSUPPORTED, "no-alloc launch: the shared operand needs " +
                                           std::to_string(need) + " bytes of scratch, more than " +
                                           std::to_string(kScratchBytes));
      if (p.fem.cls == 1) {
        FemApplyArgs a;
        int rc = bes::bind_fem_apply(p, src.data(), out_ptrs, a, err);
        if (rc) return fail(rc, err);
        void *ws = nullptr;
        if ((rc = scratch_of_current_device(&ws)) != BES_OK) return rc;
        e = bes::launch_fem_apply(f64, p.fem.NI, p.fem.NJ, p.fem.NR, p.fem.NX, p.fem.diag, a, ws,
                                  p.cfg.p[1], p.cfg.p[2], stream, (hipEvent_t)p.time_start,
                                  (hipEvent_t)p.time_stop);
        if (e != hipSuccess) return hip_fail(e, "FEM-stream apply launch");
        return BES_OK;
      }
      FemArgs a;
      int rc = bes::bind_fem(p, src.data(), out_ptrs, a, err);
      if (rc) return fail(rc, err);
      void *ws = nullptr;
      if ((rc = scratch_of_current_device(&ws)) != BES_OK) return rc;
      e = bes::launch_fem(f64, p.fem.NI, p.fem.NJ, p.fem.NR, p.fem.NX, a, ws, p.cfg.p[1],
                          p.cfg.p[2], stream, (hipEvent_t)p.time_start,
                          (hipEvent_t)p.time_stop);
      if (e != hipSuccess) return hip_fail(e, "FEM-stream launch");
      return BES_OK;
    }
    case BES_T_MFMA: {
      if (accumulating_slots_overlap(p, out_ptrs))
        return fail(BES_E_UNSUPPORTED, "no-alloc launch: accumulating outputs overlap");
      MfmaArgs a;
      int rc = bes::bind_mfma(p, src.data(), out_ptrs, a, err);
      if (rc) return fail(rc, err);
      if (!bes::mfma_args_ok(a))
        return fail(BES_E_UNSUPPORTED, "no-alloc launch: operands unaligned for the MFMA tiles");
      if ((e = record(p.time_start)) != hipSuccess) return hip_fail(e, "timing event");
      e = bes::launch_mfma(a, p.cfg.p[0], p.cfg.p[1], stream);
      if (e != hipSuccess) return hip_fail(e, "MFMA launch");
      if ((e = record(p.time_stop)) != hipSuccess) return hip_fail(e, "timing event");
      return BES_OK;
    }
    default:
      return fail(BES_E_UNSUPPORTED,
                  "no-alloc launch covers the FEM-stream and MFMA templates only");
  }
}

int bes_plan_set_output(bes_plan *plan, int32_t slot, int64_t offset, const int64_t *strides,
                        int32_t accumulate) {
  if (!plan) return fail(BES_E_INVALID, "NULL plan");
  bes::Plan &p = plan->p;
  if (slot < 0 || slot >= p.n_slots) return fail(BES_E_INVALID, "slot out of range");
  if (offset < 0) return fail(BES_E_INVALID, "negative offset");
  bes::OutLayout L;
  L.accumulate = accumulate != 0;
  if (strides || offset) {
    L.custom = true;
    L.offset = offset;
    const std::vector<int64_t> dense = bes::dense_out_strides(p);
    for (size_t d = 0; d < p.spec.out.size(); ++d) L.stride[d] = strides ? strides[d] : dense[d];
  }
  p.out_layout[slot] = L;
  return BES_OK;
}

int bes_fill_zero(void *ptr, int64_t n, int32_t dtype, void *hip_stream) {
  if (n < 0 || (n > 0 && !ptr)) return fail(BES_E_INVALID, "bad buffer");
  int bytes = dtype == BES_FLOAT64 ? 8 : dtype == BES_FLOAT32 ? 4 : 0;
  if (!bytes) return fail(BES_E_UNSUPPORTED, "fill supports float32 and float64");
  hipError_t e = bes::launch_fill_zero(ptr, n, bytes, (hipStream_t)hip_stream);
  return e == hipSuccess ? BES_OK : hip_fail(e, "fill");
}

// ---------------------------------------------------------------------------
// Persistent batched launch
// ---------------------------------------------------------------------------

void bes_batch_destroy(bes_batch *b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
  if (b->staged) (void)hipEventDestroy(b->staged);
  if (b->d_table) (void)hipFree(b->d_table);
  if (b->d_ptrs) (void)hipFree(b->d_ptrs);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_counters) (void)hipFree(b->d_counters);
  if (b->h_ptrs) (void)hipHostFree(b->h_ptrs);
  delete b;
}

int bes_batch_create(bes_ctx *ctx, bes_plan *const *plans, int32_t count, bes_batch **out) {
  (void)ctx;
  if (!out || !plans || count <= 0) return fail(BES_E_INVALID, "bad arguments");
  *out = nullptr;
  bes_batch *B = new (std::nothrow) bes_batch;
  if (!B) return fail(BES_E_NOMEM, "out of host memory");
  std::vector<GenEinsum> table(count);
  std::vector<GenItem> items;
  std::vector<double> cost;
  std::string err;
  // target serial chain of value reads per work-item (measured best between
  // 64 and 128 on the 256-einsum batch; 32 and 256 are slower)
  const double chain = 128.0;
  for (int k = 0; k < count; ++k) {
    if (!plans[k]) {
      bes_batch_destroy(B);
      return fail(BES_E_INVALID, "NULL plan");
    }
    const bes::Plan &p = plans[k]->p;
    if (!p.exprs.empty()) {
      bes_batch_destroy(B);
      return fail(BES_E_UNSUPPORTED, "plans with expression operands launch with bes_launch");
    }
    bool f64 = p.spec.dtype == BES_FLOAT64;
    if (k == 0) B->f64 = f64;
    if (f64 != B->f64) {
      bes_batch_destroy(B);
      return fail(BES_E_UNSUPPORTED, "a batch must have one dtype");
    }
    bes_config c = p.cfg;
    c.template_id = BES_T_GENERIC;
    c.p[0] = 256;
    c.p[1] = 1;
    c.p[2] = 1;
    int rc = bes::bind_generic_static(p, c, table[k], err);
    if (rc) {
      bes_batch_destroy(B);
      return fail(rc, err);
    }
    B->plans.push_back(&p);
    GenEinsum &g = table[k];
    if (!g.narrow) B->narrow = false;
    // Value reads per output: `per` at each shared row (the row-dependent
    // operands' exclusive sums) and `once` for the other operands.
    double per = 0.0, once = 0.0;
    for (int op = 0; op < g.n_ops; ++op) {
      const double ex = (double)std::max<int64_t>(g.ex_size[op], 1);
      if ((g.row_dep >> op) & 1) per += ex;
      else once += ex;
    }
    const int64_t sh = std::max<int64_t>(g.sh_size, 1);
    // The einsum shares the machine with the others, so its decomposition is
    // the batch's own (a plan's tuned config fills the whole device alone):
    // lanes and chunks cut each work-item's serial chain of reads to about
    // `chain`.  Lanes split the shared rows while each keeps at least half a
    // chain and their share of the `once` sums stays below the row reads;
    // where the `once` sums alone exceed a chain, lanes split them too
    // (those reads cost more: each decodes its full index).  Chunks split
    // the rows further while the rows exceed twice `chain`; a tile takes as
    // many passes as fit in one chain.
    const double rows = (double)sh * std::max(per, 1.0);
    int lanes = 1;
    while (lanes < 64 && lanes * 2 <= sh && rows / (lanes * 2) >= chain * 0.5 &&
           once * lanes * 2 <= rows)
      lanes *= 2;
    while (lanes < 64 && once / lanes > chain) lanes *= 2;
    int chunks = 1;
    while (chunks < 64 && (int64_t)lanes * chunks * 2 <= sh &&
           rows / ((double)lanes * chunks) > 2.0 * chain)
      chunks *= 2;
    const double lane_chain = once / lanes + rows / ((double)lanes * chunks);
    const int64_t per_pass = 256 / lanes;
    const int64_t passes =
        std::max<int64_t>(1, std::min<int64_t>((int64_t)(chain / lane_chain),
                                               (g.out_size + per_pass - 1) / per_pass));
    g.lanes = lanes;
    g.split = chunks;
    g.tile = (int32_t)(per_pass * passes);
    if (g.split > 1) B->any_split = true;
    for (int s = 0; s < g.n_slots; ++s) {
      const int members = g.slot_m1[s] - g.slot_m0[s];
      for (int64_t f = 0; f < g.out_size; f += g.tile) {
        for (int ch = 0; ch < chunks; ++ch) {
          GenItem it;
          std::memset(&it, 0, sizeof it);
          it.einsum = k;
          it.slot = s;
          it.first = f;
          it.count = std::min<int64_t>(g.tile, g.out_size - f);
          it.chunk = ch;
          items.push_back(it);
          const int64_t np = (it.count + per_pass - 1) / per_pass;
          cost.push_back((double)np * members * lane_chain);
        }
      }
    }
  }
  // Longest-processing-time first: the dynamic counter then balances the tail.
  std::vector<int> order(items.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<GenItem> sorted;
  for (int i : order) sorted.push_back(items[i]);
  B->n_items = (int)sorted.size();
  hipError_t e;
  if ((e = hipGetDevice(&B->device)) != hipSuccess ||
      (e = hipMalloc((void **)&B->d_table, sizeof(GenEinsum) * count)) != hipSuccess ||
      (e = hipMalloc((void **)&B->d_ptrs, sizeof(GenPtrs) * count)) != hipSuccess ||
      (e = hipMalloc((void **)&B->d_items, sizeof(GenItem) * std::max(1, B->n_items))) !=
          hipSuccess ||
      (e = hipMalloc((void **)&B->d_counters, 2 * sizeof(unsigned))) != hipSuccess ||
      (e = hipHostMalloc((void **)&B->h_ptrs, sizeof(GenPtrs) * count)) != hipSuccess ||
      (e = hipMemcpy(B->d_table, table.data(), sizeof(GenEinsum) * count,
                     hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(B->d_items, sorted.data(), sizeof(GenItem) * B->n_items,
                     hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemset(B->d_counters, 0, 2 * sizeof(unsigned))) != hipSuccess ||
      (e = hipEventCreateWithFlags(&B->staged, hipEventDisableTiming)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&B->capture_stream, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipDeviceSynchronize()) != hipSuccess) {
    bes_batch_destroy(B);
    return hip_fail(e, "batch setup");
  }
  B->last.resize(count);
  B->grid = std::min(B->n_items, bes::device_cu_count() * 4);
  B->use_graph = !env_flag("BES_NO_GRAPH");
  *out = B;
  return BES_OK;
}

int bes_batch_launch(bes_batch *B, const void *const *const *src_ptrs, void *const *const *out_ptrs,
                     void *hip_stream) {
  int rc = bes_batch_bind(B, src_ptrs, out_ptrs, hip_stream);
  return rc < 0 ? rc : bes_batch_replay(B, hip_stream);
}

int bes_batch_bind(bes_batch *B, const void *const *const *src_ptrs, void *const *const *out_ptrs,
                   void *hip_stream) {
  if (!B || !src_ptrs || !out_ptrs) return fail(BES_E_INVALID, "NULL argument");
  hipStream_t stream = (hipStream_t)hip_stream;
  const int count = (int)B->plans.size();
  std::vector<GenPtrs> cur(count);
  for (int k = 0; k < count; ++k) {
    const bes::Plan &p = *B->plans[k];
    if (!src_ptrs[k] || !out_ptrs[k]) return fail(BES_E_INVALID, "NULL pointer list");
    std::vector<const void *> src(p.n_src);
    for (int q = 0; q < p.n_src; ++q) src[q] = p.adjoint ? src_ptrs[k][p.src_from[q]] : src_ptrs[k][q];
    bes::bind_generic_ptrs(p, src.data(), out_ptrs[k], cur[k]);
  }
  hipError_t e;
  bool changed = !B->have_last ||
                 std::memcmp(cur.data(), B->last.data(), sizeof(GenPtrs) * count) != 0;
  if (changed) {
    // the previous staging copy must have been consumed before it is rewritten
    if (B->have_last && (e = hipEventSynchronize(B->staged)) != hipSuccess)
      return hip_fail(e, "batch staging sync");
    std::memcpy(B->h_ptrs, cur.data(), sizeof(GenPtrs) * count);
    if ((e = hipMemcpyAsync(B->d_ptrs, B->h_ptrs, sizeof(GenPtrs) * count,
                            hipMemcpyHostToDevice, stream)) != hipSuccess ||
        (e = hipEventRecord(B->staged, stream)) != hipSuccess)
      return hip_fail(e, "batch pointer upload");
    B->last = cur;
    B->have_last = true;
  }
  return BES_OK;
}

int bes_batch_replay(bes_batch *B, void *hip_stream) {
  if (!B) return fail(BES_E_INVALID, "NULL batch");
  if (!B->have_last) return fail(BES_E_STATE, "bind pointers before the first replay");
  hipStream_t stream = (hipStream_t)hip_stream;
  hipError_t e;
  if (B->use_graph && !B->exec) {
    bool ok = hipStreamBeginCapture(B->capture_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      hipError_t le = bes::launch_persistent(B->f64, B->d_table, B->d_ptrs, B->d_items, B->n_items,
                                             B->d_counters, B->grid, B->capture_stream,
                                             (int)B->plans.size(), B->any_split, B->narrow);
      hipGraph_t g = nullptr;
      hipError_t ce = hipStreamEndCapture(B->capture_stream, &g);
      ok = le == hipSuccess && ce == hipSuccess && g;
      if (ok && hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        ok = false;
        B->exec = nullptr;
      }
      if (ok) B->graph = g;
      else if (g) (void)hipGraphDestroy(g);
    }
    if (!ok) {
      (void)hipGetLastError();
      B->use_graph = false;  // fall back to direct persistent launches
    }
  }
  if (B->use_graph && B->exec) {
    e = hipGraphLaunch(B->exec, stream);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    return BES_OK;
  }
  e = bes::launch_persistent(B->f64, B->d_table, B->d_ptrs, B->d_items, B->n_items, B->d_counters,
                             B->grid, stream, (int)B->plans.size(), B->any_split, B->narrow);
  if (e != hipSuccess) return hip_fail(e, "persistent launch");
  return BES_OK;
}

int bes_identify(const bes_plan *ref, const bes_plan *raised, int32_t *member_map,
                 int32_t *pos_map, int32_t *arg_map, char *index_map) {
  if (!ref || !raised) return fail(BES_E_INVALID, "NULL plan");
  const bes::Plan &r = ref->p, &k = raised->p;
  if (r.key != k.key)
    return fail(BES_E_INVALID, "the batched einsums are not isomorphic: canonical forms differ");
  const bes::Canonical &cr = r.canon, &ck = k.canon;
  // canonical name -> reference name and canonical name -> raised name,
  // composed: reference name -> raised name
  if (member_map)
    for (size_t c = 0; c < cr.member_map.size(); ++c) member_map[cr.member_map[c]] = ck.member_map[c];
  if (pos_map)
    for (size_t c = 0; c < cr.pos_map.size(); ++c) pos_map[cr.pos_map[c]] = ck.pos_map[c];
  if (arg_map)
    for (size_t c = 0; c < cr.arg_map.size(); ++c) arg_map[cr.arg_map[c]] = ck.arg_map[c];
  if (index_map)
    for (size_t c = 0; c < cr.index_map.size(); ++c)
      index_map[cr.index_map[c]] = (char)('a' + ck.index_map[c]);
  return BES_OK;
}

int bes_adjoint(bes_ctx *ctx, const bes_plan *fwd, int32_t pos, bes_plan **out, int32_t *n_out) {
  if (!fwd || !out) return fail(BES_E_INVALID, "NULL argument");
  *out = nullptr;
  try {
    bes_plan *P = new bes_plan;
    std::string err;
    int nout = 0;
    int rc = bes::build_adjoint(fwd->p, pos, P->p, nout, err);
    if (rc) {
      delete P;
      return fail(rc, err);
    }
    if (n_out) *n_out = nout;
    rc = apply_lookup(ctx, P->p, kDefaultArch);
    *out = P;
    return rc;
  } catch (const std::bad_alloc &) {
    return fail(BES_E_NOMEM, "out of host memory");
  }
}

}  // extern "C"
