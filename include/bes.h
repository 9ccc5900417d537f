/*
 * bes.h -- C ABI of the batched-einsum library (gfx950 / MI355X).
 *
 * A batched einsum is b einsums that share one Einstein notation and possibly
 * some operands (Definition "Batched Einstein Summation"; arxiv 2601.12220).
 * Operands may be functional: each argument is a function of its index tuple
 * evaluated from one or two source buffers (Definition "Functional Batched
 * Einstein Summation").  The library
 *
 *   1. parses and validates the notation and the b x n argument table,
 *   2. maps the batched einsum to its colored induced graph (Appendix B.1),
 *   3. labels that graph canonically (Algorithm "CanonicalizeBatchedEinsum"),
 *   4. rebuilds the canonical batched einsum from the labeled graph (Appendix
 *      B.2) together with the substitution maps back to the caller's names,
 *   5. looks up a tuning record by (canonical key, GPU arch),
 *   6. binds the caller's buffers to the canonical operand slots, and
 *   7. launches hand-written HIP kernels on the caller's stream.
 *
 * Conventions shared by every entry point
 *   - Every function returns an int status (enum bes_status): 0 success,
 *     > 0 success with a warning, < 0 error.  Nothing throws across the ABI.
 *     On error, bes_last_error() returns a thread-local message.
 *   - Device pointers are plain HIP device addresses; `hip_stream` is a
 *     hipStream_t (NULL = the default stream).  The caller owns every device
 *     buffer and every stream; the library keeps raw device pointers only for
 *     the duration of a launch (a bes_batch keeps its own descriptor table).
 *   - All shapes and strides are in elements, not bytes.
 *   - Index names are the letters 'a'..'z' (grammar of the Listing "Grammar
 *     for an index"), so a batched einsum has at most 26 distinct indices.
 */
#ifndef BES_H
#define BES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum bes_status {
  BES_OK = 0,
  BES_W_NOTFOUND = 1,     /* no tuning record: the template default is used */
  BES_E_INVALID = -1,     /* malformed notation or table, violated soundness
                             condition of Eq. (1), repeated output index */
  BES_E_UNSUPPORTED = -2, /* dtype the kernels lack, 0-dim operand, kind or
                             size outside the library's limits */
  BES_E_HIP = -3,         /* a HIP runtime call failed */
  BES_E_NOMEM = -4,       /* host or device allocation failed */
  BES_E_BUFFER = -5,      /* caller buffer too small; *len holds the need */
  BES_E_STATE = -6        /* call not valid for this object (e.g. no GPU) */
};

/* Dtype codes are the DtypeRank values of the induced-graph construction
 * (Appendix B.1, dtype ranks).  Canonicalization accepts all eight; the GPU
 * kernels evaluate float32 and float64 only. */
enum bes_dtype {
  BES_INT8 = 1, BES_INT32 = 2, BES_INT64 = 3, BES_FLOAT16 = 4,
  BES_FLOAT32 = 5, BES_FLOAT64 = 6, BES_COMPLEX64 = 7, BES_COMPLEX128 = 8
};

/* Operand kinds: the functions M(A) of a functional batched einsum that the
 * kernels evaluate in registers (never materialized in device memory). */
enum bes_kind {
  BES_ARRAY = 0,        /* M(A)[idx] = S0[idx], S0 dense row-major, or
                           strided if src_strides[0] is non-zero */
  BES_VIEW = 1,         /* M(A)[idx] = S0[src_offset[0] + sum idx_k*stride_k] */
  BES_ELEMENTWISE = 2,  /* M(A)[idx] = alpha*op(S0[idx]) + beta (+ S1[idx]
                           when nsrc == 2) */
  BES_TET_JACOBIAN = 3, /* M(A)[e,x,r] = S0[e,r+1,x] - S0[e,0,x]: Jacobian of
                           the affine map of a tetrahedron whose 4 vertex
                           coordinates are S0[e,4,3]; the operand is 3-d with
                           extents (e,3,3); src_strides[0] are S0's strides */
  BES_EXPR = 4          /* M(A)[idx] = f(S0[idx], S1[idx]) for an expression
                           body f given at registration (bes_register_expr):
                           the substitution-rule bodies of the paper's
                           retrieval listing; compiled at run time */
};

enum bes_unary { BES_OP_ID = 0, BES_OP_SIN = 1, BES_OP_COS = 2, BES_OP_SQUARE = 3 };

#define BES_MAX_DIM 8
#define BES_MAX_SRC 2
#define BES_MAX_B 64
#define BES_MAX_N 8

/* Descriptor of one argument of the batched einsum.
 *   kind, dtype, ndim, shape: as above; ndim in 1..BES_MAX_DIM.
 *   nsrc: number of source buffers (1, or 2 for ELEMENTWISE with S1).
 *   src_offset[s], src_strides[s][d]: element offset and strides of source s
 *     (all-zero strides mean dense row-major in `shape`; for TET_JACOBIAN the
 *     three strides address S0[e, vertex, coordinate]).
 *   op, alpha, beta: the ELEMENTWISE function. */
typedef struct bes_operand {
  int32_t kind;
  int32_t dtype;
  int32_t ndim;
  int32_t nsrc;
  int64_t shape[BES_MAX_DIM];
  int64_t src_offset[BES_MAX_SRC];
  int64_t src_strides[BES_MAX_SRC][BES_MAX_DIM];
  int32_t op;
  int32_t reserved;
  double alpha;
  double beta;
} bes_operand;

/* Kernel templates and their tunable parameters (the "transformations" whose
 * performance facts the tuning database stores, Section "Integration ..."). */
enum bes_template {
  BES_T_AUTO = 0,        /* let the planner pick */
  BES_T_FEM_STREAM = 1,  /* per-element operands streamed from HBM, small
                            shared operand uniform per wave; p[0] = elements
                            per tile (64: one wave), p[1] = grid size in
                            blocks per compute unit (1..64), p[2] = kernel
                            variant: 0 the lean kernel with two waves per
                            64-element tile where the batch allows it, 2 the
                            lean kernel with one wave per tile, 1 always the
                            descriptor-driven kernel, 3 for FP32 batches of
                            one stage-1 group (at most three members, plain
                            u, G views of one row) stage 1 on the matrix
                            cores (other batches as 0); for the face-mass /
                            divergence class p[1] = blocks of four waves
                            per compute unit, p[2] = 0 or 1 the shared
                            matrix in LDS, 2 as scalar operands, 3 (FP64,
                            plain streamed operand with contiguous element
                            rows) the shared-matrix product on the matrix
                            cores */
  BES_T_GENERIC = 2,     /* any batched einsum; p[0] = outputs per tile,
                            p[1] = lanes per output (1,2,4,...,64),
                            p[2] = chunks of the shared contracted index
                            space per output (0 or 1: none; up to 64) */
  BES_T_MFMA = 3,        /* dense contraction on MFMA (FP32 in, FP32 acc);
                            p[0] = tile M, p[1] = tile N, p[2] = split */
  BES_T_GETT = 4         /* any binary contraction (FP32 or FP64) on the
                            matrix cores: arbitrary index groups and strides
                            through offset tables, affine operands
                            alpha*A+beta applied while loading, ragged
                            edges; p[0], p[1] unused (64),
                            p[2] = K ranges per output tile (0: chosen by
                            the launcher; > 1: partial tiles add
                            atomically into the zeroed output), p[3] =
                            tile shape (0: by the output's extents; 1: 16
                            x 128, 2: 32 x 128, 3: 128 x 32, 4: 128 x 16,
                            5: 64 x 64, 6: 64 x 64 with K staged 32 deep,
                            7: 128 x 64), p[4] = 1: with eight or more K
                            ranges the partial tiles go to a plan-owned
                            workspace (allocated on the first such launch,
                            at most 64 MiB) and a second kernel sums them */
};

typedef struct bes_config {
  int32_t template_id;
  int32_t p[6];
} bes_config;

typedef struct bes_ctx bes_ctx;
typedef struct bes_plan bes_plan;
typedef struct bes_batch bes_batch;

/* Context: owns the tuning database (DS9).  `tuning_db_path` may be NULL
 * (no database).  A missing file is created on the first record; malformed
 * lines are skipped with a warning on stderr when BES_LOG >= 1.
 * Makes no HIP call. */
int bes_ctx_create(bes_ctx **out, const char *tuning_db_path);
void bes_ctx_destroy(bes_ctx *ctx);

/* Register a batched einsum (steps 1-6 above; host only, no HIP call).
 *   notation: "in_1,...,in_n->out", letters a..z (repeated letters inside one
 *     input address a diagonal; output letters must be distinct and appear in
 *     some input -- the soundness conditions after Eq. (1)).
 *   b, n: batch size (1..BES_MAX_B) and operands per einsum (1..BES_MAX_N).
 *   args[n_args]: argument descriptors; every argument must occur in `table`.
 *   table[b*n]: row-major argument ids; row i lists the operands of member i.
 * Every index must have one extent across the whole batch.  All arguments
 * share one dtype (the output dtype).  On success *out owns a plan; destroy it
 * with bes_plan_destroy.  The returned status is BES_W_NOTFOUND when the
 * context has no record for the plan's key on `gfx950`. */
int bes_register(bes_ctx *ctx, const char *notation, int32_t b, int32_t n,
                 int32_t n_args, const bes_operand *args, const int32_t *table,
                 bes_plan **out);
void bes_plan_destroy(bes_plan *plan);

/* bes_register with expression operands (kind BES_EXPR; Definition
 * "Functional Batched Einstein Summation" with the substitution-rule bodies
 * of Section "Integration ...", e.g. "s0*s0", "3*cos(s0)+5", "sin(s0)+s1").
 * exprs[a] is the body of argument a (NULL for other kinds; exprs may be NULL
 * when no argument is an expression).  A body is a C expression over s0 and
 * s1 (the argument's first and second source at the same index, each through
 * its own offset and strides; nsrc 1 or 2), decimal constants, + - * / and
 * parentheses, and the functions sin cos tan exp log sqrt fabs tanh pow fmin
 * fmax; anything else is BES_E_INVALID.  Bodies are not part of the
 * canonical key (a tuning record transfers between functional variants).
 * Plans with expression operands are evaluated by the generic template,
 * built with hipRTC for their bodies at the first launch on a device. */
int bes_register_expr(bes_ctx *ctx, const char *notation, int32_t b, int32_t n,
                      int32_t n_args, const bes_operand *args, const int32_t *table,
                      const char *const *exprs, bes_plan **out);

/* Canonical key (the tuning-database identity): the canonical batched einsum
 * with its extents and dtypes, identical for every isomorphic registration
 * (Definition "Canonicalization of a batched einsum").  Written with a NUL
 * into buf[cap]; *len receives the length without the NUL.  buf may be NULL
 * to query the length (returns BES_E_BUFFER when cap is too small). */
int bes_plan_key(const bes_plan *plan, char *buf, size_t cap, size_t *len);

/* The canonical batched einsum in the paper's tuple notation, e.g.
 * "(1, 2, (a), ((a b), (a c)), ((A_0, A_1)))"; same buffer convention. */
int bes_plan_canonical(const bes_plan *plan, char *buf, size_t cap, size_t *len);

/* Substitution maps from the canonical form to the registration
 * (Algorithm "CanonicalizeBatchedEinsum" returns sigma^A and sigma^I; the
 * library also returns sigma^i and sigma^j):
 *   member_map[k] = user member of canonical member k        (b entries)
 *   pos_map[j]    = user operand position of canonical pos j (n entries)
 *   arg_map[a]    = user argument id of canonical arg A_a    (n_args entries)
 *   index_map[c]  = user letter of canonical index 'a'+c     (n_index chars)
 * Any pointer may be NULL.  *n_index (optional) gets the number of indices. */
int bes_plan_maps(const bes_plan *plan, int32_t *member_map, int32_t *pos_map,
                  int32_t *arg_map, char *index_map, int32_t *n_index);

/* Identify one registered batched einsum as another (Algorithm
 * "IdentifyAsEinsum"): when `raised` (for example one raised from a traced
 * program) and `ref` (the batched einsum a transformation or tuning record
 * was written for) have the same canonical form, return the composed
 * substitution from the reference's names to the raised one's:
 *   member_map[i] = raised member of reference member i       (b entries)
 *   pos_map[j]    = raised operand position of reference pos j (n entries)
 *   arg_map[a]    = raised argument id of reference argument a (n_args)
 *   index_map[x]  = raised letter of reference index 'a' + x   (indexed by
 *                   the reference's index letter minus 'a'; 26 entries,
 *                   untouched where the reference has no such index)
 * Any pointer may be NULL.  BES_E_INVALID when the canonical forms differ
 * (the algorithm's exception).  Host only. */
int bes_identify(const bes_plan *ref, const bes_plan *raised, int32_t *member_map,
                 int32_t *pos_map, int32_t *arg_map, char *index_map);

/* Induced graph of the registration (Appendix B.1) and of the canonical form:
 * n_nodes, then optionally the row-major adjacency (n_nodes^2 bytes, 0/1) and
 * the colors (1..9).  which = 0: induced graph in construction order;
 * which = 1: canonically relabeled graph. */
int bes_plan_graph(const bes_plan *plan, int32_t which, int32_t *n_nodes,
                   uint8_t *adj, int32_t *colors);

/* Check compliance conditions C1-C30 of Appendix B.2 on a colored digraph.
 * Returns 0 if compliant, else the number (1..30) of the first violated
 * condition.  adj is n*n row-major bytes, colors n entries. */
int bes_check_compliance(int32_t n, const uint8_t *adj, const int32_t *colors);

/* Canonical labeling of a vertex-colored digraph (the GetCanonLabel step):
 * label[v] = canonical position of vertex v.  Labels are invariant: two
 * isomorphic colored digraphs relabel to the same adjacency. */
int bes_canonical_labeling(int32_t n, const uint8_t *adj, const int32_t *colors,
                           int32_t *label);

/* Tuning: look up (key, arch) and install the record's config in the plan.
 * Returns BES_OK on a hit, BES_W_NOTFOUND (and installs the template default)
 * on a miss. */
int bes_plan_lookup(bes_ctx *ctx, bes_plan *plan, const char *arch);
int bes_plan_get_config(const bes_plan *plan, bes_config *cfg);
/* Install a config (autotuner); BES_E_UNSUPPORTED if the template cannot
 * evaluate this plan. */
int bes_plan_set_config(bes_plan *plan, const bes_config *cfg);
/* Append a performance fact; the last record for (key, arch) wins. */
int bes_db_record(bes_ctx *ctx, const char *key, const char *arch,
                  const bes_config *cfg, double seconds);
/* Number of lookups that hit / missed since the context was created. */
int bes_ctx_stats(const bes_ctx *ctx, int64_t *hits, int64_t *misses);

/* Launch one plan on `hip_stream`.
 *   src_ptrs: device pointers of every argument's sources, flattened in user
 *     argument order then source order (sum over args of nsrc entries).
 *   out_ptrs: b device pointers of the outputs in user member order; output i
 *     is dense row-major with the extents of the output indices in the
 *     notation's order and is overwritten.
 * Asynchronous; returns BES_E_HIP if the launch could not be enqueued.
 * The first launch of a plan on a device (and of a new config or output
 * layout) allocates and uploads the plan's device state (descriptors, offset
 * tables, workspaces); later launches of it only enqueue kernels, so a
 * caller that captures launches in a HIP graph launches once before capture,
 * or uses bes_launch_noalloc.  Launches of one plan that overlap in time on
 * different streams share its workspaces and race. */
int bes_launch(const bes_plan *plan, const void *const *src_ptrs,
               void *const *out_ptrs, void *hip_stream);

/* bes_launch for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results and stream semantics as bes_launch, but it calls no
 * hipMalloc, hipFree or allocating library routine: the FEM-stream
 * template's re-laid shared operand goes to a fixed 256 KiB device array
 * that the library holds on every GPU it runs on until the process ends
 * (enough for every compiled FEM shape with up to 8 stage-1 groups).  Only
 * plans whose current template is FEM-stream or MFMA are accepted; others,
 * a shared operand larger than the array, an accumulating FEM output and
 * MFMA operands unaligned for its vector tiles give BES_E_UNSUPPORTED
 * (bes_launch evaluates those).  Calls on one GPU share its array: calls
 * that overlap in time on one GPU (on different streams, or from several
 * host threads) race; calls ordered on one stream do not. */
int bes_launch_noalloc(const bes_plan *plan, const void *const *src_ptrs,
                       void *const *out_ptrs, void *hip_stream);

/* Output layout of output slot `slot` (0 .. number of outputs - 1: the b
 * members of a plain plan in user order, the n_out outputs of an adjoint
 * plan).  The launch writes element (i_1, ..., i_k) of that output, indices
 * in the notation's output order, at out_ptrs[slot] + offset + sum_d i_d *
 * strides[d] (elements), and with accumulate != 0 adds its value to what is
 * there instead of overwriting it.  strides == NULL and offset == 0 restore
 * dense row-major.  This is how an adjoint writes the gradient of a VIEW
 * argument straight into its source buffer's gradient and how gradients of
 * one buffer from several operand positions are summed (Section "Batched
 * Einstein Summation": a shared argument's gradient is the sum over every
 * slot that reads it).  Accumulating outputs that overlap in memory are
 * added atomically; overwritten outputs must not overlap.  The FEM-stream
 * template overwrites only: a plan that accumulates is evaluated by the
 * generic template.  The caller owns the memory; makes no HIP call. */
int bes_plan_set_output(bes_plan *plan, int32_t slot, int64_t offset, const int64_t *strides,
                        int32_t accumulate);

/* Zero n elements of `dtype` (BES_FLOAT32 / BES_FLOAT64) at device pointer
 * ptr on `hip_stream` with a fill kernel (no memset node, so it can be
 * captured in a HIP graph).  For gradients that only accumulate. */
int bes_fill_zero(void *ptr, int64_t n, int32_t dtype, void *hip_stream);

/* Profiling hook.  With both events non-NULL (hipEvent_t handles the caller
 * owns and keeps alive), every later bes_launch of the plan records
 * start_event on its stream right before the plan's evaluation kernel(s) and
 * stop_event right after them; a re-layout of the shared operand that the
 * FEM-stream template may enqueue first is outside the pair.  NULL, NULL
 * turns it off.  BES_E_INVALID if only one event is given.  Makes no HIP
 * call itself. */
int bes_plan_set_timing(bes_plan *plan, void *start_event, void *stop_event);

/* Persistent batched launch of many plans (one kernel over a device work list
 * of (plan, member, tile) items, captured once in a hipGraph).
 * bes_batch_create evaluates every plan with the generic template and picks
 * its own decomposition per plan for the shared launch (lanes per output,
 * chunks of the contracted space, outputs per work item, sized so that each
 * work item reads about 128 values in sequence), since a plan's own config is
 * tuned for a launch that has the device to itself; it uploads the descriptor
 * table once.  bes_batch_launch binds pointers (src_ptrs[p], out_ptrs[p] as in
 * bes_launch for plan p) and replays.  Pointers may change between launches.
 * Set BES_NO_GRAPH=1 to launch without graph capture. */
int bes_batch_create(bes_ctx *ctx, bes_plan *const *plans, int32_t count,
                     bes_batch **out);
int bes_batch_launch(bes_batch *batch, const void *const *const *src_ptrs,
                     void *const *const *out_ptrs, void *hip_stream);
void bes_batch_destroy(bes_batch *batch);

/* bes_batch_launch in two parts, for callers that launch the same batch on
 * the same buffers many times: bes_batch_bind binds the pointers (as
 * bes_batch_launch does; the device copy is refreshed on `hip_stream` only
 * when a pointer changed) and bes_batch_replay launches the persistent work
 * on `hip_stream` with the pointers bound last, without touching the 256
 * per-plan pointer sets again.  BES_E_STATE if nothing was bound yet. */
int bes_batch_bind(bes_batch *batch, const void *const *const *src_ptrs,
                   void *const *const *out_ptrs, void *hip_stream);
int bes_batch_replay(bes_batch *batch, void *hip_stream);

/* Adjoint: the batched einsum giving d<G, R>/dA for the arguments at operand
 * position `pos` of a forward plan.  Its operands are, per forward member i,
 * (G_i, the other operands of member i) and its output index list is the
 * forward index list of position `pos`.  Members whose position-`pos`
 * argument is the same are summed into one output.  The adjoint plan is
 * itself registered (canonicalized, keyed, tuned).
 *   Launch it with src_ptrs = [the b gradients G_i (dense, forward output
 *   shape), then the forward plan's src_ptrs] and out_ptrs = one pointer per
 *   distinct position-`pos` argument, in order of first occurrence down the
 *   rows (n_out receives that count).  Outputs are dense in the argument's
 *   shape and overwritten by default; bes_plan_set_output on the adjoint plan
 *   writes the gradient of a VIEW argument through the view's offset and
 *   strides into its source's gradient, and accumulates into a gradient that
 *   another position or plan already wrote.
 * BES_E_UNSUPPORTED if the position has a repeated index.  Functional
 * arguments at other positions are evaluated as in the forward plan; the
 * gradient with respect to the sources of a functional (ELEMENTWISE,
 * TET_JACOBIAN) argument is not provided. */
int bes_adjoint(bes_ctx *ctx, const bes_plan *fwd, int32_t pos,
                bes_plan **out, int32_t *n_out);

const char *bes_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BES_H */
