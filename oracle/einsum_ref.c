/*
 * Oracle: plain FP64 loop-nest evaluation of one einsum.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the HIP library.
 *
 * Semantics: Eq. (1) of the einsum definition (Section "Einstein Notation"):
 *   R[I_out] = sum over every index of the inputs that is not in I_out of
 *              prod_k A^k[I^{in,k}].
 * A batched einsum (Section "Batched Einstein Summation") is b independent
 * einsums of one notation, so the batch loop lives in the Python wrapper.
 *
 * Conventions: indices are integers 0..25 (letters a..z); every operand is a
 * dense row-major FP64 array whose axis extents are extent[label]; a label that
 * repeats inside one operand addresses its diagonal (the strides of the repeated
 * axes add up).  The contracted indices are visited in ascending label order
 * (alphabetical), innermost last.  No factoring, no reordering, no blocking.
 */
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#define MAXL 26
#define MAXOPS 16

typedef long long i64;

/* Per-operand, per-label element stride (summed over repeated axes). */
static int build_strides(int n_ops, const int *ndim, const int *labels,
                         const i64 *extent, i64 stride[MAXOPS][MAXL]) {
  int off = 0;
  for (int k = 0; k < n_ops; ++k) {
    for (int l = 0; l < MAXL; ++l) stride[k][l] = 0;
    i64 s = 1;
    for (int d = ndim[k] - 1; d >= 0; --d) {
      int L = labels[off + d];
      if (L < 0 || L >= MAXL) return -1;
      stride[k][L] += s;
      s *= extent[L];
    }
    off += ndim[k];
  }
  return 0;
}

/* Labels used by any input, and whether each is an output label. */
static int classify(int n_ops, const int *ndim, const int *labels, int n_out,
                    const int *out_labels, int used[MAXL], int in_out[MAXL]) {
  int total = 0;
  for (int k = 0; k < n_ops; ++k) total += ndim[k];
  for (int l = 0; l < MAXL; ++l) used[l] = in_out[l] = 0;
  for (int t = 0; t < total; ++t) {
    if (labels[t] < 0 || labels[t] >= MAXL) return -1;
    used[labels[t]] = 1;
  }
  for (int d = 0; d < n_out; ++d) {
    int L = out_labels[d];
    if (L < 0 || L >= MAXL) return -1;
    if (in_out[L]) return -1; /* an output index may appear only once */
    if (!used[L]) return -1;  /* every output index must index some input */
    in_out[L] = 1;
  }
  return 0;
}

/* Value of one output element given its multi-index (out_idx[d] for out
 * label d), summing over the contracted labels in ascending order. */
static double one_entry(int n_ops, const double *const *ops,
                        i64 stride[MAXOPS][MAXL], int n_out,
                        const int *out_labels, const i64 *out_idx,
                        int n_con, const int *con, const i64 *extent) {
  i64 base[MAXOPS];
  for (int k = 0; k < n_ops; ++k) {
    base[k] = 0;
    for (int d = 0; d < n_out; ++d) base[k] += out_idx[d] * stride[k][out_labels[d]];
  }
  i64 n_terms = 1;
  for (int c = 0; c < n_con; ++c) n_terms *= extent[con[c]];
  double acc = 0.0;
  i64 cidx[MAXL];
  for (i64 t = 0; t < n_terms; ++t) {
    /* decode t into the contracted multi-index, last label fastest */
    i64 rem = t;
    for (int c = n_con - 1; c >= 0; --c) {
      cidx[c] = rem % extent[con[c]];
      rem /= extent[con[c]];
    }
    double prod = 1.0;
    for (int k = 0; k < n_ops; ++k) {
      i64 o = base[k];
      for (int c = 0; c < n_con; ++c) o += cidx[c] * stride[k][con[c]];
      prod *= ops[k][o];
    }
    acc += prod;
  }
  return acc;
}

/* Full evaluation.  Returns 0 on success, -1 on an invalid notation. */
int oracle_einsum(int n_ops, const int *ndim, const int *labels, int n_out,
                  const int *out_labels, const i64 *extent,
                  const double *const *ops, double *out) {
  if (n_ops < 1 || n_ops > MAXOPS) return -1;
  int used[MAXL], in_out[MAXL];
  if (classify(n_ops, ndim, labels, n_out, out_labels, used, in_out)) return -1;
  i64 stride[MAXOPS][MAXL];
  if (build_strides(n_ops, ndim, labels, extent, stride)) return -1;
  int con[MAXL], n_con = 0;
  for (int l = 0; l < MAXL; ++l)
    if (used[l] && !in_out[l]) con[n_con++] = l;
  i64 n_outputs = 1;
  for (int d = 0; d < n_out; ++d) n_outputs *= extent[out_labels[d]];
#pragma omp parallel for schedule(static)
  for (i64 o = 0; o < n_outputs; ++o) {
    i64 idx[MAXL];
    i64 rem = o;
    for (int d = n_out - 1; d >= 0; --d) {
      idx[d] = rem % extent[out_labels[d]];
      rem /= extent[out_labels[d]];
    }
    out[o] = one_entry(n_ops, ops, stride, n_out, out_labels, idx, n_con, con, extent);
  }
  return 0;
}

/* Selected output elements only: flat row-major output positions in `where`.
 * Used to check very large outputs one element at a time. */
int oracle_einsum_at(int n_ops, const int *ndim, const int *labels, int n_out,
                     const int *out_labels, const i64 *extent,
                     const double *const *ops, i64 n_where, const i64 *where,
                     double *vals) {
  if (n_ops < 1 || n_ops > MAXOPS) return -1;
  int used[MAXL], in_out[MAXL];
  if (classify(n_ops, ndim, labels, n_out, out_labels, used, in_out)) return -1;
  i64 stride[MAXOPS][MAXL];
  if (build_strides(n_ops, ndim, labels, extent, stride)) return -1;
  int con[MAXL], n_con = 0;
  for (int l = 0; l < MAXL; ++l)
    if (used[l] && !in_out[l]) con[n_con++] = l;
#pragma omp parallel for schedule(dynamic, 1)
  for (i64 w = 0; w < n_where; ++w) {
    i64 idx[MAXL];
    i64 rem = where[w];
    for (int d = n_out - 1; d >= 0; --d) {
      idx[d] = rem % extent[out_labels[d]];
      rem /= extent[out_labels[d]];
    }
    vals[w] = one_entry(n_ops, ops, stride, n_out, out_labels, idx, n_con, con, extent);
  }
  return 0;
}

/* Selected entries of the gradient below: for each flat row-major position
 * of operand `wrt` (whose labels must be distinct), the sum over every other
 * label of G[I_out] * prod_{m != wrt} A^m.  Used at sizes where the full
 * gradient loop would take too long. */
int oracle_einsum_grad_at(int n_ops, const int *ndim, const int *labels, int n_out,
                          const int *out_labels, const i64 *extent,
                          const double *const *ops, const double *G, int wrt,
                          i64 n_where, const i64 *where, double *vals) {
  if (n_ops < 1 || n_ops > MAXOPS || wrt < 0 || wrt >= n_ops) return -1;
  int used[MAXL], in_out[MAXL];
  if (classify(n_ops, ndim, labels, n_out, out_labels, used, in_out)) return -1;
  i64 stride[MAXOPS][MAXL];
  if (build_strides(n_ops, ndim, labels, extent, stride)) return -1;
  int off = 0;
  for (int k = 0; k < wrt; ++k) off += ndim[k];
  const int *wl = labels + off;
  int in_w[MAXL];
  for (int l = 0; l < MAXL; ++l) in_w[l] = 0;
  for (int d = 0; d < ndim[wrt]; ++d) {
    if (in_w[wl[d]]) return -1; /* repeated label in the wrt operand */
    in_w[wl[d]] = 1;
  }
  i64 gstride[MAXL];
  for (int l = 0; l < MAXL; ++l) gstride[l] = 0;
  {
    i64 s = 1;
    for (int d = n_out - 1; d >= 0; --d) {
      gstride[out_labels[d]] = s;
      s *= extent[out_labels[d]];
    }
  }
  int rest[MAXL], n_rest = 0;
  for (int l = 0; l < MAXL; ++l)
    if (used[l] && !in_w[l]) rest[n_rest++] = l;
  i64 n_terms = 1;
  for (int a = 0; a < n_rest; ++a) n_terms *= extent[rest[a]];
#pragma omp parallel for schedule(dynamic, 1)
  for (i64 w = 0; w < n_where; ++w) {
    i64 val[MAXL];
    for (int l = 0; l < MAXL; ++l) val[l] = 0;
    i64 rem = where[w];
    for (int d = ndim[wrt] - 1; d >= 0; --d) {
      val[wl[d]] = rem % extent[wl[d]];
      rem /= extent[wl[d]];
    }
    double acc = 0.0;
    for (i64 t = 0; t < n_terms; ++t) {
      i64 r = t;
      for (int a = n_rest - 1; a >= 0; --a) {
        val[rest[a]] = r % extent[rest[a]];
        r /= extent[rest[a]];
      }
      i64 go = 0;
      for (int l = 0; l < MAXL; ++l) go += val[l] * gstride[l];
      double prod = G[go];
      for (int k = 0; k < n_ops; ++k) {
        if (k == wrt) continue;
        i64 o = 0;
        for (int l = 0; l < MAXL; ++l) o += val[l] * stride[k][l];
        prod *= ops[k][o];
      }
      acc += prod;
    }
    vals[w] = acc;
  }
  return 0;
}

/* Gradient of sum(G * R) with respect to operand `wrt`, by the definition of
 * the derivative of a multilinear form: for every assignment of all indices,
 *   dA_wrt[I^{in,wrt}] += G[I_out] * prod_{m != wrt} A^m[I^{in,m}].
 * dA is overwritten.  Serial on purpose: it is only used at small sizes. */
int oracle_einsum_grad(int n_ops, const int *ndim, const int *labels, int n_out,
                       const int *out_labels, const i64 *extent,
                       const double *const *ops, const double *G, int wrt,
                       double *dA) {
  if (n_ops < 1 || n_ops > MAXOPS || wrt < 0 || wrt >= n_ops) return -1;
  int used[MAXL], in_out[MAXL];
  if (classify(n_ops, ndim, labels, n_out, out_labels, used, in_out)) return -1;
  i64 stride[MAXOPS][MAXL];
  if (build_strides(n_ops, ndim, labels, extent, stride)) return -1;
  i64 gstride[MAXL];
  for (int l = 0; l < MAXL; ++l) gstride[l] = 0;
  {
    i64 s = 1;
    for (int d = n_out - 1; d >= 0; --d) {
      gstride[out_labels[d]] = s;
      s *= extent[out_labels[d]];
    }
  }
  int all[MAXL], n_all = 0;
  for (int l = 0; l < MAXL; ++l)
    if (used[l]) all[n_all++] = l;
  i64 wsize = 1;
  for (int d = 0; d < ndim[wrt]; ++d) {
    int off = 0;
    for (int k = 0; k < wrt; ++k) off += ndim[k];
    wsize *= extent[labels[off + d]];
  }
  memset(dA, 0, sizeof(double) * (size_t)wsize);
  i64 n_assign = 1;
  for (int a = 0; a < n_all; ++a) n_assign *= extent[all[a]];
  i64 idx[MAXL];
  for (i64 t = 0; t < n_assign; ++t) {
    i64 rem = t;
    for (int a = n_all - 1; a >= 0; --a) {
      idx[a] = rem % extent[all[a]];
      rem /= extent[all[a]];
    }
    i64 go = 0;
    for (int a = 0; a < n_all; ++a) go += idx[a] * gstride[all[a]];
    double prod = G[go];
    for (int k = 0; k < n_ops; ++k) {
      if (k == wrt) continue;
      i64 o = 0;
      for (int a = 0; a < n_all; ++a) o += idx[a] * stride[k][all[a]];
      prod *= ops[k][o];
    }
    i64 wo = 0;
    for (int a = 0; a < n_all; ++a) wo += idx[a] * stride[wrt][all[a]];
    /* A repeated label in the wrt operand addresses its diagonal, whose
     * derivative lands on that diagonal only. */
    dA[wo] += prod;
  }
  return 0;
}
