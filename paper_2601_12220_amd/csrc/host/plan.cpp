// Template analysis, default configs, binding and the adjoint builder.
//
// Role analysis runs on the canonical form (Algorithm
// "CanonicalizeBatchedEinsum" output), so every isomorphic registration gets
// the same template and the same tuning record; binding then routes each
// canonical operand slot to the caller's buffer through the substitution maps
// (the composition step of Algorithm "IdentifyAsEinsum").
#include "plan.h"

#include <algorithm>
#include <cstring>
#include <map>

#include "../fem_shapes.h"

namespace bes {

// The MFMA template is selected by default (128 x 128 output tiles, K in
// steps of 16).
constexpr bool kMfmaTemplateReady = true;

namespace {

bool contains(const std::vector<int> &v, int x) {
  return std::find(v.begin(), v.end(), x) != v.end();
}

bool has_repeat(const std::vector<int> &v) {
  for (size_t a = 0; a < v.size(); ++a)
    for (size_t b = a + 1; b < v.size(); ++b)
      if (v[a] == v[b]) return true;
  return false;
}

// User argument bound to canonical slot (member k, position j).
int slot_arg(const Plan &p, int k, int j) {
  return p.spec.arg(p.canon.member_map[k], p.canon.pos_map[j]);
}

// Stride of source s of the operand at canonical position j (an argument)
// along canonical index c (summed over repeated axes; 0 if absent).
int64_t stride_of(const Plan &p, int arg, int j, int s, int c) {
  const Operand &o = p.spec.args[arg];
  int64_t st = 0;
  const auto &labels = p.canon.form.ins[j];
  for (int d = 0; d < (int)labels.size(); ++d)
    if (labels[d] == c) st += o.src_strides[s][d];
  return st;
}

// Axis of canonical index c in the operand at canonical position j.
int axis_of(const Plan &p, int j, int c) {
  const auto &labels = p.canon.form.ins[j];
  for (int d = 0; d < (int)labels.size(); ++d)
    if (labels[d] == c) return d;
  return -1;
}

void analyse_fem_grad(Plan &p) {
  const CanonEinsum &e = p.canon.form;
  auto fail = [&](const char *why) {
    p.fem_ok = false;
    p.fem_why = why;
  };
  if (p.adjoint) return fail("adjoint plans sum members");
  if (p.spec.dtype != BES_FLOAT32 && p.spec.dtype != BES_FLOAT64) return fail("dtype");
  if (e.b > BES_FEM_MAX_MEMBERS) return fail("b > 8");
  if (e.n != 2 && e.n != 3) return fail("n not in {2,3}");
  for (const auto &l : e.ins)
    if (has_repeat(l)) return fail("repeated index");
  // Stream index: the output index of strictly largest extent.
  int E = -1;
  int64_t best = -1;
  bool tie = false;
  for (int c : e.out) {
    if (e.extent[c] > best) {
      best = e.extent[c];
      E = c;
      tie = false;
    } else if (e.extent[c] == best) {
      tie = true;
    }
  }
  if (E < 0) return fail("no output index");
  for (int c = 0; c < (int)e.extent.size(); ++c)
    if (c != E && e.extent[c] >= best) tie = true;
  if (tie) return fail("no unique stream index");
  FemRoles R;
  R.e = E;
  std::vector<int> with_e, without_e;
  for (int j = 0; j < e.n; ++j) (contains(e.ins[j], E) ? with_e : without_e).push_back(j);
  if (without_e.size() != 1) return fail("need exactly one operand without the stream index");
  R.posS = without_e[0];
  const auto &S = e.ins[R.posS];
  auto in_out = [&](int c) { return contains(e.out, c); };
  if (e.n == 2) {
    R.posU = with_e[0];
    const auto &U = e.ins[R.posU];
    if (U.size() != 2 || S.size() != 2) return fail("2-operand form needs S[i,j], U[e,j]");
    int j = U[0] == E ? U[1] : U[0];
    if (!contains(S, j) || in_out(j)) return fail("U's contracted index must be in S");
    int i = S[0] == j ? S[1] : S[0];
    if (!in_out(i) || contains(U, i)) return fail("S's free index must be an output index");
    if (e.out.size() != 2) return fail("output must be (e, i)");
    R.i = i;
    R.j = j;
  } else {
    // Which e-operand is U = {e, j}: j shared with S only and contracted.
    // When both qualify (G = {e, r} has the same pattern), take the one whose
    // argument repeats across the most members, so that stage 1 is hoisted
    // out of the member loop; then the larger contracted extent (cheaper
    // stage 2); then the lower canonical position.
    int cand = -1;
    int best_distinct = 1 << 30;
    int64_t best_ext = -1;
    for (int k = 0; k < 2; ++k) {
      const auto &X = e.ins[with_e[k]];
      const auto &Y = e.ins[with_e[1 - k]];
      if (X.size() != 2) continue;
      int j = X[0] == E ? X[1] : X[0];
      if (!(contains(S, j) && !in_out(j) && !contains(Y, j))) continue;
      // the extents this choice gives the kernel must be compiled
      int rr = -1, xx = -1, ii = -1;
      for (int c : Y) {
        if (c == E) continue;
        if (contains(S, c) && !in_out(c)) rr = c;
        else if (in_out(c) && !contains(S, c)) xx = c;
      }
      for (int c : S)
        if (c != rr && c != j) ii = c;
      if (rr >= 0 && ii >= 0 && S.size() == 3 &&
          !fem_shape_compiled(p.spec.dtype == BES_FLOAT64, (int)e.extent[ii], (int)e.extent[j],
                              (int)e.extent[rr], xx >= 0 ? (int)e.extent[xx] : 1))
        continue;
      std::vector<int> distinct;
      for (int m = 0; m < e.b; ++m) {
        int a = e.arg(m, with_e[k]);
        if (!contains(distinct, a)) distinct.push_back(a);
      }
      int nd = (int)distinct.size();
      if (nd < best_distinct || (nd == best_distinct && e.extent[j] > best_ext)) {
        best_distinct = nd;
        best_ext = e.extent[j];
        cand = k;
        R.j = j;
      }
    }
    if (cand < 0) return fail("no U[e,j] operand");
    R.posU = with_e[cand];
    R.posG = with_e[1 - cand];
    const auto &G = e.ins[R.posG];
    if (S.size() != 3) return fail("3-operand form needs S[r,i,j]");
    int r = -1, x = -1;
    for (int c : G) {
      if (c == E) continue;
      if (contains(S, c) && !in_out(c)) {
        if (r >= 0) return fail("G has two contracted indices");
        r = c;
      } else if (in_out(c) && !contains(S, c)) {
        if (x >= 0) return fail("G has two free indices");
        x = c;
      } else {
        return fail("G index with unsupported role");
      }
    }
    if (r < 0) return fail("G lacks a contracted index shared with S");
    int i = -1;
    for (int c : S)
      if (c != r && c != R.j) i = c;
    if (i < 0 || !in_out(i)) return fail("S's free index must be an output index");
    if (e.out.size() != (size_t)(x >= 0 ? 3 : 2)) return fail("output must be (e, [x,] i)");
    if (G.size() != (size_t)(x >= 0 ? 3 : 2)) return fail("G must be (e, [x,] r)");
    R.i = i;
    R.r = r;
    R.x = x;
  }
  R.NI = (int)e.extent[R.i];
  R.NJ = (int)e.extent[R.j];
  R.NR = R.r >= 0 ? (int)e.extent[R.r] : 1;
  R.NX = R.x >= 0 ? (int)e.extent[R.x] : 1;
  if (!fem_shape_compiled(p.spec.dtype == BES_FLOAT64, R.NI, R.NJ, R.NR, R.NX))
    return fail("no compiled instantiation for these extents");
  // Operand kinds (S may have any strides: the launcher packs it).
  for (int k = 0; k < e.b; ++k) {
    const Operand &s = p.spec.args[slot_arg(p, k, R.posS)];
    if (s.kind != BES_ARRAY && s.kind != BES_VIEW) return fail("S must be an array or view");
    const Operand &u = p.spec.args[slot_arg(p, k, R.posU)];
    if (u.kind == BES_TET_JACOBIAN) return fail("U cannot be a Jacobian operand");
    if (u.kind == BES_EXPR) return fail("expression operands run on the generic template");
    if (R.posG >= 0) {
      const Operand &g = p.spec.args[slot_arg(p, k, R.posG)];
      if (g.kind == BES_EXPR) return fail("expression operands run on the generic template");
      if (g.kind == BES_TET_JACOBIAN && (R.NX != 3 || R.NR != 3))
        return fail("Jacobian operand needs x = r = 3");
    }
    // The kernel addresses a 64-element tile with 32-bit element offsets.
    for (int pos : {R.posU, R.posG}) {
      if (pos < 0) continue;
      const Operand &o = p.spec.args[slot_arg(p, k, pos)];
      for (int s = 0; s < o.nsrc; ++s) {
        int64_t span = 0;
        for (int d = 0; d < o.ndim; ++d) {
          int64_t st = o.src_strides[s][d] < 0 ? -o.src_strides[s][d] : o.src_strides[s][d];
          int64_t ext = (o.kind == BES_TET_JACOBIAN) ? 4 : o.shape[d];
          span += (d == 0 ? 64 : ext) * st;
        }
        if (span >= ((int64_t)1 << 31)) return fail("per-tile offsets exceed 32 bits");
      }
    }
  }
  p.fem = R;
  p.fem_ok = true;
  p.fem_why.clear();
}

// The "apply" class of the FEM-stream template (face mass and local
// divergence, Section "Batched einsums in DG-FEM Operators"): three operands,
// output (e, i); S[c, i, j] without the stream index; G[x, c, e] (or G[c, e]:
// diagonal in the component, face mass) and U[x, e, j] (U[c, e, j]) with it.
// S and G must be the same arguments in every member.
void analyse_fem_apply(Plan &p) {
  const CanonEinsum &e = p.canon.form;
  auto fail = [&](const char *why) {
    p.fem_ok = false;
    p.fem_why = std::string("apply class: ") + why;
  };
  if (p.adjoint) return fail("adjoint plans sum members");
  if (p.spec.dtype != BES_FLOAT32 && p.spec.dtype != BES_FLOAT64) return fail("dtype");
  if (e.b > BES_FEM_APPLY_MAX_MEMBERS) return fail("b > 16");
  if (e.n != 3) return fail("n != 3");
  if (e.out.size() != 2) return fail("output must be (e, i)");
  for (const auto &l : e.ins)
    if (has_repeat(l)) return fail("repeated index");
  const int E = e.extent[e.out[0]] > e.extent[e.out[1]] ? e.out[0]
                : e.extent[e.out[1]] > e.extent[e.out[0]] ? e.out[1] : -1;
  if (E < 0) return fail("no unique stream index");
  for (int c = 0; c < (int)e.extent.size(); ++c)
    if (c != E && e.extent[c] >= e.extent[E]) return fail("no unique stream index");
  const int I = e.out[0] == E ? e.out[1] : e.out[0];
  std::vector<int> with_e, without_e;
  for (int j = 0; j < e.n; ++j) (contains(e.ins[j], E) ? with_e : without_e).push_back(j);
  if (without_e.size() != 1 || with_e.size() != 2) return fail("need one operand without e");
  FemRoles R;
  R.cls = 1;
  R.e = E;
  R.i = I;
  R.posS = without_e[0];
  const auto &S = e.ins[R.posS];
  if (S.size() != 3 || !contains(S, I)) return fail("S must be (c, i, j)");
  std::vector<int> sc;
  for (int c : S)
    if (c != I) sc.push_back(c);
  // Every assignment of (U, G) and (c, j) that matches the pattern; the
  // divergence pattern is symmetric under (G, c) <-> (U, j), so prefer a G
  // that all members share, then a compiled instantiation.
  std::vector<FemRoles> cands;
  for (int pu = 0; pu < 2; ++pu) {
    const auto &U = e.ins[with_e[pu]];
    const auto &G = e.ins[with_e[1 - pu]];
    if (U.size() != 3 || contains(U, I) || contains(G, I)) continue;
    for (int t = 0; t < 2; ++t) {
      const int c = sc[t], j = sc[1 - t];
      if (!contains(U, j) || contains(G, j) || !contains(G, c)) continue;
      FemRoles C = R;
      if (G.size() == 2 && contains(U, c)) {              // G[c, e], U[c, e, j]
        C.diag = true;
        C.r = c;
        C.x = c;
      } else if (G.size() == 3 && !contains(U, c)) {      // G[x, c, e], U[x, e, j]
        int x = -1;
        for (int q : G)
          if (q != E && q != c) x = q;
        if (x < 0 || !contains(U, x) || contains(S, x) || contains(e.out, x)) continue;
        C.diag = false;
        C.r = c;
        C.x = x;
      } else {
        continue;
      }
      C.j = j;
      C.posU = with_e[pu];
      C.posG = with_e[1 - pu];
      C.NI = (int)e.extent[C.i];
      C.NJ = (int)e.extent[C.j];
      C.NR = (int)e.extent[C.r];
      C.NX = (int)e.extent[C.x];
      cands.push_back(C);
    }
  }
  if (cands.empty()) return fail("operands do not match S[c,i,j], G[x,c,e], U[x,e,j]");
  auto shared_g = [&](const FemRoles &C) {
    for (int k = 1; k < e.b; ++k)
      if (slot_arg(p, k, C.posG) != slot_arg(p, 0, C.posG)) return false;
    return true;
  };
  int best = -1, best_score = -1;
  for (size_t q = 0; q < cands.size(); ++q) {
    const FemRoles &C = cands[q];
    const int score = (shared_g(C) ? 2 : 0) +
                      (fem_apply_shape_listed(C.NI, C.NJ, C.NR, C.NX, C.diag) ? 1 : 0);
    if (score > best_score) {
      best_score = score;
      best = (int)q;
    }
  }
  R = cands[best];
  if (!fem_apply_shape_listed(R.NI, R.NJ, R.NR, R.NX, R.diag))
    return fail("no compiled instantiation for these extents");
  const int s0 = slot_arg(p, 0, R.posS), g0 = slot_arg(p, 0, R.posG);
  const int u0 = slot_arg(p, 0, R.posU);
  const Operand &uo = p.spec.args[u0];
  for (int k = 0; k < e.b; ++k) {
    if (slot_arg(p, k, R.posS) != s0 || slot_arg(p, k, R.posG) != g0)
      return fail("S and G must be shared by every member");
    const Operand &u = p.spec.args[slot_arg(p, k, R.posU)];
    if (u.kind == BES_TET_JACOBIAN) return fail("U cannot be a Jacobian operand");
    if (u.kind == BES_EXPR) return fail("expression operands run on the generic template");
    if ((u.kind == BES_ELEMENTWISE) != (uo.kind == BES_ELEMENTWISE) || u.op != uo.op ||
        u.alpha != uo.alpha || u.beta != uo.beta)
      return fail("every member's U must be the same kind of function");
    // per-lane offsets inside a 64-element tile are 32-bit
    const int ua = slot_arg(p, k, R.posU);
    for (int sidx = 0; sidx < u.nsrc; ++sidx) {
      const int64_t se = stride_of(p, ua, R.posU, sidx, R.e);
      const int64_t sj = stride_of(p, ua, R.posU, sidx, R.j);
      const int64_t span = 64 * (se < 0 ? -se : se) + R.NJ * (sj < 0 ? -sj : sj);
      if (span >= ((int64_t)1 << 31)) return fail("per-tile offsets exceed 32 bits");
    }
  }
  for (int a : {s0, g0}) {
    const Operand &o = p.spec.args[a];
    if (o.kind != BES_ARRAY && o.kind != BES_VIEW) return fail("S and G must be arrays or views");
  }
  p.fem = R;
  p.fem_ok = true;
  p.fem_why.clear();
}

void analyse_fem(Plan &p) {
  analyse_fem_grad(p);
  if (p.fem_ok) return;
  const std::string why_grad = p.fem_why;
  analyse_fem_apply(p);
  if (!p.fem_ok) p.fem_why = why_grad + "; " + p.fem_why;
}

// Merged stride of a group of canonical indices (in merge order) for one
// operand; false if the group does not merge into one strided axis.
bool merge_group(const Plan &p, int arg, int j, const std::vector<int> &grp,
                 const std::vector<int64_t> &ext, int64_t &stride) {
  if (grp.empty()) {
    stride = 0;
    return true;
  }
  for (size_t k = 0; k + 1 < grp.size(); ++k) {
    int64_t a = stride_of(p, arg, j, 0, grp[k]);
    int64_t b = stride_of(p, arg, j, 0, grp[k + 1]);
    if (a != b * ext[grp[k + 1]]) return false;
  }
  stride = stride_of(p, arg, j, 0, grp.back());
  return true;
}

// Merged stride of an index group in an output with strides `st` along
// `out`; false if the group does not merge into one strided axis.
bool merge_out_strided(const std::vector<int> &out, const std::vector<int64_t> &st,
                       const std::vector<int> &grp, const std::vector<int64_t> &ext,
                       int64_t &stride) {
  auto sof = [&](int c) {
    for (size_t d = 0; d < out.size(); ++d)
      if (out[d] == c) return st[d];
    return (int64_t)0;
  };
  for (size_t k = 0; k + 1 < grp.size(); ++k)
    if (sof(grp[k]) != sof(grp[k + 1]) * ext[grp[k + 1]]) return false;
  stride = grp.empty() ? 0 : sof(grp.back());
  return true;
}

void analyse_mfma(Plan &p) {
  const CanonEinsum &e = p.canon.form;
  auto fail = [&](const char *why) {
    p.mfma_ok = false;
    p.mfma_why = why;
  };
  if (p.spec.dtype != BES_FLOAT32) return fail("MFMA template is FP32");
  if (e.n != 2) return fail("n != 2");
  if (e.b > BES_MFMA_MAX_B) return fail("b > 8");
  if (e.out.empty()) return fail("scalar output");
  for (const auto &l : e.ins)
    if (has_repeat(l)) return fail("repeated index");
  const int nidx = (int)e.extent.size();
  for (int c = 0; c < nidx; ++c) {
    int cnt = contains(e.ins[0], c) + contains(e.ins[1], c) + contains(e.out, c);
    if (cnt != 2) return fail("not a pure two-operand contraction");
  }
  MfmaRoles R;
  R.posA = contains(e.ins[0], e.out[0]) ? 0 : 1;
  R.posB = 1 - R.posA;
  for (int c : e.out) (contains(e.ins[R.posA], c) ? R.Mi : R.Ni).push_back(c);
  for (int c : e.ins[R.posA])
    if (contains(e.ins[R.posB], c)) R.Ki.push_back(c);
  if (R.Ni.empty() || R.Ki.empty()) return fail("degenerate GEMM shape");
  // Output must be (M group, N group) or (N group, M group) as one block each.
  std::vector<int> mn = R.Mi, nm = R.Ni;
  mn.insert(mn.end(), R.Ni.begin(), R.Ni.end());
  nm.insert(nm.end(), R.Mi.begin(), R.Mi.end());
  if (e.out == mn) R.c_mn = true;
  else if (e.out == nm) R.c_mn = false;
  else return fail("output interleaves M and N indices");
  R.M = R.N = R.K = 1;
  for (int c : R.Mi) R.M *= e.extent[c];
  for (int c : R.Ni) R.N *= e.extent[c];
  for (int c : R.Ki) R.K *= e.extent[c];
  if (R.M % 128 || R.N % 128 || R.K % 16)
    return fail("M, N not multiples of 128 or K of 16");
  int64_t st;
  for (int k = 0; k < e.b; ++k) {
    int a = slot_arg(p, k, R.posA), b = slot_arg(p, k, R.posB);
    for (int arg : {a, b}) {
      const Operand &o = p.spec.args[arg];
      if (o.kind != BES_ARRAY && o.kind != BES_VIEW) return fail("MFMA operands must be arrays or views");
    }
    if (!merge_group(p, a, R.posA, R.Mi, e.extent, st) ||
        !merge_group(p, a, R.posA, R.Ki, e.extent, st) ||
        !merge_group(p, b, R.posB, R.Ki, e.extent, st) ||
        !merge_group(p, b, R.posB, R.Ni, e.extent, st))
      return fail("an index group does not merge into one strided axis");
  }
  p.mf = R;
  p.mfma_ok = true;
  p.mfma_why.clear();
}

// Any pure binary contraction (every index in exactly two of A, B and the
// output) with array, view or affine (alpha*S0 + beta) operands.
void analyse_gett(Plan &p) {
  const CanonEinsum &e = p.canon.form;
  auto fail = [&](const char *why) {
    p.gett_ok = false;
    p.gett_why = why;
  };
  if (p.spec.dtype != BES_FLOAT32 && p.spec.dtype != BES_FLOAT64) return fail("dtype");
  if (e.n != 2) return fail("n != 2");
  if (e.b > BES_GETT_MAX_B) return fail("b > 8");
  for (const auto &l : e.ins)
    if (has_repeat(l)) return fail("repeated index");
  const int nidx = (int)e.extent.size();
  for (int c = 0; c < nidx; ++c) {
    const int cnt = contains(e.ins[0], c) + contains(e.ins[1], c) + contains(e.out, c);
    if (cnt != 2) return fail("not a pure two-operand contraction");
  }
  GettRoles R;
  R.posA = (!e.out.empty() && contains(e.ins[1], e.out[0]) && !contains(e.ins[0], e.out[0]))
               ? 1 : 0;
  R.posB = 1 - R.posA;
  for (int c : e.out) (contains(e.ins[R.posA], c) ? R.Mi : R.Ni).push_back(c);
  for (int c : e.ins[R.posA])
    if (contains(e.ins[R.posB], c)) R.Ki.push_back(c);
  for (int c : R.Mi) R.M *= e.extent[c];
  for (int c : R.Ni) R.N *= e.extent[c];
  for (int c : R.Ki) R.K *= e.extent[c];
  // Linearize each group in its operand's memory order (largest stride
  // first) so that consecutive tile rows or columns are consecutive
  // addresses: M by A's strides, N by B's, K by A's unless only B is
  // contiguous along K (first member's layout; the tables hold any order).
  const int a0 = slot_arg(p, 0, R.posA), b0 = slot_arg(p, 0, R.posB);
  auto by_stride = [&](std::vector<int> &g, int arg, int pos) {
    std::stable_sort(g.begin(), g.end(), [&](int x, int y) {
      int64_t sx = stride_of(p, arg, pos, 0, x), sy = stride_of(p, arg, pos, 0, y);
      return (sx < 0 ? -sx : sx) > (sy < 0 ? -sy : sy);
    });
  };
  auto unit_in = [&](const std::vector<int> &g, int arg, int pos) {
    for (int c : g) {
      const int64_t st = stride_of(p, arg, pos, 0, c);
      if (st == 1 || st == -1) return true;
    }
    return false;
  };
  by_stride(R.Mi, a0, R.posA);
  by_stride(R.Ni, b0, R.posB);
  if (unit_in(R.Ki, b0, R.posB) && !unit_in(R.Ki, a0, R.posA)) by_stride(R.Ki, b0, R.posB);
  else by_stride(R.Ki, a0, R.posA);
  for (int k = 0; k < e.b; ++k)
    for (int pos : {R.posA, R.posB}) {
      const Operand &o = p.spec.args[slot_arg(p, k, pos)];
      const bool affine = o.kind == BES_ELEMENTWISE && o.op == BES_OP_ID && o.nsrc == 1;
      if (o.kind != BES_ARRAY && o.kind != BES_VIEW && !affine)
        return fail("operands must be arrays, views or alpha*S+beta");
    }
  p.gt = R;
  p.gett_ok = true;
  p.gett_why.clear();
}

}  // namespace

namespace {

// Offsets of every multi-index of a group (last index fastest) for one set of
// strides: out[l] = sum_d idx_d(l) * stride_d.
void group_offsets(const std::vector<int64_t> &ext, const std::vector<int64_t> &st,
                   std::vector<int64_t> &out) {
  int64_t n = 1;
  for (int64_t x : ext) n *= x;
  const size_t base = out.size();
  out.resize(base + (size_t)std::max<int64_t>(n, 1), 0);
  if (n <= 0) return;
  std::vector<int64_t> idx(ext.size(), 0);
  int64_t off = 0;
  for (int64_t l = 0; l < n; ++l) {
    out[base + l] = off;
    for (int d = (int)ext.size() - 1; d >= 0; --d) {
      if (++idx[d] < ext[d]) {
        off += st[d];
        break;
      }
      off -= (ext[d] - 1) * st[d];
      idx[d] = 0;
    }
  }
}

}  // namespace

int bind_gett_static(const Plan &p, std::vector<int64_t> &tab, GettArgs &a, std::string &err) {
  if (!p.gett_ok) {
    err = "plan is not a binary contraction: " + p.gett_why;
    return BES_E_UNSUPPORTED;
  }
  const GettRoles &R = p.gt;
  const CanonEinsum &e = p.canon.form;
  std::memset(&a, 0, sizeof a);
  a.M = R.M;
  a.N = R.N;
  a.K = R.K;
  a.n_members = e.b;
  a.n_slots = p.n_slots;
  tab.clear();
  auto exts = [&](const std::vector<int> &g) {
    std::vector<int64_t> x;
    for (int c : g) x.push_back(e.extent[c]);
    return x;
  };
  auto strides = [&](int arg, int pos, const std::vector<int> &g) {
    std::vector<int64_t> x;
    for (int c : g) x.push_back(stride_of(p, arg, pos, 0, c));
    return x;
  };
  const std::vector<int64_t> eM = exts(R.Mi), eN = exts(R.Ni), eK = exts(R.Ki);
  std::vector<int> order;
  for (int sl = 0; sl < p.n_slots; ++sl)
    for (int k = 0; k < e.b; ++k)
      if (p.slot_of_member[p.canon.member_map[k]] == sl) order.push_back(k);
  int m = 0;
  for (int sl = 0; sl < p.n_slots; ++sl) {
    GettSlot &S = a.slot[sl];
    const std::vector<int64_t> ost = out_strides(p, sl);
    auto ostride = [&](const std::vector<int> &g) {
      std::vector<int64_t> x;
      for (int c : g)
        for (size_t d = 0; d < e.out.size(); ++d)
          if (e.out[d] == c) x.push_back(ost[d]);
      return x;
    };
    S.rowC = (int64_t)tab.size();
    group_offsets(eM, ostride(R.Mi), tab);
    S.colC = (int64_t)tab.size();
    group_offsets(eN, ostride(R.Ni), tab);
    S.acc = p.out_layout[sl].accumulate ? 1 : 0;
    S.m0 = m;
    for (int k : order) {
      if (p.slot_of_member[p.canon.member_map[k]] != sl) continue;
      GettMember &M = a.mem[m++];
      const int aa = slot_arg(p, k, R.posA), bb = slot_arg(p, k, R.posB);
      const Operand &oa = p.spec.args[aa], &ob = p.spec.args[bb];
      M.rowA = (int64_t)tab.size();
      group_offsets(eM, strides(aa, R.posA, R.Mi), tab);
      M.colA = (int64_t)tab.size();
      group_offsets(eK, strides(aa, R.posA, R.Ki), tab);
      M.rowB = (int64_t)tab.size();
      group_offsets(eK, strides(bb, R.posB, R.Ki), tab);
      M.colB = (int64_t)tab.size();
      group_offsets(eN, strides(bb, R.posB, R.Ni), tab);
      const bool affA = oa.kind == BES_ELEMENTWISE, affB = ob.kind == BES_ELEMENTWISE;
      M.a_alpha = affA ? oa.alpha : 1.0;
      M.a_beta = affA ? oa.beta : 0.0;
      M.b_alpha = affB ? ob.alpha : 1.0;
      M.b_beta = affB ? ob.beta : 0.0;
      // read each tile along the side on which the operand is contiguous
      auto unit = [&](int64_t off) { return R.K > 1 && (tab[off + 1] - tab[off] == 1 ||
                                                        tab[off + 1] - tab[off] == -1); };
      M.a_kfast = unit(M.colA) ? 1 : 0;
      M.b_nfast = unit(M.rowB) ? 0 : 1;
    }
    S.m1 = m;
  }
  return BES_OK;
}

void bind_gett_ptrs(const Plan &p, const void *const *src, void *const *out, GettArgs &a) {
  const GettRoles &R = p.gt;
  const CanonEinsum &e = p.canon.form;
  const int64_t item = p.spec.dtype == BES_FLOAT64 ? 8 : 4;
  std::vector<int> order;
  for (int sl = 0; sl < p.n_slots; ++sl)
    for (int k = 0; k < e.b; ++k)
      if (p.slot_of_member[p.canon.member_map[k]] == sl) order.push_back(k);
  int m = 0;
  for (int sl = 0; sl < p.n_slots; ++sl) {
    a.slot[sl].C = (char *)out[sl] +
                   (p.out_layout[sl].custom ? p.out_layout[sl].offset * item : 0);
    for (int k : order) {
      if (p.slot_of_member[p.canon.member_map[k]] != sl) continue;
      GettMember &M = a.mem[m++];
      const int aa = slot_arg(p, k, R.posA), bb = slot_arg(p, k, R.posB);
      M.A = (const char *)src[p.src_base[aa]] + p.spec.args[aa].src_offset[0] * item;
      M.B = (const char *)src[p.src_base[bb]] + p.spec.args[bb].src_offset[0] * item;
    }
  }
}

bool template_supported(const Plan &p, int t) {
  switch (t) {
    case BES_T_FEM_STREAM: return p.fem_ok;
    case BES_T_MFMA: return p.mfma_ok && kMfmaTemplateReady;
    case BES_T_GETT: return p.gett_ok;
    case BES_T_GENERIC:
      return (p.spec.dtype == BES_FLOAT32 || p.spec.dtype == BES_FLOAT64) &&
             p.spec.b <= BES_GEN_MAX_B && p.spec.n <= BES_GEN_MAX_OPS &&
             (int)p.canon.form.out.size() <= BES_GEN_MAX_IDX &&
             (int)p.canon.form.extent.size() - (int)p.canon.form.out.size() <= BES_GEN_MAX_IDX;
    default: return false;
  }
}

bes_config default_config(const Plan &p) {
  bes_config c{};
  if (p.mfma_ok && kMfmaTemplateReady) {
    c.template_id = BES_T_MFMA;
    c.p[0] = 128;
    c.p[1] = 128;
  } else if (p.fem_ok && p.fem.cls == 1) {
    c.template_id = BES_T_FEM_STREAM;
    c.p[0] = 64;   // elements per tile
    c.p[1] = 8;    // blocks of four waves per CU in the grid
  } else if (p.fem_ok) {
    c.template_id = BES_T_FEM_STREAM;
    c.p[0] = 64;   // elements per tile
    c.p[1] = 64;   // blocks per CU in the grid: one tile per block at
                   // e = 2^20 (measured best for the lean kernel)
    c.p[2] = 0;    // lean kernel, two waves per tile, where the batch allows
  } else if (p.gett_ok && std::min(p.gt.M, p.gt.N) >= 4 &&
             p.gt.M * p.gt.N * std::max<int64_t>(p.gt.K, 1) >= ((int64_t)1 << 20)) {
    // a contraction large enough to fill the 64 x 64 matrix-core tiles
    c.template_id = BES_T_GETT;
    c.p[0] = 64;
    c.p[1] = 64;
  } else if (template_supported(p, BES_T_GENERIC)) {
    // Lanes per output grow with the shared contraction length (about 64
    // rows per lane; the generic template splits those rows across lanes and
    // sums each operand's exclusive indices inside the operand).
    const CanonEinsum &f = p.canon.form;
    int64_t con = 1;
    bool any_shared = false;
    for (int c2 = 0; c2 < (int)f.extent.size(); ++c2) {
      if (std::find(f.out.begin(), f.out.end(), c2) != f.out.end()) continue;
      int h = 0;
      for (const auto &l : f.ins) h += std::find(l.begin(), l.end(), c2) != l.end() ? 1 : 0;
      if (h >= 2) {
        con *= f.extent[c2];
        any_shared = true;
      }
    }
    if (!any_shared)   // the largest exclusive set takes the shared place
      for (const auto &l : f.ins) {
        int64_t ex = 1;
        for (int c2 : l)
          if (std::find(f.out.begin(), f.out.end(), c2) == f.out.end()) ex *= f.extent[c2];
        con = std::max(con, ex);
      }
    int lanes = 1;
    while (lanes < 64 && (int64_t)lanes * 64 < con) lanes *= 2;
    // Few outputs over a long shared contraction: split the shared space
    // into chunks that add into the zeroed outputs (more work items).
    int64_t outs = (int64_t)p.n_slots;
    for (int c2 : f.out) outs *= f.extent[c2];
    int split = 1;
    while (split < 64 && outs * split < 4096 && con / (split * 2) >= 1024) split *= 2;
    c.template_id = BES_T_GENERIC;
    c.p[0] = 256;
    c.p[1] = lanes;
    c.p[2] = split;
  } else {
    c.template_id = BES_T_AUTO;  // nothing evaluates this plan
  }
  return c;
}

std::vector<int64_t> dense_out_strides(const Plan &p) {
  const Spec &s = p.spec;
  std::vector<int64_t> st(s.out.size());
  int64_t v = 1;
  for (int d = (int)s.out.size() - 1; d >= 0; --d) {
    st[d] = v;
    v *= s.extent[s.out[d]];
  }
  return st;
}

std::vector<int64_t> out_strides(const Plan &p, int slot) {
  if (slot < (int)p.out_layout.size() && p.out_layout[slot].custom) {
    const OutLayout &L = p.out_layout[slot];
    return std::vector<int64_t>(L.stride, L.stride + p.spec.out.size());
  }
  return dense_out_strides(p);
}

bool outputs_plain(const Plan &p) {
  for (const OutLayout &L : p.out_layout)
    if (L.custom || L.accumulate) return false;
  return true;
}

bool any_accumulate(const Plan &p) {
  for (const OutLayout &L : p.out_layout)
    if (L.accumulate) return true;
  return false;
}

int build_plan(Plan &p, std::string &err) {
  int rc = canonicalize(p.spec, p.canon, err);
  if (rc) return rc;
  p.key = key_string(p.canon.form);
  p.tuple = tuple_string(p.canon.form);
  if (p.slot_of_member.empty()) {
    p.slot_of_member.resize(p.spec.b);
    for (int i = 0; i < p.spec.b; ++i) p.slot_of_member[i] = i;
    p.n_slots = p.spec.b;
  }
  p.out_layout.assign(p.n_slots, OutLayout());
  p.exprs.clear();
  for (const Operand &o : p.spec.args)
    if (o.kind == BES_EXPR && std::find(p.exprs.begin(), p.exprs.end(), o.expr) == p.exprs.end())
      p.exprs.push_back(o.expr);
  p.src_base.resize(p.spec.args.size());
  p.n_src = 0;
  for (size_t a = 0; a < p.spec.args.size(); ++a) {
    p.src_base[a] = p.n_src;
    p.n_src += p.spec.args[a].nsrc;
  }
  analyse_fem(p);
  analyse_mfma(p);
  analyse_gett(p);
  // A plan no template can evaluate (e.g. an integer dtype) still has a
  // canonical form and a key; launching it reports BES_E_UNSUPPORTED.
  p.cfg = default_config(p);
  return BES_OK;
}

// ---------------------------------------------------------------------------
// Binding
// ---------------------------------------------------------------------------

namespace {

void fill_src(const Plan &p, int arg, int j, const std::vector<int> &roles,
              const void *const *src, FemSrc &f) {
  const Operand &o = p.spec.args[arg];
  std::memset(&f, 0, sizeof f);
  f.p0 = src[p.src_base[arg]];
  f.p1 = o.nsrc > 1 ? src[p.src_base[arg] + 1] : nullptr;
  f.off0 = o.src_offset[0];
  f.off1 = o.nsrc > 1 ? o.src_offset[1] : 0;
  f.op = o.op;
  f.alpha = o.alpha;
  f.beta = o.beta;
  if (o.kind == BES_TET_JACOBIAN) {
    f.kind = FEM_SRC_TET;
    for (int k = 0; k < 3; ++k) f.s0[k] = o.src_strides[0][k];  // V[e, vertex, coord]
    // The operand's axis order is (e, x, r); roles (e, x, r) of the kernel may
    // be swapped relative to it: encode with the sign of s1[0].
    int ax = axis_of(p, j, roles[1]);
    f.s1[0] = (ax == 2) ? 1 : 0;  // 1: kernel x is the operand's r axis
    return;
  }
  f.kind = o.kind == BES_ELEMENTWISE ? FEM_SRC_ELEMENTWISE : FEM_SRC_ARRAY;
  for (size_t k = 0; k < roles.size(); ++k) {
    if (roles[k] < 0) continue;
    f.s0[k] = stride_of(p, arg, j, 0, roles[k]);
    if (o.nsrc > 1) f.s1[k] = stride_of(p, arg, j, 1, roles[k]);
  }
}

}  // namespace

int bind_fem(const Plan &p, const void *const *src, void *const *out, FemArgs &a,
             std::string &err) {
  if (!p.fem_ok || p.fem.cls != 0) {
    err = "plan is not FEM-stream compatible: " + p.fem_why;
    return BES_E_UNSUPPORTED;
  }
  const FemRoles &R = p.fem;
  const CanonEinsum &e = p.canon.form;
  std::memset(&a, 0, sizeof a);
  a.E = e.extent[R.e];
  // Stage-1 groups: canonical members with the same (S, U) arguments, kept
  // contiguous by ordering members by group.
  std::vector<std::pair<int, int>> keys;
  std::vector<int> group_of(e.b);
  for (int k = 0; k < e.b; ++k) {
    std::pair<int, int> key(slot_arg(p, k, R.posS), slot_arg(p, k, R.posU));
    auto it = std::find(keys.begin(), keys.end(), key);
    if (it == keys.end()) {
      group_of[k] = (int)keys.size();
      keys.push_back(key);
    } else {
      group_of[k] = (int)(it - keys.begin());
    }
  }
  a.n_groups = (int)keys.size();
  a.n_members = e.b;
  if (any_accumulate(p)) {
    err = "the FEM-stream template overwrites its outputs";
    return BES_E_UNSUPPORTED;
  }
  const int64_t item = p.spec.dtype == BES_FLOAT64 ? 8 : 4;
  int m = 0;
  for (int g = 0; g < a.n_groups; ++g) {
    FemGroup &G = a.grp[g];
    G.S = src[p.src_base[keys[g].first]];
    const Operand &so = p.spec.args[keys[g].first];
    G.S = (const char *)G.S + so.src_offset[0] * (p.spec.dtype == BES_FLOAT64 ? 8 : 4);
    G.ss[0] = R.r >= 0 ? stride_of(p, keys[g].first, R.posS, 0, R.r) : 0;
    G.ss[1] = stride_of(p, keys[g].first, R.posS, 0, R.i);
    G.ss[2] = stride_of(p, keys[g].first, R.posS, 0, R.j);
    int k0 = -1;
    for (int k = 0; k < e.b; ++k)
      if (group_of[k] == g) {
        k0 = k;
        break;
      }
    fill_src(p, keys[g].second, R.posU, {R.e, R.j}, src, G.u);
    G.m0 = m;
    for (int k = 0; k < e.b; ++k) {
      if (group_of[k] != g) continue;
      FemMember &M = a.mem[m];
      if (R.posG >= 0) {
        fill_src(p, slot_arg(p, k, R.posG), R.posG, {R.e, R.x, R.r}, src, M.g);
      } else {
        std::memset(&M.g, 0, sizeof M.g);
        M.g.kind = FEM_SRC_NONE;
      }
      // Output strides along (e, x, i): the canonical output axes are the
      // caller's output axes in the same order, renamed.
      const int slot = p.slot_of_member[p.canon.member_map[k]];
      const std::vector<int64_t> ost = out_strides(p, slot);
      auto ostride = [&](int c) -> int64_t {
        for (size_t d = 0; d < e.out.size(); ++d)
          if (e.out[d] == c) return ost[d];
        return 0;
      };
      M.out = (char *)out[slot] +
              (p.out_layout[slot].custom ? p.out_layout[slot].offset * item : 0);
      M.oe = ostride(R.e);
      M.ox = R.x >= 0 ? ostride(R.x) : 0;
      M.oi = ostride(R.i);
      M.group = g;
      ++m;
    }
    G.m1 = m;
    (void)k0;
    // Shared G row: all members read one contiguous row of <= 12 components
    // per element from the same source.
    G.g_row = 0;
    G.g_off = 0;
    if (R.posG >= 0 && G.m1 > G.m0) {
      const FemSrc &f0 = a.mem[G.m0].g;
      bool same = true, views = f0.kind == FEM_SRC_ARRAY, tets = f0.kind == FEM_SRC_TET;
      int64_t hi = -1;
      for (int q = G.m0; q < G.m1 && same; ++q) {
        const FemSrc &f = a.mem[q].g;
        same = f.p0 == f0.p0 && f.s0[0] == f0.s0[0] && f.kind == f0.kind;
        if (views) {
          for (int x = 0; x < R.NX && same; ++x)
            for (int r = 0; r < R.NR; ++r) {
              int64_t c = f.off0 + x * f.s0[1] + r * f.s0[2];
              if (c < 0 || c >= 12) same = false;
              hi = std::max(hi, c);
            }
        } else if (tets) {
          same = same && f.off0 == f0.off0 && f.s0[1] == 3 && f.s0[2] == 1;
        } else {
          same = false;
        }
      }
      if (same && f0.s0[0] > 0 && f0.s0[0] < (1 << 24)) {
        G.g_row = views ? (int32_t)(hi + 1) : 12;
        G.g_off = views ? 0 : f0.off0;
      }
    }
  }
  return BES_OK;
}

int bind_fem_apply(const Plan &p, const void *const *src, void *const *out, FemApplyArgs &a,
                   std::string &err) {
  if (!p.fem_ok || p.fem.cls != 1) {
    err = "plan is not of the FEM-stream apply class: " + p.fem_why;
    return BES_E_UNSUPPORTED;
  }
  if (any_accumulate(p)) {
    err = "the FEM-stream template overwrites its outputs";
    return BES_E_UNSUPPORTED;
  }
  const FemRoles &R = p.fem;
  const CanonEinsum &e = p.canon.form;
  const int64_t item = p.spec.dtype == BES_FLOAT64 ? 8 : 4;
  std::memset(&a, 0, sizeof a);
  a.E = e.extent[R.e];
  const int sa = slot_arg(p, 0, R.posS), ga = slot_arg(p, 0, R.posG);
  a.S = (const char *)src[p.src_base[sa]] + p.spec.args[sa].src_offset[0] * item;
  a.ss[0] = stride_of(p, sa, R.posS, 0, R.r);
  a.ss[1] = stride_of(p, sa, R.posS, 0, R.i);
  a.ss[2] = stride_of(p, sa, R.posS, 0, R.j);
  a.G = (const char *)src[p.src_base[ga]] + p.spec.args[ga].src_offset[0] * item;
  a.gs[0] = R.diag ? 0 : stride_of(p, ga, R.posG, 0, R.x);
  a.gs[1] = stride_of(p, ga, R.posG, 0, R.r);
  a.gs[2] = stride_of(p, ga, R.posG, 0, R.e);
  a.n_members = e.b;
  const Operand &u0 = p.spec.args[slot_arg(p, 0, R.posU)];
  a.u_kind = u0.kind == BES_ELEMENTWISE ? FEM_SRC_ELEMENTWISE : FEM_SRC_ARRAY;
  a.op = u0.op;
  a.alpha = u0.alpha;
  a.beta = u0.beta;
  for (int k = 0; k < e.b; ++k) {
    FemApplyMember &M = a.mem[k];
    const int ua = slot_arg(p, k, R.posU);
    const Operand &u = p.spec.args[ua];
    M.u0 = src[p.src_base[ua]];
    M.uoff0 = u.src_offset[0];
    M.us0[0] = stride_of(p, ua, R.posU, 0, R.x);
    M.us0[1] = stride_of(p, ua, R.posU, 0, R.e);
    M.us0[2] = stride_of(p, ua, R.posU, 0, R.j);
    if (u.kind == BES_ELEMENTWISE && u.nsrc > 1) {
      M.u1 = src[p.src_base[ua] + 1];
      M.uoff1 = u.src_offset[1];
      M.us1[0] = stride_of(p, ua, R.posU, 1, R.x);
      M.us1[1] = stride_of(p, ua, R.posU, 1, R.e);
      M.us1[2] = stride_of(p, ua, R.posU, 1, R.j);
    }
    const int slot = p.slot_of_member[p.canon.member_map[k]];
    const std::vector<int64_t> ost = out_strides(p, slot);
    M.out = (char *)out[slot] +
            (p.out_layout[slot].custom ? p.out_layout[slot].offset * item : 0);
    for (size_t d = 0; d < e.out.size(); ++d) {
      if (e.out[d] == R.e) M.oe = ost[d];
      if (e.out[d] == R.i) M.oi = ost[d];
    }
  }
  return BES_OK;
}

int bind_generic_static(const Plan &p, const bes_config &cfg, GenEinsum &g, std::string &err) {
  if (!template_supported(p, BES_T_GENERIC)) {
    err = "generic template limits exceeded";
    return BES_E_UNSUPPORTED;
  }
  const Spec &s = p.spec;
  std::memset(&g, 0, sizeof g);
  g.n_ops = s.n;
  g.b = s.b;
  g.n_out = (int)s.out.size();
  // Contracted indices: shared ones first, then each operand's exclusive
  // ones (an index is exclusive when exactly one operand position carries
  // it, possibly on several axes).
  std::vector<int> con;
  auto holders = [&](int c) {
    int h = 0;
    for (int j = 0; j < s.n; ++j) h += contains(s.ins[j], c) ? 1 : 0;
    return h;
  };
  for (int c : s.used_indices())
    if (!contains(s.out, c) && holders(c) >= 2) con.push_back(c);
  // Without shared indices, the largest exclusive set takes their place, so
  // that the lanes and chunks split its sum.
  int promoted = -1;
  if (con.empty()) {
    int64_t best = 1;
    for (int j = 0; j < s.n; ++j) {
      int64_t ex = 1;
      for (int c : s.used_indices())
        if (!contains(s.out, c) && contains(s.ins[j], c)) ex *= s.extent[c];
      if (ex > best) {
        best = ex;
        promoted = j;
      }
    }
    if (promoted >= 0)
      for (int c : s.used_indices())
        if (!contains(s.out, c) && contains(s.ins[promoted], c)) con.push_back(c);
  }
  g.n_sh = (int)con.size();
  g.row_dep = 0;
  for (int j = 0; j < s.n; ++j) {
    g.ex_off[j] = (int)con.size();
    if (j != promoted)
      for (int c : s.used_indices())
        if (!contains(s.out, c) && holders(c) == 1 && contains(s.ins[j], c)) con.push_back(c);
    g.ex_n[j] = (int)con.size() - g.ex_off[j];
    for (int q = 0; q < g.n_sh; ++q)
      if (contains(s.ins[j], con[q])) g.row_dep |= 1 << j;
  }
  g.n_con = (int)con.size();
  g.out_size = 1;
  for (int d = g.n_out - 1; d >= 0; --d) {
    g.out_ext[d] = s.extent[s.out[d]];
    g.out_size *= g.out_ext[d];
  }
  g.o_dense = outputs_plain(p) ? 1 : 0;
  for (int sl = 0; sl < p.n_slots; ++sl) {
    std::vector<int64_t> st = out_strides(p, sl);
    for (int d = 0; d < g.n_out; ++d) g.o_str[sl][d] = st[d];
    const OutLayout *L = sl < (int)p.out_layout.size() ? &p.out_layout[sl] : nullptr;
    g.o_off[sl] = L && L->custom ? L->offset : 0;
    g.o_acc[sl] = L && L->accumulate ? 1 : 0;
  }
  g.con_size = 1;
  for (int d = 0; d < g.n_con; ++d) {
    g.con_ext[d] = s.extent[con[d]];
    g.con_size *= g.con_ext[d];
  }
  g.sh_size = 1;
  for (int d = 0; d < g.n_sh; ++d) g.sh_size *= g.con_ext[d];
  for (int j = 0; j < s.n; ++j) {
    g.ex_size[j] = 1;
    for (int d = 0; d < g.ex_n[j]; ++d) g.ex_size[j] *= g.con_ext[g.ex_off[j] + d];
  }
  // 32-bit decoding: multipliers for every extent, each checked at the
  // edges of its range (any failure keeps the 64-bit path)
  const int64_t lim = (int64_t)1 << 31;
  bool narrow = g.out_size < lim && g.sh_size < lim;
  for (int k = 0; k < s.n; ++k) narrow = narrow && g.ex_size[k] < lim;
  auto magic = [&](int64_t ext, uint32_t &mul, int32_t &shift) {
    if (ext <= 1) {
      mul = 1;
      shift = 0;
      return true;
    }
    int l = 0;
    while (((int64_t)1 << l) < ext) ++l;
    mul = (uint32_t)((((uint64_t)1 << 32) * (((uint64_t)1 << l) - (uint64_t)ext)) / (uint64_t)ext +
                     1);
    shift = l;
    for (uint32_t x : {0u, (uint32_t)ext - 1, (uint32_t)ext, 2u * (uint32_t)ext - 1,
                       (uint32_t)(lim - 1)}) {
      const uint32_t hi = (uint32_t)(((uint64_t)x * mul) >> 32);
      if ((uint32_t)((hi + x) >> shift) != x / (uint32_t)ext) return false;
    }
    return true;
  };
  for (int d = 0; d < BES_GEN_MAX_IDX; ++d) {
    if (d < g.n_out) narrow = narrow && magic(g.out_ext[d], g.out_mul[d], g.out_shift[d]);
    if (d < g.n_con) narrow = narrow && magic(g.con_ext[d], g.con_mul[d], g.con_shift[d]);
  }
  g.narrow = narrow ? 1 : 0;
  g.tile = cfg.p[0] > 0 ? cfg.p[0] : 256;
  g.lanes = cfg.p[1] > 0 ? cfg.p[1] : 1;
  g.split = cfg.p[2] > 0 ? cfg.p[2] : 1;
  if (g.split > 64) {
    err = "split of the shared space must be <= 64";
    return BES_E_INVALID;
  }
  if (g.lanes > 64 || (g.lanes & (g.lanes - 1))) {
    err = "lanes per output must be a power of two <= 64";
    return BES_E_INVALID;
  }
  g.n_layouts = 0;
  for (int m = 0; m < s.b; ++m) {
    for (int j = 0; j < s.n; ++j) {
      int arg = s.arg(m, j);
      const Operand &o = s.args[arg];
      GenLayout L;
      std::memset(&L, 0, sizeof L);
      L.op = o.op;
      L.alpha = o.alpha;
      L.beta = o.beta;
      auto put = [&](int64_t *so, int64_t *sc, int d, int64_t st) {
        int c = s.ins[j][d];
        for (int q = 0; q < g.n_out; ++q)
          if (s.out[q] == c) so[q] += st;
        for (int q = 0; q < g.n_con; ++q)
          if (con[q] == c) sc[q] += st;
      };
      if (o.kind == BES_TET_JACOBIAN) {
        // M[e,x,r] = V[e, r+1, x] - V[e, 0, x]
        L.kind = GEN_TET;
        int64_t se = o.src_strides[0][0], sv = o.src_strides[0][1], sc = o.src_strides[0][2];
        L.off0 = o.src_offset[0] + sv;
        L.off1 = o.src_offset[0];
        put(L.so0, L.sc0, 0, se);
        put(L.so0, L.sc0, 1, sc);
        put(L.so0, L.sc0, 2, sv);
        put(L.so1, L.sc1, 0, se);
        put(L.so1, L.sc1, 1, sc);
      } else if (o.kind == BES_EXPR) {
        // body `op` of the plan's list at (S0, S1); a one-source body reads
        // S0 for s1 as well (an in-bounds value the body ignores)
        L.kind = GEN_EXPR;
        L.op = (int32_t)(std::find(p.exprs.begin(), p.exprs.end(), o.expr) - p.exprs.begin());
        const int s1 = o.nsrc > 1 ? 1 : 0;
        L.off0 = o.src_offset[0];
        L.off1 = o.src_offset[s1];
        for (int d = 0; d < o.ndim; ++d) {
          put(L.so0, L.sc0, d, o.src_strides[0][d]);
          put(L.so1, L.sc1, d, o.src_strides[s1][d]);
        }
      } else {
        L.kind = o.kind != BES_ELEMENTWISE ? GEN_ARRAY
                 : (o.nsrc > 1 ? GEN_ELEMENTWISE2 : GEN_ELEMENTWISE);
        L.off0 = o.src_offset[0];
        for (int d = 0; d < o.ndim; ++d) put(L.so0, L.sc0, d, o.src_strides[0][d]);
        if (o.nsrc > 1) {
          L.off1 = o.src_offset[1];
          for (int d = 0; d < o.ndim; ++d) put(L.so1, L.sc1, d, o.src_strides[1][d]);
        }
      }
      int id = -1;
      for (int q = 0; q < g.n_layouts; ++q)
        if (!std::memcmp(&g.lay[q], &L, sizeof L)) {
          id = q;
          break;
        }
      if (id < 0) {
        id = g.n_layouts++;
        g.lay[id] = L;
      }
      g.layout[m][j] = id;
    }
  }
  g.n_slots = p.n_slots;
  int q = 0;
  for (int sl = 0; sl < p.n_slots; ++sl) {
    g.slot_m0[sl] = q;
    for (int m = 0; m < s.b; ++m)
      if (p.slot_of_member[m] == sl) g.slot_members[q++] = m;
    g.slot_m1[sl] = q;
  }
  for (int m = 0; m < s.b; ++m) g.slot_of[m] = p.slot_of_member[m];
  return BES_OK;
}

int bind_generic_ptrs(const Plan &p, const void *const *src, void *const *out, GenPtrs &ptrs) {
  std::memset(&ptrs, 0, sizeof ptrs);
  const Spec &s = p.spec;
  for (int m = 0; m < s.b; ++m)
    for (int j = 0; j < s.n; ++j) {
      int arg = s.arg(m, j);
      ptrs.src[m][j][0] = src[p.src_base[arg]];
      ptrs.src[m][j][1] = s.args[arg].nsrc > 1 ? src[p.src_base[arg] + 1] : src[p.src_base[arg]];
    }
  for (int sl = 0; sl < p.n_slots; ++sl) ptrs.out[sl] = out[sl];
  return BES_OK;
}

int bind_mfma(const Plan &p, const void *const *src, void *const *out, MfmaArgs &a,
              std::string &err) {
  if (!p.mfma_ok) {
    err = "plan is not MFMA compatible: " + p.mfma_why;
    return BES_E_UNSUPPORTED;
  }
  const MfmaRoles &R = p.mf;
  const CanonEinsum &e = p.canon.form;
  std::memset(&a, 0, sizeof a);
  a.M = R.M;
  a.N = R.N;
  a.K = R.K;
  a.n_members = e.b;
  a.n_slots = p.n_slots;
  // members ordered by slot so that each slot is a contiguous range
  std::vector<int> order;
  for (int sl = 0; sl < p.n_slots; ++sl)
    for (int k = 0; k < e.b; ++k)
      if (p.slot_of_member[p.canon.member_map[k]] == sl) order.push_back(k);
  int m = 0;
  for (int sl = 0; sl < p.n_slots; ++sl) {
    MfmaSlot &S = a.slot[sl];
    S.C = (float *)out[sl] + (p.out_layout[sl].custom ? p.out_layout[sl].offset : 0);
    S.acc = p.out_layout[sl].accumulate ? 1 : 0;
    int64_t cm, cn;
    const std::vector<int64_t> ost = out_strides(p, sl);
    if (!merge_out_strided(e.out, ost, R.Mi, e.extent, cm) ||
        !merge_out_strided(e.out, ost, R.Ni, e.extent, cn)) {
      err = "output layout does not merge the M and N index groups";
      return BES_E_UNSUPPORTED;
    }
    S.scm = cm;
    S.scn = cn;
    S.m0 = m;
    for (int k : order) {
      if (p.slot_of_member[p.canon.member_map[k]] != sl) continue;
      MfmaMember &M = a.mem[m++];
      int aa = slot_arg(p, k, R.posA), bb = slot_arg(p, k, R.posB);
      M.A = (const float *)src[p.src_base[aa]] + p.spec.args[aa].src_offset[0];
      M.B = (const float *)src[p.src_base[bb]] + p.spec.args[bb].src_offset[0];
      merge_group(p, aa, R.posA, R.Mi, e.extent, M.sam);
      merge_group(p, aa, R.posA, R.Ki, e.extent, M.sak);
      merge_group(p, bb, R.posB, R.Ki, e.extent, M.sbk);
      merge_group(p, bb, R.posB, R.Ni, e.extent, M.sbn);
    }
    S.m1 = m;
  }
  return BES_OK;
}

// ---------------------------------------------------------------------------
// Adjoint
// ---------------------------------------------------------------------------

int build_adjoint(const Plan &fwd, int pos, Plan &adj, int &n_out, std::string &err) {
  const Spec &f = fwd.spec;
  if (pos < 0 || pos >= f.n) {
    err = "position out of range";
    return BES_E_INVALID;
  }
  const auto &W = f.ins[pos];
  if (has_repeat(W)) {
    err = "adjoint of a position with a repeated index is not supported";
    return BES_E_UNSUPPORTED;
  }
  for (int c : W) {
    bool found = contains(f.out, c);
    for (int m = 0; m < f.n && !found; ++m)
      if (m != pos && contains(f.ins[m], c)) found = true;
    if (!found) {
      err = "adjoint would broadcast over an index used only by this position";
      return BES_E_UNSUPPORTED;
    }
  }
  // Output slots: distinct arguments at `pos`, in order of first occurrence.
  std::vector<int> slot_args;
  std::vector<int> slot_of(f.b);
  for (int i = 0; i < f.b; ++i) {
    int a = f.arg(i, pos);
    auto it = std::find(slot_args.begin(), slot_args.end(), a);
    if (it == slot_args.end()) {
      slot_of[i] = (int)slot_args.size();
      slot_args.push_back(a);
    } else {
      slot_of[i] = (int)(it - slot_args.begin());
    }
  }
  n_out = (int)slot_args.size();
  // Arguments of the adjoint: G_0..G_{b-1}, then the forward arguments used at
  // positions != pos, in forward order.
  std::vector<int> keep(f.args.size(), -1);
  std::vector<bes_operand> args;
  std::vector<int> src_from;
  for (int i = 0; i < f.b; ++i) {
    bes_operand g;
    std::memset(&g, 0, sizeof g);
    g.kind = BES_ARRAY;
    g.dtype = f.dtype;
    g.ndim = (int)f.out.size();
    g.nsrc = 1;
    g.alpha = 1.0;
    for (int d = 0; d < g.ndim; ++d) g.shape[d] = f.extent[f.out[d]];
    args.push_back(g);
    src_from.push_back(i);
  }
  if (f.out.empty()) {
    err = "adjoint of a scalar-output einsum is not supported";
    return BES_E_UNSUPPORTED;
  }
  for (int i = 0; i < f.b; ++i)
    for (int m = 0; m < f.n; ++m)
      if (m != pos) keep[f.arg(i, m)] = 0;
  for (size_t a = 0; a < f.args.size(); ++a) {
    if (keep[a] < 0) continue;
    keep[a] = (int)args.size();
    const Operand &o = f.args[a];
    bes_operand d;
    std::memset(&d, 0, sizeof d);
    d.kind = o.kind;
    d.dtype = o.dtype;
    d.ndim = o.ndim;
    d.nsrc = o.nsrc;
    d.op = o.op;
    d.alpha = o.alpha;
    d.beta = o.beta;
    for (int k = 0; k < o.ndim; ++k) d.shape[k] = o.shape[k];
    for (int s = 0; s < o.nsrc; ++s) {
      d.src_offset[s] = o.src_offset[s];
      for (int k = 0; k < o.ndim; ++k) d.src_strides[s][k] = o.src_strides[s][k];
      src_from.push_back(f.b + fwd.src_base[a] + s);
    }
    args.push_back(d);
  }
  std::vector<const char *> exprs(args.size(), nullptr);
  for (size_t a = 0; a < f.args.size(); ++a)
    if (keep[a] >= 0 && f.args[a].kind == BES_EXPR) exprs[keep[a]] = f.args[a].expr.c_str();
  std::vector<int32_t> table;
  std::string nota;
  for (int c : f.out) nota += char('a' + c);
  for (int m = 0; m < f.n; ++m) {
    if (m == pos) continue;
    nota += ',';
    for (int c : f.ins[m]) nota += char('a' + c);
  }
  nota += "->";
  for (int c : W) nota += char('a' + c);
  for (int i = 0; i < f.b; ++i) {
    table.push_back(i);
    for (int m = 0; m < f.n; ++m)
      if (m != pos) table.push_back(keep[f.arg(i, m)]);
  }
  adj = Plan();
  int rc = make_spec(nota.c_str(), f.b, f.n, (int)args.size(), args.data(), table.data(),
                     adj.spec, err, exprs.data());
  if (rc) return rc;
  adj.adjoint = true;
  adj.slot_of_member = slot_of;
  adj.n_slots = n_out;
  adj.src_from = src_from;
  return build_plan(adj, err);
}

}  // namespace bes
