// Canonical labeling of colored digraphs and the canonical form of a batched
// einsum.
//
// The paper leaves GetCanonLabel open ("any graph canonization"; Algorithm
// "CanonicalizeBatchedEinsum").  This is the project's own
// individualization-refinement search:
//   * the root partition is the color partition, ordered by color 1..9;
//   * refinement splits every cell by the multiset of (neighbour cell,
//     direction) pairs of its vertices until stable (an equitable partition of
//     the digraph), ordering the pieces by that multiset;
//   * the target cell is the first smallest non-singleton cell;
//   * a leaf's certificate is the adjacency bitstring of the graph relabeled
//     by the leaf's discrete partition; the lexicographically smallest wins;
//   * two leaves with equal certificates give an automorphism, which prunes
//     children in one orbit of the path's pointwise stabilizer and abandons a
//     subtree equivalent to the first path's.
// Every choice depends only on the ordered partition, never on vertex ids, so
// the canonical graph is invariant under relabeling of the input.
#include "canon.h"

#include <algorithm>
#include <numeric>

namespace bes {

namespace {

using Cells = std::vector<std::vector<int>>;

class Searcher {
 public:
  explicit Searcher(const Digraph &g) : g_(g), N_(g.n), W_((g.n + 63) / 64) {}

  std::vector<int> run(CanonStats *stats) {
    Cells cells;
    for (int c = 1; c <= 9; ++c) {
      std::vector<int> cell;
      for (int v = 0; v < N_; ++v)
        if (g_.color[v] == c) cell.push_back(v);
      if (!cell.empty()) cells.push_back(cell);
    }
    // Colors outside 1..9 (not produced by the induced-graph builder) form
    // further cells in ascending color order.
    std::vector<int> extra;
    for (int v = 0; v < N_; ++v)
      if (g_.color[v] < 1 || g_.color[v] > 9) extra.push_back(g_.color[v]);
    std::sort(extra.begin(), extra.end());
    extra.erase(std::unique(extra.begin(), extra.end()), extra.end());
    for (int c : extra) {
      std::vector<int> cell;
      for (int v = 0; v < N_; ++v)
        if (g_.color[v] == c) cell.push_back(v);
      cells.push_back(cell);
    }
    refine(cells);
    std::vector<int> path;
    if (N_ > 0) search(cells, path);
    std::vector<int> label(N_);
    for (int k = 0; k < N_; ++k) label[best_lab_[k]] = k;
    if (stats) *stats = st_;
    return label;
  }

 private:
  const Digraph &g_;
  int N_, W_;
  bool have_first_ = false;
  std::vector<uint64_t> first_cert_, best_cert_;
  std::vector<int> first_lab_, best_lab_, first_path_;
  std::vector<std::vector<int>> autos_;
  CanonStats st_;
  std::vector<int> cell_of_;
  std::vector<std::vector<int>> sig_;

  void refine(Cells &cells) {
    cell_of_.assign(N_, 0);
    sig_.resize(N_);
    for (;;) {
      for (int c = 0; c < (int)cells.size(); ++c)
        for (int v : cells[c]) cell_of_[v] = c;
      bool split = false;
      Cells next;
      next.reserve(cells.size() + 4);
      for (const auto &C : cells) {
        if (C.size() == 1) {
          next.push_back(C);
          continue;
        }
        for (int v : C) {
          auto &s = sig_[v];
          s.clear();
          for (int u : g_.succ[v]) s.push_back(2 * cell_of_[u]);
          for (int u : g_.pred[v]) s.push_back(2 * cell_of_[u] + 1);
          std::sort(s.begin(), s.end());
        }
        std::vector<int> m = C;
        std::stable_sort(m.begin(), m.end(),
                         [&](int a, int b) { return sig_[a] < sig_[b]; });
        size_t start = 0;
        int pieces = 0;
        for (size_t k = 1; k <= m.size(); ++k) {
          if (k == m.size() || sig_[m[k]] != sig_[m[start]]) {
            next.emplace_back(m.begin() + start, m.begin() + k);
            start = k;
            ++pieces;
          }
        }
        split |= pieces > 1;
      }
      cells.swap(next);
      if (!split) break;
    }
  }

  static Cells individualize(const Cells &cells, int t, int v) {
    Cells r;
    r.reserve(cells.size() + 1);
    for (int c = 0; c < (int)cells.size(); ++c) {
      if (c != t) {
        r.push_back(cells[c]);
        continue;
      }
      r.push_back({v});
      std::vector<int> rest;
      rest.reserve(cells[c].size() - 1);
      for (int u : cells[c])
        if (u != v) rest.push_back(u);
      r.push_back(rest);
    }
    return r;
  }

  int find(std::vector<int> &p, int x) {
    while (p[x] != x) {
      p[x] = p[p[x]];
      x = p[x];
    }
    return x;
  }

  // Is v in the orbit of an explored sibling under the automorphisms found so
  // far that fix the current path pointwise?
  bool pruned(int v, const std::vector<int> &explored, const std::vector<int> &path) {
    if (explored.empty() || autos_.empty()) return false;
    std::vector<int> p(N_);
    std::iota(p.begin(), p.end(), 0);
    bool any = false;
    for (const auto &gam : autos_) {
      bool fixes = true;
      for (int x : path)
        if (gam[x] != x) {
          fixes = false;
          break;
        }
      if (!fixes) continue;
      any = true;
      for (int x = 0; x < N_; ++x) {
        int a = find(p, x), b = find(p, gam[x]);
        if (a != b) p[std::max(a, b)] = std::min(a, b);
      }
    }
    if (!any) return false;
    int rv = find(p, v);
    for (int w : explored)
      if (find(p, w) == rv) return true;
    return false;
  }

  int search(const Cells &cells, std::vector<int> &path) {
    ++st_.nodes;
    int t = -1;
    size_t best = (size_t)-1;
    for (int c = 0; c < (int)cells.size(); ++c) {
      if (cells[c].size() > 1 && cells[c].size() < best) {
        best = cells[c].size();
        t = c;
      }
    }
    if (t < 0) return leaf(cells, path);
    std::vector<int> C = cells[t];
    std::sort(C.begin(), C.end());
    const int depth = (int)path.size();
    std::vector<int> explored;
    for (int v : C) {
      if (pruned(v, explored, path)) continue;
      Cells child = individualize(cells, t, v);
      refine(child);
      path.push_back(v);
      int r = search(child, path);
      path.pop_back();
      explored.push_back(v);
      if (r >= 0 && r < depth) return r;  // abandon up to the divergence node
    }
    return -1;
  }

  int leaf(const Cells &cells, const std::vector<int> &path) {
    ++st_.leaves;
    std::vector<int> lab(N_), pos(N_);
    for (int k = 0; k < N_; ++k) {
      lab[k] = cells[k][0];
      pos[lab[k]] = k;
    }
    std::vector<uint64_t> cert((size_t)N_ * W_, 0);
    for (int k = 0; k < N_; ++k)
      for (int u : g_.succ[lab[k]]) {
        int p = pos[u];
        cert[(size_t)k * W_ + p / 64] |= 1ull << (p % 64);
      }
    if (!have_first_) {
      have_first_ = true;
      first_cert_ = best_cert_ = cert;
      first_lab_ = best_lab_ = lab;
      first_path_ = path;
      return -1;
    }
    if (cert == first_cert_) {
      add_auto(first_lab_, lab);
      int d = 0;
      while (d < (int)path.size() && d < (int)first_path_.size() && path[d] == first_path_[d]) ++d;
      return d;
    }
    if (cert == best_cert_) {
      add_auto(best_lab_, lab);
      return -1;
    }
    if (cert < best_cert_) {
      best_cert_.swap(cert);
      best_lab_ = lab;
    }
    return -1;
  }

  void add_auto(const std::vector<int> &from, const std::vector<int> &to) {
    std::vector<int> gam(N_);
    for (int k = 0; k < N_; ++k) gam[from[k]] = to[k];
    ++st_.automorphisms;
    autos_.push_back(std::move(gam));
  }
};

}  // namespace

std::vector<int> canonical_labeling(const Digraph &g, CanonStats *stats) {
  Searcher s(g);
  return s.run(stats);
}

Digraph relabel(const Digraph &g, const std::vector<int> &label) {
  Digraph r;
  r.resize(g.n);
  for (int v = 0; v < g.n; ++v) {
    r.color[label[v]] = g.color[v];
    r.length_of[label[v]] = g.length_of[v];
    r.dtype_of[label[v]] = g.dtype_of[v];
    for (int u : g.succ[v]) r.add_edge(label[v], label[u]);
  }
  r.finalize();
  return r;
}

// ---------------------------------------------------------------------------
// ToBatchedEinsum (Appendix B.2).  Readings of the garbled steps: Step 2 orders
// V_arg-pos nodes; Steps 7 and 10 take the index predecessor of an input
// access node and the length predecessor of InputIndex(d, j).
// ---------------------------------------------------------------------------

namespace {
int pick(const Digraph &g, const std::vector<int> &xs, int color) {
  for (int x : xs)
    if (g.color[x] == color) return x;
  return -1;
}
}  // namespace

int to_batched_einsum(const Digraph &g, CanonEinsum &e, Inferred &inf, std::string &err) {
  std::vector<int> V[10];
  for (int v = 0; v < g.n; ++v) {
    if (g.color[v] < 1 || g.color[v] > 9) {
      err = "node color outside 1..9";
      return BES_E_INVALID;
    }
    V[g.color[v]].push_back(v);  // ascending label order
  }
  inf.output_nodes = V[kOutput];
  inf.argpos_nodes = V[kArgPos];
  inf.index_nodes = V[kIndex];
  inf.arg_nodes = V[kArg];
  std::vector<int> ord(g.n, -1);
  for (int c : {kOutput, kArgPos, kIndex, kArg})
    for (int k = 0; k < (int)V[c].size(); ++k) ord[V[c][k]] = k;
  auto dim_pos = [&](int d) { return (int)std::count_if(g.pred[d].begin(), g.pred[d].end(),
                                                          [&](int p) { return g.color[p] == kDim; }); };
  e = CanonEinsum();
  e.b = (int)V[kOutput].size();
  e.n = (int)V[kArgPos].size();
  // Step 7: output index list.
  e.out.assign(V[kAccessOut].size(), -1);
  for (int a : V[kAccessOut]) {
    int d = pick(g, g.pred[a], kDim), i = pick(g, g.pred[a], kIndex);
    int k = dim_pos(d);
    if (k < 0 || k >= (int)e.out.size() || e.out[k] >= 0) {
      err = "output accesses do not cover consecutive dims";
      return BES_E_INVALID;
    }
    e.out[k] = ord[i];
  }
  // Steps 8-9: ArgDim(j) and InputIndex(d, j).
  e.ins.assign(e.n, {});
  for (int j = 0; j < e.n; ++j) {
    int pj = V[kArgPos][j];
    std::vector<int> idx_at_dim;
    for (int a : g.succ[pj]) {
      int d = dim_pos(pick(g, g.pred[a], kDim));
      int i = ord[pick(g, g.pred[a], kIndex)];
      if (d >= (int)idx_at_dim.size()) idx_at_dim.resize(d + 1, -1);
      if (idx_at_dim[d] >= 0 && idx_at_dim[d] != i) {
        err = "inconsistent input indexing across members";
        return BES_E_INVALID;
      }
      idx_at_dim[d] = i;
    }
    for (int x : idx_at_dim)
      if (x < 0) {
        err = "argument dims are not consecutive";
        return BES_E_INVALID;
      }
    e.ins[j] = idx_at_dim;
  }
  // Step 10: ArgLabel(i, j), DtypeLabel and LengthLabel.
  e.table.assign((size_t)e.b * e.n, -1);
  for (int i = 0; i < e.b; ++i) {
    int oi = V[kOutput][i];
    for (int a : g.succ[oi]) {
      int pj = pick(g, g.pred[a], kArgPos);
      int arg = pick(g, g.succ[a], kArg);
      int j = ord[pj];
      int &slot = e.table[(size_t)i * e.n + j];
      if (slot >= 0 && slot != ord[arg]) {
        err = "more than one argument in one slot";
        return BES_E_INVALID;
      }
      slot = ord[arg];
    }
  }
  for (int x : e.table)
    if (x < 0) {
      err = "empty argument slot";
      return BES_E_INVALID;
    }
  e.extent.assign(V[kIndex].size(), -1);
  for (int k = 0; k < (int)V[kIndex].size(); ++k) {
    int L = pick(g, g.pred[V[kIndex][k]], kLength);
    e.extent[k] = L >= 0 ? g.length_of[L] : -1;
  }
  e.dtype.assign(V[kArg].size(), 0);
  for (int k = 0; k < (int)V[kArg].size(); ++k) {
    int t = pick(g, g.pred[V[kArg][k]], kDtype);
    e.dtype[k] = t >= 0 ? g.dtype_of[t] : 0;
  }
  return BES_OK;
}

int canonicalize(const Spec &spec, Canonical &c, std::string &err) {
  c = Canonical();
  c.induced = to_induced_graph(spec);
  int bad = check_compliance(c.induced.g);
  if (bad) {
    err = "induced graph violates compliance condition C" + std::to_string(bad);
    return BES_E_INVALID;
  }
  c.label = canonical_labeling(c.induced.g, &c.stats);
  c.canon_graph = relabel(c.induced.g, c.label);
  Inferred inf;
  int rc = to_batched_einsum(c.canon_graph, c.form, inf, err);
  if (rc) return rc;
  // Substitution maps (Algorithm "CanonicalizeBatchedEinsum", last loop):
  // canonical node -> induced node -> the caller's symbol.
  std::vector<int> inv(c.label.size());
  for (int v = 0; v < (int)c.label.size(); ++v) inv[c.label[v]] = v;
  const InducedGraph &G = c.induced;
  for (int node : inf.output_nodes) c.member_map.push_back(inv[node] - G.outp0);
  for (int node : inf.argpos_nodes) c.pos_map.push_back(inv[node] - G.pos0);
  for (int node : inf.arg_nodes) c.arg_map.push_back(inv[node] - G.arg0);
  for (int node : inf.index_nodes) c.index_map.push_back(G.index_symbol[inv[node] - G.idx0]);
  return BES_OK;
}

std::string key_string(const CanonEinsum &e) {
  std::string s = "b=" + std::to_string(e.b) + ";n=" + std::to_string(e.n) + ";";
  for (int j = 0; j < e.n; ++j) {
    if (j) s += ',';
    for (int c : e.ins[j]) s += char('a' + c);
  }
  s += "->";
  for (int c : e.out) s += char('a' + c);
  s += ";";
  for (int i = 0; i < e.b; ++i) {
    if (i) s += '/';
    for (int j = 0; j < e.n; ++j) {
      if (j) s += ',';
      s += std::to_string(e.arg(i, j));
    }
  }
  s += ";ext=";
  for (size_t k = 0; k < e.extent.size(); ++k) {
    if (k) s += ',';
    s += std::to_string(e.extent[k]);
  }
  s += ";dt=";
  for (size_t k = 0; k < e.dtype.size(); ++k) {
    if (k) s += ',';
    s += dtype_name(e.dtype[k]);
  }
  return s;
}

std::string tuple_string(const CanonEinsum &e) {
  std::string s = "(" + std::to_string(e.b) + ", " + std::to_string(e.n) + ", (";
  for (size_t d = 0; d < e.out.size(); ++d) {
    if (d) s += ' ';
    s += char('a' + e.out[d]);
  }
  s += "), (";
  for (int j = 0; j < e.n; ++j) {
    if (j) s += ", ";
    s += '(';
    for (size_t d = 0; d < e.ins[j].size(); ++d) {
      if (d) s += ' ';
      s += char('a' + e.ins[j][d]);
    }
    s += ')';
  }
  s += "), (";
  for (int i = 0; i < e.b; ++i) {
    if (i) s += ", ";
    s += '(';
    for (int j = 0; j < e.n; ++j) {
      if (j) s += ", ";
      s += "A_" + std::to_string(e.arg(i, j));
    }
    s += ')';
  }
  s += "))";
  return s;
}

}  // namespace bes
