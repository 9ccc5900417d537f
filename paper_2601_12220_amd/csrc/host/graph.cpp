// ToInducedGraph (Appendix B.1) and the compliance conditions (Appendix B.2).
#include "graph.h"

#include <algorithm>
#include <map>
#include <set>

namespace bes {

void Digraph::resize(int nn) {
  n = nn;
  color.assign(n, 0);
  succ.assign(n, {});
  pred.assign(n, {});
  length_of.assign(n, -1);
  dtype_of.assign(n, 0);
}

void Digraph::add_edge(int u, int v) {
  succ[u].push_back(v);
  pred[v].push_back(u);
}

void Digraph::finalize() {
  for (int v = 0; v < n; ++v) {
    std::sort(succ[v].begin(), succ[v].end());
    succ[v].erase(std::unique(succ[v].begin(), succ[v].end()), succ[v].end());
    std::sort(pred[v].begin(), pred[v].end());
    pred[v].erase(std::unique(pred[v].begin(), pred[v].end()), pred[v].end());
  }
}

bool Digraph::has_edge(int u, int v) const {
  return std::binary_search(succ[u].begin(), succ[u].end(), v);
}

std::vector<uint8_t> Digraph::dense() const {
  std::vector<uint8_t> a((size_t)n * n, 0);
  for (int u = 0; u < n; ++u)
    for (int v : succ[u]) a[(size_t)u * n + v] = 1;
  return a;
}

Digraph Digraph::from_dense(int n, const uint8_t *adj, const int32_t *colors) {
  Digraph g;
  g.resize(n);
  for (int u = 0; u < n; ++u) {
    g.color[u] = colors[u];
    for (int v = 0; v < n; ++v)
      if (adj[(size_t)u * n + v]) g.add_edge(u, v);
  }
  g.finalize();
  return g;
}

InducedGraph to_induced_graph(const Spec &s) {
  InducedGraph G;
  const int b = s.b, n = s.n;
  // N_arg, N_index, N_length (a set of distinct axis lengths), N_dim (max of
  // AllDims), N_dtype, N_access,in, N_access,out.
  G.n_arg = (int)s.args.size();
  std::vector<int> idx = s.used_indices();
  G.n_index = (int)idx.size();
  std::set<int64_t> lengths;
  for (int c : idx) lengths.insert(s.extent[c]);
  G.n_length = (int)lengths.size();
  int ndim = (int)s.out.size();
  for (const auto &a : s.args) ndim = std::max(ndim, (int)a.ndim);
  G.n_dim = ndim;
  std::set<int> dtypes;
  for (const auto &a : s.args) dtypes.insert(a.dtype);
  G.n_dtype = (int)dtypes.size();
  int per_member = 0;
  for (const auto &l : s.ins) per_member += (int)l.size();
  G.n_ain = b * per_member;
  G.n_aout = (int)s.out.size();

  G.arg0 = 0;
  G.idx0 = G.arg0 + G.n_arg;
  G.ain0 = G.idx0 + G.n_index;
  G.aout0 = G.ain0 + G.n_ain;
  G.outp0 = G.aout0 + G.n_aout;
  G.pos0 = G.outp0 + b;
  G.dt0 = G.pos0 + n;
  G.len0 = G.dt0 + G.n_dtype;
  G.dim0 = G.len0 + G.n_length;
  const int N = G.dim0 + G.n_dim;  // Eq. for N^IDG
  Digraph &g = G.g;
  g.resize(N);

  int node_of_index[kLetters];
  for (int c = 0; c < kLetters; ++c) node_of_index[c] = -1;
  G.index_symbol = idx;
  for (int k = 0; k < G.n_index; ++k) node_of_index[idx[k]] = G.idx0 + k;
  std::map<int64_t, int> node_of_length;
  {
    int k = 0;
    for (int64_t L : lengths) {  // ascending
      node_of_length[L] = G.len0 + k;
      g.length_of[G.len0 + k] = L;
      ++k;
    }
  }
  std::map<int, int> node_of_dtype;
  {
    int k = 0;
    for (int d : dtypes) {  // ascending DtypeRank
      node_of_dtype[d] = G.dt0 + k;
      g.dtype_of[G.dt0 + k] = d;
      ++k;
    }
  }
  auto dim_node = [&](int d) { return G.dim0 + d; };  // d is 0-based position

  // Colors.
  for (int v = 0; v < N; ++v) {
    int c;
    if (v < G.idx0) c = kArg;
    else if (v < G.ain0) c = kIndex;
    else if (v < G.aout0) c = kAccessIn;
    else if (v < G.outp0) c = kAccessOut;
    else if (v < G.pos0) c = kOutput;
    else if (v < G.dt0) c = kArgPos;
    else if (v < G.len0) c = kDtype;
    else if (v < G.dim0) c = kLength;
    else c = kDim;
    g.color[v] = c;
  }

  // Input accesses (i, j, I_in^j_d, d) and their edges:
  // E_access,in-to-arg, E_arg-pos-to-access,in, E_output-to-access,in,
  // E_index-to-access,in, E_dim-to-access,in.
  int acc = G.ain0;
  for (int i = 0; i < b; ++i) {
    for (int j = 0; j < n; ++j) {
      int a = s.arg(i, j);
      for (int d = 0; d < (int)s.ins[j].size(); ++d) {
        g.add_edge(acc, G.arg0 + a);
        g.add_edge(G.pos0 + j, acc);
        g.add_edge(G.outp0 + i, acc);
        g.add_edge(node_of_index[s.ins[j][d]], acc);
        g.add_edge(dim_node(d), acc);
        ++acc;
      }
    }
  }
  // Output accesses: E_index-to-access,out and E_dim-to-access,out.
  for (int d = 0; d < (int)s.out.size(); ++d) {
    g.add_edge(node_of_index[s.out[d]], G.aout0 + d);
    g.add_edge(dim_node(d), G.aout0 + d);
  }
  // E_length: length -> index.
  for (int c : idx) g.add_edge(node_of_length[s.extent[c]], node_of_index[c]);
  // E_dtype: dtype -> arg.
  for (int a = 0; a < G.n_arg; ++a) g.add_edge(node_of_dtype[s.args[a].dtype], G.arg0 + a);
  // Rank tournaments: smaller -> larger.
  for (int p = 0; p < G.n_length; ++p)
    for (int q = p + 1; q < G.n_length; ++q) g.add_edge(G.len0 + p, G.len0 + q);
  for (int p = 0; p < G.n_dtype; ++p)
    for (int q = p + 1; q < G.n_dtype; ++q) g.add_edge(G.dt0 + p, G.dt0 + q);
  for (int p = 0; p < G.n_dim; ++p)
    for (int q = p + 1; q < G.n_dim; ++q) g.add_edge(dim_node(p), dim_node(q));
  g.finalize();
  return G;
}

// ---------------------------------------------------------------------------
// Compliance (Appendix B.2).  Readings of the garbled conditions: C12's third
// line is read with V_access,out; C30 applies only when the output has at
// least one index (a scalar output has no output accesses).
// ---------------------------------------------------------------------------

namespace {

struct Sets {
  std::vector<int> of[10];
};

bool all_in(const std::vector<int> &xs, const Digraph &g, std::initializer_list<int> cols) {
  for (int x : xs) {
    bool ok = false;
    for (int c : cols) ok |= g.color[x] == c;
    if (!ok) return false;
  }
  return true;
}

int count_col(const std::vector<int> &xs, const Digraph &g, int c) {
  int k = 0;
  for (int x : xs) k += g.color[x] == c;
  return k;
}

int first_col(const std::vector<int> &xs, const Digraph &g, int c) {
  for (int x : xs)
    if (g.color[x] == c) return x;
  return -1;
}

bool transitive_tournament(const Digraph &g, const std::vector<int> &vs) {
  // Orderable so that v_j in Succs(v_i) iff i < j: in-degrees within the set
  // are exactly 0, 1, ..., m-1 and the induced edges respect that order.
  int m = (int)vs.size();
  std::vector<std::pair<int, int>> deg;
  for (int v : vs) {
    int k = 0;
    for (int u : g.pred[v])
      if (std::find(vs.begin(), vs.end(), u) != vs.end()) ++k;
    deg.push_back({k, v});
  }
  std::sort(deg.begin(), deg.end());
  for (int i = 0; i < m; ++i)
    if (deg[i].first != i) return false;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      bool e = g.has_edge(deg[i].second, deg[j].second);
      if (e != (i < j)) return false;
    }
  return true;
}

}  // namespace

int check_compliance(const Digraph &g) {
  Sets S;
  for (int v = 0; v < g.n; ++v) {
    if (g.color[v] < 1 || g.color[v] > 9) return 1;  // C1
    S.of[g.color[v]].push_back(v);
  }
  for (int v : S.of[kArg]) {
    if (!g.succ[v].empty()) return 2;                                   // C2
    if (!all_in(g.pred[v], g, {kAccessIn, kDtype})) return 3;          // C3
    if (count_col(g.pred[v], g, kDtype) != 1) return 4;                 // C4
  }
  for (int v : S.of[kDtype]) {
    if (!all_in(g.pred[v], g, {kDtype})) return 5;                     // C5
    if (!all_in(g.succ[v], g, {kArg, kDtype})) return 6;               // C6
  }
  for (int v : S.of[kAccessIn]) {
    if (!all_in(g.succ[v], g, {kArg})) return 7;                       // C7
    if (g.pred[v].size() != 4 || count_col(g.pred[v], g, kArgPos) != 1 ||
        count_col(g.pred[v], g, kIndex) != 1 || count_col(g.pred[v], g, kOutput) != 1 ||
        count_col(g.pred[v], g, kDim) != 1)
      return 8;                                                          // C8
  }
  for (int v : S.of[kOutput]) {
    if (!all_in(g.succ[v], g, {kAccessIn})) return 9;                  // C9
    if (!g.pred[v].empty()) return 10;                                  // C10
  }
  for (int v : S.of[kAccessOut]) {
    if (!g.succ[v].empty()) return 11;                                  // C11
    if (g.pred[v].size() != 2 || count_col(g.pred[v], g, kIndex) != 1 ||
        count_col(g.pred[v], g, kDim) != 1)
      return 12;                                                         // C12
  }
  for (int v : S.of[kIndex]) {
    if (!all_in(g.succ[v], g, {kAccessIn, kAccessOut})) return 13;     // C13
    if (g.pred[v].size() != 1 || count_col(g.pred[v], g, kLength) != 1) return 14;  // C14
  }
  for (int v : S.of[kLength]) {
    if (!all_in(g.pred[v], g, {kLength})) return 15;                   // C15
    if (!all_in(g.succ[v], g, {kIndex, kLength})) return 16;           // C16
  }
  for (int v : S.of[kDim]) {
    if (!all_in(g.pred[v], g, {kDim})) return 17;                      // C17
    if (!all_in(g.succ[v], g, {kAccessIn, kAccessOut, kDim})) return 18;  // C18
  }
  for (int v : S.of[kArgPos]) {
    if (!g.pred[v].empty()) return 19;                                  // C19
    if (!all_in(g.succ[v], g, {kAccessIn})) return 20;                 // C20
  }
  if (!transitive_tournament(g, S.of[kDim])) return 21;                 // C21
  if (!transitive_tournament(g, S.of[kLength])) return 22;              // C22
  if (!transitive_tournament(g, S.of[kDtype])) return 23;               // C23
  // C24: accesses of the same argument along the same dim use indices of the
  // same length.
  {
    std::map<std::pair<int, int>, std::vector<int>> len_preds;
    for (int v : S.of[kAccessIn]) {
      int a = first_col(g.succ[v], g, kArg);
      int d = first_col(g.pred[v], g, kDim);
      int i = first_col(g.pred[v], g, kIndex);
      auto key = std::make_pair(a, d);
      auto it = len_preds.find(key);
      if (it == len_preds.end()) len_preds[key] = g.pred[i];
      else if (it->second != g.pred[i]) return 24;
    }
  }
  // C25: an output index also indexes some input access.
  for (int v : S.of[kAccessOut]) {
    int i = first_col(g.pred[v], g, kIndex);
    if (count_col(g.succ[i], g, kAccessIn) == 0) return 25;
  }
  // C26: every output has exactly one access with the same (index, dim,
  // arg-pos) as any input access.
  {
    std::map<std::tuple<int, int, int, int>, int> cnt;
    for (int v : S.of[kAccessIn]) {
      int i = first_col(g.pred[v], g, kIndex), d = first_col(g.pred[v], g, kDim),
          k = first_col(g.pred[v], g, kArgPos), o = first_col(g.pred[v], g, kOutput);
      cnt[std::make_tuple(i, d, k, o)]++;
    }
    for (int v : S.of[kAccessIn]) {
      int i = first_col(g.pred[v], g, kIndex), d = first_col(g.pred[v], g, kDim),
          k = first_col(g.pred[v], g, kArgPos);
      for (int o : S.of[kOutput]) {
        auto it = cnt.find(std::make_tuple(i, d, k, o));
        if (it == cnt.end() || it->second != 1) return 26;
      }
    }
  }
  // C27: output indices are distinct.
  {
    std::set<int> idx;
    for (int v : S.of[kAccessOut]) idx.insert(first_col(g.pred[v], g, kIndex));
    if (idx.size() != S.of[kAccessOut].size()) return 27;
  }
  // C28 / C29: per (arg-pos, output) a single argument, and its dims start
  // at the first dim node with every other dim having a predecessor among them.
  for (int k : S.of[kArgPos]) {
    for (int o : S.of[kOutput]) {
      std::set<int> args, dims;
      for (int v : g.succ[k]) {
        if (!g.has_edge(o, v)) continue;
        for (int a : g.succ[v]) args.insert(a);
        dims.insert(first_col(g.pred[v], g, kDim));
      }
      if (args.size() != 1) return 28;
      int roots = 0, inner = 0;
      for (int d : dims) {
        if (count_col(g.pred[d], g, kDim) == 0) ++roots;
        bool has = false;
        for (int p : g.pred[d]) has |= dims.count(p) > 0;
        inner += has;
      }
      if (roots != 1 || inner != (int)dims.size() - 1) return 29;
    }
  }
  if (!S.of[kAccessOut].empty()) {
    std::set<int> dims;
    for (int v : S.of[kAccessOut]) dims.insert(first_col(g.pred[v], g, kDim));
    int roots = 0, inner = 0;
    for (int d : dims) {
      if (count_col(g.pred[d], g, kDim) == 0) ++roots;
      bool has = false;
      for (int p : g.pred[d]) has |= dims.count(p) > 0;
      inner += has;
    }
    if (roots != 1 || inner != (int)dims.size() - 1) return 30;          // C30
  }
  return 0;
}

}  // namespace bes
