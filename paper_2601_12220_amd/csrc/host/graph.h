// Colored induced digraph of a batched einsum (Appendix B, "Induced Graph").
#pragma once

#include <cstdint>
#include <vector>

#include "spec.h"

namespace bes {

// Node colors of the coloring equation (Appendix B.1), in this order.
enum NodeColor {
  kArg = 1, kIndex = 2, kAccessIn = 3, kAccessOut = 4, kOutput = 5,
  kArgPos = 6, kDtype = 7, kLength = 8, kDim = 9
};

struct Digraph {
  int n = 0;
  std::vector<int> color;                 // 1..9
  std::vector<std::vector<int>> succ;     // sorted out-neighbours
  std::vector<std::vector<int>> pred;     // sorted in-neighbours
  std::vector<int64_t> length_of;         // iota_length (length nodes), else -1
  std::vector<int> dtype_of;              // iota_dtype (dtype nodes), else 0

  void resize(int nn);
  void add_edge(int u, int v);            // idempotent
  void finalize();                        // sort and dedupe adjacency
  bool has_edge(int u, int v) const;
  std::vector<uint8_t> dense() const;     // row-major 0/1 adjacency
  static Digraph from_dense(int n, const uint8_t *adj, const int32_t *colors);
};

struct InducedGraph {
  Digraph g;
  // First node of each kind, in the construction order of Appendix B.1:
  // args, indices, input accesses, output accesses, outputs, arg positions,
  // dtypes, lengths, dims.
  int arg0 = 0, idx0 = 0, ain0 = 0, aout0 = 0, outp0 = 0, pos0 = 0, dt0 = 0,
      len0 = 0, dim0 = 0;
  int n_arg = 0, n_index = 0, n_ain = 0, n_aout = 0, n_dtype = 0, n_length = 0,
      n_dim = 0;
  std::vector<int> index_symbol;  // index node k -> letter
};

// ToInducedGraph (Appendix B.1).
InducedGraph to_induced_graph(const Spec &spec);

// Compliance conditions C1..C30 (Appendix B.2).  0 if compliant, else the
// number of the first violated condition.
int check_compliance(const Digraph &g);

}  // namespace bes
