// Canonical form of a batched einsum (Section "A Canonical form for Batched
// Einsums", Algorithm "CanonicalizeBatchedEinsum", Appendix B.2).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "graph.h"
#include "spec.h"

namespace bes {

// GetCanonLabel: canonical labeling of a vertex-colored digraph.  Returns
// label[v] = canonical position of v.  Deterministic and invariant: for any
// relabeling pi of g, relabel(g, label) == relabel(pi(g), label_pi).
struct CanonStats {
  int64_t leaves = 0;
  int64_t nodes = 0;
  int64_t automorphisms = 0;
};
std::vector<int> canonical_labeling(const Digraph &g, CanonStats *stats = nullptr);

// Apply a relabeling: result node label[v] <- node v (adjacency, colors, iota).
Digraph relabel(const Digraph &g, const std::vector<int> &label);

// A batched einsum written with canonical names: index k is the letter 'a'+k,
// argument k is A_k.
struct CanonEinsum {
  int b = 0, n = 0;
  std::vector<int> out;               // index ordinals
  std::vector<std::vector<int>> ins;  // per position, index ordinals
  std::vector<int> table;             // b*n argument ordinals
  std::vector<int64_t> extent;        // per index ordinal
  std::vector<int> dtype;             // per argument ordinal
  int arg(int i, int j) const { return table[i * n + j]; }
};

// ToBatchedEinsum (Appendix B.2, Steps 1-11) on a compliant graph: nodes of
// each kind are enumerated in label order.  Also returns, per kind, the node
// enumerations it chose (iota^inferred): the k-th output / arg-position /
// index / argument node.
struct Inferred {
  std::vector<int> output_nodes, argpos_nodes, index_nodes, arg_nodes;
};
int to_batched_einsum(const Digraph &g, CanonEinsum &e, Inferred &inf, std::string &err);

// Full canonicalization: returns C(e) and the substitution maps from
// canonical names to the caller's names (sigma^i, sigma^j, sigma^A, sigma^I).
struct Canonical {
  InducedGraph induced;
  std::vector<int> label;     // canonical position of every induced node
  Digraph canon_graph;        // relabeled induced graph
  CanonEinsum form;
  std::vector<int> member_map;  // canonical member -> user member
  std::vector<int> pos_map;     // canonical position -> user position
  std::vector<int> arg_map;     // canonical argument -> user argument
  std::vector<int> index_map;   // canonical index -> user letter
  CanonStats stats;
};
int canonicalize(const Spec &spec, Canonical &c, std::string &err);

// Serializations of C(e).
std::string key_string(const CanonEinsum &e);     // tuning-database identity
std::string tuple_string(const CanonEinsum &e);   // the paper's tuple notation

}  // namespace bes
