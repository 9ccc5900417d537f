// Host-side representation of a (functional) batched einsum.
//
// Definitions "Batched Einstein Summation" and "Functional Batched Einstein
// Summation" (arxiv 2601.12220): a quintuple (b, n, I_out, (I_in^j), (A^{i,j}))
// whose arguments are functions of their index tuples.  Indices are the
// letters a..z, stored as integers 0..25.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../../include/bes.h"

namespace bes {

constexpr int kLetters = 26;

struct Operand {
  int32_t kind = BES_ARRAY;
  int32_t dtype = BES_FLOAT64;
  int32_t ndim = 0;
  int32_t nsrc = 1;
  int64_t shape[BES_MAX_DIM] = {0};
  int64_t src_offset[BES_MAX_SRC] = {0};
  // Element strides per source and axis (filled in for dense sources).
  int64_t src_strides[BES_MAX_SRC][BES_MAX_DIM] = {{0}};
  int32_t op = BES_OP_ID;
  double alpha = 1.0;
  double beta = 0.0;
  std::string expr;   // body of a BES_EXPR operand over s0, s1
};

struct Spec {
  int b = 0;
  int n = 0;
  std::vector<int> out;               // I_out
  std::vector<std::vector<int>> ins;  // I_in^j, j = 0..n-1
  std::vector<Operand> args;          // user arguments
  std::vector<int> table;             // b*n argument ids, row-major
  int64_t extent[kLetters];           // extent of every used index, else -1
  int dtype = BES_FLOAT64;            // common dtype of the arguments, 0 if mixed

  int arg(int i, int j) const { return table[i * n + j]; }
  std::vector<int> used_indices() const;  // ascending letters used by inputs
};

// Parse "in_1,...,in_n->out".  Returns 0 or BES_E_INVALID with `err` set.
int parse_notation(const char *notation, std::vector<std::vector<int>> &ins,
                   std::vector<int> &out, std::string &err);

// Build and validate a spec from ABI inputs: soundness conditions after
// Eq. (1), one extent per index across the batch, every argument used,
// distinct output indices (C27), common dtype.  Fills dense source strides.
// exprs (may be NULL) holds the body of every BES_EXPR argument.
int make_spec(const char *notation, int b, int n, int n_args,
              const bes_operand *args, const int32_t *table, Spec &spec,
              std::string &err, const char *const *exprs = nullptr);

// Is `body` an expression the run-time build accepts: s0, s1, decimal
// constants, + - * / ( ) , and the functions listed in bes.h?
bool valid_expression(const std::string &body, std::string &err);

const char *dtype_name(int dtype);  // "f64", "f32", ...

}  // namespace bes
