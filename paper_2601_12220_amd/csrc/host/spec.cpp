// Parsing and validation of batched einsums.
//
// Grammar: Listings "Grammar for an index" and "Grammar for an index list";
// soundness: the four conditions stated after Eq. (1); batched form:
// Definition "Batched Einstein Summation".
#include "spec.h"

#include <cctype>

#include <cstring>

namespace bes {

std::vector<int> Spec::used_indices() const {
  bool used[kLetters] = {false};
  for (const auto &l : ins)
    for (int c : l) used[c] = true;
  std::vector<int> r;
  for (int c = 0; c < kLetters; ++c)
    if (used[c]) r.push_back(c);
  return r;
}

const char *dtype_name(int dtype) {
  switch (dtype) {
    case BES_INT8: return "i8";
    case BES_INT32: return "i32";
    case BES_INT64: return "i64";
    case BES_FLOAT16: return "f16";
    case BES_FLOAT32: return "f32";
    case BES_FLOAT64: return "f64";
    case BES_COMPLEX64: return "c64";
    case BES_COMPLEX128: return "c128";
    default: return "?";
  }
}

int parse_notation(const char *notation, std::vector<std::vector<int>> &ins,
                   std::vector<int> &out, std::string &err) {
  ins.clear();
  out.clear();
  if (!notation) {
    err = "notation is NULL";
    return BES_E_INVALID;
  }
  const char *arrow = std::strstr(notation, "->");
  if (!arrow) {
    err = "notation lacks '->'";
    return BES_E_INVALID;
  }
  if (std::strstr(arrow + 2, "->")) {
    err = "notation has more than one '->'";
    return BES_E_INVALID;
  }
  std::vector<int> cur;
  for (const char *p = notation; p < arrow; ++p) {
    if (*p == ',') {
      ins.push_back(cur);
      cur.clear();
    } else if (*p >= 'a' && *p <= 'z') {
      cur.push_back(*p - 'a');
    } else {
      err = std::string("invalid character '") + *p + "' in notation";
      return BES_E_INVALID;
    }
  }
  ins.push_back(cur);
  for (const char *p = arrow + 2; *p; ++p) {
    if (*p >= 'a' && *p <= 'z') {
      out.push_back(*p - 'a');
    } else {
      err = std::string("invalid character '") + *p + "' in output";
      return BES_E_INVALID;
    }
  }
  return BES_OK;
}

static bool supported_kind(int k) {
  return k == BES_ARRAY || k == BES_VIEW || k == BES_ELEMENTWISE || k == BES_TET_JACOBIAN ||
         k == BES_EXPR;
}

bool valid_expression(const std::string &body, std::string &err) {
  // A recognizer for: expr := term (('+'|'-'|'*'|'/') term)*;
  // term := ('+'|'-')* (number | s0 | s1 | '(' expr ')' | func '(' args ')');
  // args := expr (',' expr)*.  Tracked as a token-class state machine.
  static const char *const kFuncs[] = {"sin", "cos", "tan", "exp", "log", "sqrt",
                                       "fabs", "tanh", "pow", "fmin", "fmax"};
  const size_t n = body.size();
  if (n == 0 || n > 512) {
    err = "expression body must have 1..512 characters";
    return false;
  }
  std::vector<bool> call;   // per open parenthesis: a function call (allows ',')
  bool want_operand = true;
  size_t i = 0;
  auto bad = [&](const std::string &why) {
    err = why + " at position " + std::to_string(i) + " of \"" + body + "\"";
    return false;
  };
  while (i < n) {
    const char ch = body[i];
    if (ch == ' ' || ch == '\t') {
      ++i;
      continue;
    }
    if (want_operand) {
      if (ch == '+' || ch == '-') {
        ++i;
      } else if (ch == '(') {
        call.push_back(false);
        ++i;
      } else if ((ch >= '0' && ch <= '9') || ch == '.') {
        size_t j = i, digits = 0;
        while (j < n && ((body[j] >= '0' && body[j] <= '9') || body[j] == '.')) {
          digits += body[j] != '.';
          ++j;
        }
        if (digits == 0) return bad("malformed number");
        if (j < n && (body[j] == 'e' || body[j] == 'E')) {
          ++j;
          if (j < n && (body[j] == '+' || body[j] == '-')) ++j;
          if (j >= n || body[j] < '0' || body[j] > '9') return bad("malformed number");
          while (j < n && body[j] >= '0' && body[j] <= '9') ++j;
        }
        i = j;
        want_operand = false;
      } else if (std::isalpha((unsigned char)ch) || ch == '_') {
        size_t j = i;
        while (j < n && (std::isalnum((unsigned char)body[j]) || body[j] == '_')) ++j;
        const std::string id = body.substr(i, j - i);
        if (id == "s0" || id == "s1") {
          i = j;
          want_operand = false;
        } else {
          bool f = false;
          for (const char *fn : kFuncs) f |= id == fn;
          size_t k = j;
          while (k < n && (body[k] == ' ' || body[k] == '\t')) ++k;
          if (!f || k >= n || body[k] != '(') return bad("unknown name '" + id + "'");
          call.push_back(true);
          i = k + 1;
        }
      } else {
        return bad(std::string("unexpected '") + ch + "'");
      }
    } else {
      if (ch == '+' || ch == '-' || ch == '*' || ch == '/') {
        want_operand = true;
        ++i;
      } else if (ch == ',') {
        if (call.empty() || !call.back()) return bad("',' outside a function call");
        want_operand = true;
        ++i;
      } else if (ch == ')') {
        if (call.empty()) return bad("unbalanced ')'");
        call.pop_back();
        ++i;
      } else {
        return bad(std::string("unexpected '") + ch + "'");
      }
    }
  }
  if (want_operand) return bad("expression ends without an operand");
  if (!call.empty()) return bad("unbalanced '('");
  return true;
}

int make_spec(const char *notation, int b, int n, int n_args,
              const bes_operand *args, const int32_t *table, Spec &spec,
              std::string &err, const char *const *exprs) {
  spec = Spec();
  if (b < 1 || b > BES_MAX_B) {
    err = "b out of range";
    return b < 1 ? BES_E_INVALID : BES_E_UNSUPPORTED;
  }
  if (n < 1 || n > BES_MAX_N) {
    err = "n out of range";
    return n < 1 ? BES_E_INVALID : BES_E_UNSUPPORTED;
  }
  if (n_args < 1 || !args || !table) {
    err = "missing arguments or table";
    return BES_E_INVALID;
  }
  int rc = parse_notation(notation, spec.ins, spec.out, err);
  if (rc) return rc;
  if ((int)spec.ins.size() != n) {
    err = "notation has " + std::to_string(spec.ins.size()) + " inputs, n = " + std::to_string(n);
    return BES_E_INVALID;
  }
  spec.b = b;
  spec.n = n;
  spec.table.assign(table, table + (size_t)b * n);
  spec.args.resize(n_args);
  for (int a = 0; a < n_args; ++a) {
    const bes_operand &o = args[a];
    Operand &d = spec.args[a];
    if (o.ndim < 0 || o.ndim > BES_MAX_DIM) {
      err = "operand rank out of range";
      return BES_E_UNSUPPORTED;
    }
    if (o.ndim == 0) {
      // A 0-dim argument has no access nodes in the induced graph, so its
      // member and position would be lost (Appendix B.1 edge sets).
      err = "0-dim operands are not supported";
      return BES_E_UNSUPPORTED;
    }
    if (!supported_kind(o.kind)) {
      err = "unknown operand kind";
      return BES_E_UNSUPPORTED;
    }
    if (o.dtype < BES_INT8 || o.dtype > BES_COMPLEX128) {
      err = "unknown dtype";
      return BES_E_INVALID;
    }
    int want_src = ((o.kind == BES_ELEMENTWISE || o.kind == BES_EXPR) && o.nsrc == 2) ? 2 : 1;
    if (o.nsrc != want_src) {
      err = "bad source count for operand kind";
      return BES_E_INVALID;
    }
    if (o.kind == BES_ELEMENTWISE && (o.op < BES_OP_ID || o.op > BES_OP_SQUARE)) {
      err = "unknown elementwise op";
      return BES_E_UNSUPPORTED;
    }
    if (o.kind == BES_TET_JACOBIAN && (o.ndim != 3 || o.shape[1] != 3 || o.shape[2] != 3)) {
      err = "tetrahedron Jacobian operands have shape (e,3,3)";
      return BES_E_INVALID;
    }
    if (o.kind == BES_EXPR) {
      if (!exprs || !exprs[a]) {
        err = "expression operand " + std::to_string(a) + " has no body";
        return BES_E_INVALID;
      }
      d.expr = exprs[a];
      if (!valid_expression(d.expr, err)) return BES_E_INVALID;
    }
    d.kind = o.kind;
    d.dtype = o.dtype;
    d.ndim = o.ndim;
    d.nsrc = o.nsrc;
    d.op = o.op;
    d.alpha = o.alpha;
    d.beta = o.beta;
    for (int k = 0; k < o.ndim; ++k) {
      if (o.shape[k] < 0) {
        err = "negative extent";
        return BES_E_INVALID;
      }
      d.shape[k] = o.shape[k];
    }
    for (int s = 0; s < d.nsrc; ++s) {
      d.src_offset[s] = o.src_offset[s];
      bool any = false;
      for (int k = 0; k < o.ndim; ++k) any |= o.src_strides[s][k] != 0;
      if (any) {
        for (int k = 0; k < o.ndim; ++k) d.src_strides[s][k] = o.src_strides[s][k];
      } else if (o.kind == BES_TET_JACOBIAN) {
        d.src_strides[s][0] = 12;  // S0[e, 4, 3] dense
        d.src_strides[s][1] = 3;
        d.src_strides[s][2] = 1;
      } else {
        int64_t st = 1;
        for (int k = o.ndim - 1; k >= 0; --k) {
          d.src_strides[s][k] = st;
          st *= d.shape[k];
        }
      }
    }
  }
  // Table and per-member soundness (conditions after Eq. (1)).
  std::vector<char> used(n_args, 0);
  for (int c = 0; c < kLetters; ++c) spec.extent[c] = -1;
  for (int i = 0; i < b; ++i) {
    for (int j = 0; j < n; ++j) {
      int a = spec.arg(i, j);
      if (a < 0 || a >= n_args) {
        err = "table entry out of range";
        return BES_E_INVALID;
      }
      used[a] = 1;
      const Operand &o = spec.args[a];
      if ((int)spec.ins[j].size() != o.ndim) {
        err = "operand rank differs from its index list (member " + std::to_string(i) +
              ", position " + std::to_string(j) + ")";
        return BES_E_INVALID;
      }
      for (int d = 0; d < o.ndim; ++d) {
        int c = spec.ins[j][d];
        if (spec.extent[c] < 0) {
          spec.extent[c] = o.shape[d];
        } else if (spec.extent[c] != o.shape[d]) {
          err = std::string("index '") + char('a' + c) + "' has inconsistent extents";
          return BES_E_INVALID;
        }
      }
    }
  }
  for (int a = 0; a < n_args; ++a) {
    if (!used[a]) {
      err = "argument " + std::to_string(a) + " does not occur in the table";
      return BES_E_INVALID;
    }
  }
  bool seen[kLetters] = {false};
  for (int c : spec.out) {
    if (seen[c]) {
      err = "repeated output index";  // C27
      return BES_E_INVALID;
    }
    seen[c] = true;
    if (spec.extent[c] < 0) {
      err = std::string("output index '") + char('a' + c) + "' does not index any input";
      return BES_E_INVALID;
    }
  }
  // Mixed dtypes canonicalize (the dtype nodes and their rank tournament
  // encode them) but no kernel evaluates them: spec.dtype = 0 then.
  spec.dtype = spec.args[0].dtype;
  for (const auto &o : spec.args)
    if (o.dtype != spec.dtype) spec.dtype = 0;
  return BES_OK;
}

}  // namespace bes
