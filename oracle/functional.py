"""FP64 materialization of functional operands.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Definition "Functional Batched Einstein Summation" replaces each argument A by a
function M(A): dom(A) -> codomain(A).  The oracle evaluates every such function
on its whole domain first (materializes it) and then runs the plain loop nest,
which is exactly what the definition's formula states.  The functions below are
the operand kinds the library accepts; each is written from its mathematical
definition in numpy.
"""
from __future__ import annotations

import numpy as np

UNARY_OPS = ("id", "sin", "cos", "square")


def strided_view(flat_source, shape, strides, offset=0) -> np.ndarray:
    """M(A)[i_1..i_d] = S[offset + sum_k i_k * strides[k]] (element strides)."""
    src = np.ascontiguousarray(np.asarray(flat_source, dtype=np.float64).reshape(-1))
    if len(shape) == 0:
        return np.array(src[offset])
    lo = offset + sum(min(0, (n - 1) * s) for n, s in zip(shape, strides))
    hi = offset + sum(max(0, (n - 1) * s) for n, s in zip(shape, strides))
    if any(n == 0 for n in shape):
        return np.zeros(tuple(shape))
    if lo < 0 or hi >= src.size:
        raise IndexError("view reaches outside its source")
    item = src.itemsize
    view = np.lib.stride_tricks.as_strided(src[offset:], shape=tuple(shape),
                                           strides=tuple(int(s) * item for s in strides),
                                           writeable=False)
    return np.array(view)


def unary(x, op: str) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    if op == "id":
        return x
    if op == "sin":
        return np.sin(x)
    if op == "cos":
        return np.cos(x)
    if op == "square":
        return x * x
    raise ValueError(op)


def elementwise(src0, op: str = "id", alpha: float = 1.0, beta: float = 0.0,
                src1=None) -> np.ndarray:
    """M(A)[idx] = alpha * op(S0[idx]) + beta (+ S1[idx] when given).

    Covers the affine operands (alpha*A + beta) of the TCCG experiment, the
    substitution rules u = P*P, v = 3 cos(Q) + 5, w = sin(R) of the functional
    retrieval listing, and u = sin(a) + b.
    """
    val = float(alpha) * unary(src0, op) + float(beta)
    if src1 is not None:
        val = val + np.asarray(src1, dtype=np.float64)
    return val


def tet_jacobian(V) -> np.ndarray:
    """Affine tetrahedron map x(xi) = v_0 + sum_r xi_r (v_{r+1} - v_0):
    J[e, x, r] = d x_x / d xi_r = V[e, r+1, x] - V[e, 0, x], V of shape [e,4,3]."""
    V = np.asarray(V, dtype=np.float64)
    if V.ndim != 3 or V.shape[1:] != (4, 3):
        raise ValueError("V must have shape [e, 4, 3]")
    J = np.empty((V.shape[0], 3, 3), dtype=np.float64)
    for x in range(3):
        for r in range(3):
            J[:, x, r] = V[:, r + 1, x] - V[:, 0, x]
    return J


# Functions an expression body may call, each as numpy evaluates it in FP64.
_EXPR_FUNCS = {"sin": np.sin, "cos": np.cos, "tan": np.tan, "exp": np.exp, "log": np.log,
               "sqrt": np.sqrt, "fabs": np.fabs, "tanh": np.tanh, "pow": np.power,
               "fmin": np.fmin, "fmax": np.fmax}


def expression(body: str, src0, src1=None) -> np.ndarray:
    """M(A)[idx] = body(S0[idx], S1[idx]): a substitution-rule body of the
    functional retrieval listing (e.g. "s0*s0", "3*cos(s0)+5", "sin(s0)"),
    evaluated in FP64 over the whole domain.  The body is read with Python's
    own parser and only numbers, s0, s1, + - * / , unary signs and the
    functions above are evaluated."""
    import ast

    env = {"s0": np.asarray(src0, dtype=np.float64)}
    env["s1"] = np.asarray(src1, dtype=np.float64) if src1 is not None else env["s0"]

    def ev(node):
        if isinstance(node, ast.Expression):
            return ev(node.body)
        if isinstance(node, ast.Constant) and isinstance(node.value, (int, float)):
            return float(node.value)
        if isinstance(node, ast.Name) and node.id in ("s0", "s1"):
            return env[node.id]
        if isinstance(node, ast.UnaryOp) and isinstance(node.op, (ast.USub, ast.UAdd)):
            v = ev(node.operand)
            return -v if isinstance(node.op, ast.USub) else v
        if isinstance(node, ast.BinOp):
            a, b = ev(node.left), ev(node.right)
            if isinstance(node.op, ast.Add):
                return a + b
            if isinstance(node.op, ast.Sub):
                return a - b
            if isinstance(node.op, ast.Mult):
                return a * b
            if isinstance(node.op, ast.Div):
                return a / b
        if (isinstance(node, ast.Call) and isinstance(node.func, ast.Name) and
                node.func.id in _EXPR_FUNCS and not node.keywords):
            return _EXPR_FUNCS[node.func.id](*[ev(a) for a in node.args])
        raise ValueError(f"not an expression body: {ast.dump(node)}")

    val = ev(ast.parse(body, mode="eval"))
    return np.broadcast_to(np.asarray(val, dtype=np.float64), env["s0"].shape).copy()
