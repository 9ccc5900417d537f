"""Raising traced programs to functional batched einsums.

The paper retrieves a tuned transformation for code written as ordinary loops
by *raising* it: the statements are interpreted as a functional batched
einsum, that einsum is canonicalized, and the database is queried with its
canonical form (Section "Integration with a Code Transformation Framework",
the retrieval listing).  Algorithm "IdentifyAsEinsum" then composes the
canonical substitutions of a reference batched einsum and the raised one, so
that a transformation written against the reference's names applies to the
raised program's names.

Here the program is a ``torch.fx`` graph of ``torch.einsum`` calls:

* every einsum operand must be a graph input, a strided view of one
  (``x[:, k, :]``, ``x.transpose(0, 1)``, ``x.permute(...)``), or an element-wise
  function of inputs that the library evaluates in registers:
  ``alpha * op(x) + beta (+ y)`` with op in {identity, sin, cos, square};
* einsum calls with the same notation (up to renaming of its letters) and the
  same operand shapes and dtype are grouped into one batched einsum, whose
  members share every argument they have in common (the same input, view or
  function of the same inputs) -- the automatic batching of einsums that
  share operands.

:func:`compile_fx` traces a function, raises its einsum calls, registers every
batched einsum with the library (canonicalization and tuning lookup run in
the C library) and returns a callable that evaluates each batch with one
launch.  :func:`identify_as_einsum` is Algorithm "IdentifyAsEinsum" on two
registered plans (the composition runs in the library, ``bes_identify``).
This module only walks Python graph objects and marshals descriptors.
"""
from __future__ import annotations

import operator
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence, Tuple

from . import Context, Plan, capi


@dataclass
class Func:
    """M(A)[idx] = alpha * op(S0[view]) + beta (+ S1[view]) of one or two inputs."""
    src0: str
    op: str = "id"
    alpha: float = 1.0
    beta: float = 0.0
    src1: Optional[str] = None
    shape: Tuple[int, ...] = ()
    offset: int = 0
    strides: Optional[Tuple[int, ...]] = None   # view of src0 (None: dense)

    def pure(self) -> bool:
        return self.op == "id" and self.alpha == 1.0 and self.beta == 0.0 and self.src1 is None

    def key(self):
        return (self.src0, self.op, self.alpha, self.beta, self.src1, self.shape, self.offset,
                self.strides)


@dataclass
class RaisedBatch:
    """One functional batched einsum raised from the graph."""
    notation: str
    table: List[List[str]]
    operands: Dict[str, object]          # argument name -> descriptor
    nodes: List[object]                  # the fx nodes of the members, in order
    plan: Optional[Plan] = None


@dataclass
class _Operand:
    name: str
    shape: Tuple[int, ...]
    dtype: str
    kind: str
    sources: Tuple[str, ...]
    offset: int = 0
    strides: Optional[Tuple[int, ...]] = None
    op: str = "id"
    alpha: float = 1.0
    beta: float = 0.0


_DTYPES = {"torch.float32": "float32", "torch.float64": "float64"}


def _dense_strides(shape):
    st, v = [], 1
    for s in reversed(shape):
        st.append(v)
        v *= int(s)
    return tuple(reversed(st))


def _normalize(notation: str) -> str:
    """Rename letters in order of first occurrence: 'ab,b->a' -> 'ab,b->a',
    'ij,j->i' -> 'ab,b->a'."""
    m: Dict[str, str] = {}
    out = []
    for ch in notation:
        if ch.isalpha():
            if ch not in m:
                m[ch] = chr(ord("a") + len(m))
            out.append(m[ch])
        else:
            out.append(ch)
    return "".join(out)


class _Raiser:
    def __init__(self, gm, shapes: Dict[str, Tuple[int, ...]], dtypes: Dict[str, str]):
        import torch
        self.torch = torch
        self.gm = gm
        self.shapes = shapes
        self.dtypes = dtypes
        self.funcs: Dict[object, Optional[Func]] = {}

    def _scalar(self, a):
        return isinstance(a, (int, float)) and not isinstance(a, bool)

    def func(self, node) -> Optional[Func]:
        """The element-wise function (of inputs) a node computes, or None."""
        if node in self.funcs:
            return self.funcs[node]
        f = self._func(node)
        self.funcs[node] = f
        return f

    def _func(self, node) -> Optional[Func]:
        torch = self.torch
        if not hasattr(node, "op"):
            return None
        if node.op == "placeholder":      # target: the argument's own name
            if node.target not in self.shapes:
                return None
            shp = tuple(self.shapes[node.target])
            return Func(node.target, shape=shp, strides=_dense_strides(shp))
        if node.op == "call_method" and node.target in ("transpose", "permute"):
            base = self.func(node.args[0])
            if base is None or not base.pure():
                return None
            dims = list(range(len(base.shape)))
            if node.target == "transpose":
                a, b = node.args[1], node.args[2]
                dims[a], dims[b] = dims[b], dims[a]
            else:
                dims = list(node.args[1] if len(node.args) == 2 and
                            isinstance(node.args[1], (list, tuple)) else node.args[1:])
            return Func(base.src0, shape=tuple(base.shape[d] for d in dims),
                        offset=base.offset, strides=tuple(base.strides[d] for d in dims))
        if node.op == "call_function" and node.target is operator.getitem:
            base = self.func(node.args[0])
            if base is None or not base.pure():
                return None
            idx = node.args[1] if isinstance(node.args[1], tuple) else (node.args[1],)
            shape, strides, off = [], [], base.offset
            d = 0
            for it in idx:
                if isinstance(it, int):
                    off += it * base.strides[d]
                elif isinstance(it, slice) and it.step in (None, 1):
                    start = it.start or 0
                    stop = base.shape[d] if it.stop is None else min(it.stop, base.shape[d])
                    off += start * base.strides[d]
                    shape.append(stop - start)
                    strides.append(base.strides[d])
                else:
                    return None
                d += 1
            shape += list(base.shape[d:])
            strides += list(base.strides[d:])
            return Func(base.src0, shape=tuple(shape), offset=off, strides=tuple(strides))
        if node.op != "call_function":
            return None
        t, args = node.target, node.args
        unary = {torch.sin: "sin", torch.cos: "cos", torch.square: "square"}
        if t in unary:
            f = self.func(args[0])
            if f is None or not f.pure():
                return None
            return Func(f.src0, op=unary[t], shape=f.shape, offset=f.offset, strides=f.strides)
        if t in (operator.mul, torch.mul):
            a, b = args[0], args[1]
            if not self._scalar(a) and not self._scalar(b):
                fa, fb = self.func(a), self.func(b)
                if fa is not None and fb is not None and fa.pure() and fa.key() == fb.key():
                    return Func(fa.src0, op="square", shape=fa.shape, offset=fa.offset,
                                strides=fa.strides)
                return None
            c, x = (a, b) if self._scalar(a) else (b, a)
            f = self.func(x)
            if f is None or f.src1 is not None:
                return None
            return Func(f.src0, f.op, f.alpha * c, f.beta * c, None, f.shape, f.offset, f.strides)
        if t in (operator.pow, torch.pow) and args[1] == 2:
            f = self.func(args[0])
            if f is None or not f.pure():
                return None
            return Func(f.src0, op="square", shape=f.shape, offset=f.offset, strides=f.strides)
        if t in (operator.neg, torch.neg):
            f = self.func(args[0])
            if f is None or f.src1 is not None:
                return None
            return Func(f.src0, f.op, -f.alpha, -f.beta, None, f.shape, f.offset, f.strides)
        if t in (operator.add, torch.add, operator.sub, torch.sub):
            sign = -1.0 if t in (operator.sub, torch.sub) else 1.0
            a, b = args[0], args[1]
            if self._scalar(b) or self._scalar(a):
                c, x = (b, a) if self._scalar(b) else (a, b)
                if self._scalar(a) and sign < 0:      # c - f
                    f = self.func(x)
                    if f is None or f.src1 is not None:
                        return None
                    return Func(f.src0, f.op, -f.alpha, c - f.beta, None, f.shape, f.offset,
                                f.strides)
                f = self.func(x)
                if f is None or f.src1 is not None:
                    return None
                return Func(f.src0, f.op, f.alpha, f.beta + sign * c, None, f.shape, f.offset,
                            f.strides)
            fa, fb = self.func(a), self.func(b)
            if fa is None or fb is None or sign < 0:
                return None
            # alpha*op(S0) + beta + S1: the second source is a plain dense input
            for f, g in ((fa, fb), (fb, fa)):
                if (g.pure() and f.src1 is None and g.shape == f.shape and
                        g.strides == _dense_strides(g.shape) and
                        f.strides == _dense_strides(f.shape) and f.offset == 0 and g.offset == 0):
                    return Func(f.src0, f.op, f.alpha, f.beta, g.src0, f.shape)
            return None
        return None

    def einsums(self):
        torch = self.torch
        found = []
        for node in self.gm.graph.nodes:
            if node.op == "call_function" and node.target in (torch.einsum,
                                                              torch.functional.einsum):
                nota = node.args[0]
                ops = node.args[1:]
                if len(ops) == 1 and isinstance(ops[0], (list, tuple)):
                    ops = ops[0]
                fs = [self.func(o) for o in ops]
                if "->" not in nota or any(f is None for f in fs):
                    continue
                found.append((node, nota.replace(" ", ""), fs))
        return found


def raise_fx(gm, example_inputs: Dict[str, object]) -> List[RaisedBatch]:
    """Raise the einsum calls of ``gm`` (a torch.fx.GraphModule whose inputs are
    named like ``example_inputs``' keys) to functional batched einsums."""
    shapes = {k: tuple(v.shape) for k, v in example_inputs.items()}
    dtypes = {k: _DTYPES[str(v.dtype)] for k, v in example_inputs.items()}
    r = _Raiser(gm, shapes, dtypes)
    groups: Dict[tuple, List[tuple]] = {}
    order: List[tuple] = []
    for node, nota, fs in r.einsums():
        dt = {dtypes[f.src0] for f in fs} | {dtypes[f.src1] for f in fs if f.src1}
        if len(dt) != 1:
            continue
        key = (_normalize(nota), tuple(f.shape for f in fs), dt.pop())
        if key not in groups:
            groups[key] = []
            order.append(key)
        groups[key].append((node, fs))
    out = []
    for key in order:
        nota, _, dtype = key
        members = groups[key]
        args: Dict[tuple, str] = {}
        operands: Dict[str, object] = {}
        table = []
        for node, fs in members:
            row = []
            for f in fs:
                k = f.key()
                if k not in args:
                    name = f"arg{len(args)}"
                    args[k] = name
                    srcs = (f.src0,) if f.src1 is None else (f.src0, f.src1)
                    dense = f.strides == _dense_strides(f.shape) and f.offset == 0
                    if f.op == "id" and f.alpha == 1.0 and f.beta == 0.0 and f.src1 is None:
                        kind = "array" if dense else "view"
                    else:
                        kind = "elementwise"
                    operands[name] = _Operand(name, f.shape, dtype, kind, srcs,
                                              offset=f.offset,
                                              strides=None if kind == "array" else f.strides,
                                              op=f.op, alpha=f.alpha, beta=f.beta)
                row.append(args[k])
            table.append(row)
        out.append(RaisedBatch(nota, table, operands, [m[0] for m in members]))
    return out


def identify_as_einsum(ref: Plan, raised: Plan):
    """Algorithm "IdentifyAsEinsum": the substitution from the reference
    batched einsum's names to the raised one's, as (sigma_A: reference
    argument name -> raised argument name, sigma_I: reference letter -> raised
    letter, member map, position map).  Raises capi.BesError when the two are
    not isomorphic."""
    b, n = len(ref.table), len(ref.table[0])
    mm, pm, am, im = capi.bes_identify(ref.h, raised.h, b, n, len(ref.names))
    sigma_a = {ref.names[a]: raised.names[am[a]] for a in range(len(ref.names))}
    return sigma_a, im, mm, pm


@dataclass
class CompiledFx:
    """A traced function whose einsum calls run as registered batched
    einsums, one launch per batch."""
    batches: List[RaisedBatch]
    outputs: List[object] = field(default_factory=list)   # fx nodes returned

    def __call__(self, **inputs):
        import torch
        results = {}
        for rb in self.batches:
            dev = next(iter(inputs.values())).device
            dt = {"float32": torch.float32, "float64": torch.float64}[
                rb.operands[rb.table[0][0]].dtype]
            lhs, rhs = rb.notation.split("->")
            ext = {}
            for labels, a in zip(lhs.split(","), rb.table[0]):
                for ch, s in zip(labels, rb.operands[a].shape):
                    ext[ch] = s
            outs = [torch.empty(tuple(ext[c] for c in rhs), dtype=dt, device=dev)
                    for _ in rb.table]
            bufs = {k: v.contiguous() for k, v in inputs.items()}
            rb.plan.launch(bufs, outs)
            for node, o in zip(rb.nodes, outs):
                results[node] = o
        return tuple(results[n] for n in self.outputs)


def compile_fx(fn: Callable, example_inputs: Dict[str, object],
               ctx: Optional[Context] = None) -> CompiledFx:
    """Trace ``fn`` (keyword inputs named as in ``example_inputs``; it must
    return a tuple of einsum results), raise and register its batched
    einsums.  Every returned value must come from a raised einsum."""
    import torch.fx
    ctx = ctx or Context()
    gm = torch.fx.symbolic_trace(fn)
    batches = raise_fx(gm, example_inputs)
    for rb in batches:
        rb.plan = ctx.register(rb.notation, rb.table, rb.operands)
    out_node = [n for n in gm.graph.nodes if n.op == "output"][0]
    rets = out_node.args[0]
    rets = list(rets) if isinstance(rets, (list, tuple)) else [rets]
    raised_nodes = {n for rb in batches for n in rb.nodes}
    for r_ in rets:
        if r_ not in raised_nodes:
            raise ValueError(f"output {r_} is not a raised einsum")
    return CompiledFx(batches, rets)
