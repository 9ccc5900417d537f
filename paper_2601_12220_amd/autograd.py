"""Differentiable batched einsums: torch.autograd.Function over the C ABI.

Forward launches the registered plan.  Backward launches, for every operand
position whose arguments need a gradient, the adjoint plan the library builds
for that position (bes_adjoint): a batched einsum over (G_i, the other
operands of member i) that is itself canonicalized, keyed and tuned, and that
sums the members sharing an argument.  Every output of an adjoint plan is
written by the library straight into the gradient of its source buffer
(bes_plan_set_output): through the view's offset and strides for a VIEW
argument, overwriting where this contribution is the first to cover that
memory and adding into it otherwise, so a buffer read at several positions or
through several views gets the sum of all its contributions.  This module
only allocates the gradient tensors and passes pointers.

Only ARRAY and VIEW arguments are differentiable.  Asking for the gradient of
a buffer that is also a source of an element-wise or tetrahedron-Jacobian
operand raises in forward: the library does not differentiate those functions.
"""
from __future__ import annotations

from typing import Dict, FrozenSet, List, Sequence, Tuple

import numpy as np
import torch

from . import Context, Plan, capi

_DT = {"float32": torch.float32, "float64": torch.float64}
_CODE = {"float32": capi.BES_FLOAT32, "float64": capi.BES_FLOAT64}


def _dense_strides(shape) -> Tuple[int, ...]:
    st, v = [], 1
    for s in reversed(shape):
        st.append(v)
        v *= int(s)
    return tuple(reversed(st))


class BatchedEinsum:
    """A registered batched einsum that can be called on torch tensors and
    differentiated.  ``operands`` maps argument names to descriptors with
    shape/dtype/kind/sources/offset/strides attributes (kinds ``array`` and
    ``view`` are differentiable; element-wise and Jacobian operands are
    evaluated but not differentiated)."""

    def __init__(self, ctx: Context, notation: str, table: Sequence[Sequence[str]],
                 operands: Dict[str, object]):
        self.ctx = ctx
        self.notation = notation
        self.table = [list(r) for r in table]
        self.operands = operands
        self.plan: Plan = ctx.register(notation, self.table, operands)
        self._adjoints: Dict[int, Plan] = {}
        self._programs: Dict[FrozenSet[str], list] = {}
        lhs, rhs = notation.split("->")
        ext = {}
        for labels, a in zip(lhs.split(","), self.table[0]):
            for ch, s in zip(labels, operands[a].shape):
                ext[ch] = s
        self.out_shape = tuple(ext[c] for c in rhs)
        self.dtype_name = operands[self.table[0][0]].dtype
        self.dtype = _DT[self.dtype_name]
        self.buffer_names = sorted({s for a in self.operands for s in self.operands[a].sources})
        used = {a for row in self.table for a in row}
        self.nondiff_sources = {s for a in used if self.operands[a].kind not in ("array", "view")
                                for s in self.operands[a].sources}

    def adjoint(self, pos: int) -> Plan:
        if pos not in self._adjoints:
            self._adjoints[pos] = self.plan.adjoint(pos)
        return self._adjoints[pos]

    # -- where each adjoint output goes ------------------------------------

    def _slot_args(self, pos: int) -> List[str]:
        args: List[str] = []
        for row in self.table:
            if row[pos] not in args:
                args.append(row[pos])
        return args

    def _layout(self, arg: str) -> Tuple[int, Tuple[int, ...]]:
        """(offset, strides) of argument ``arg`` in its source buffer."""
        o = self.operands[arg]
        if o.kind == "view":
            return int(o.offset), tuple(int(s) for s in o.strides)
        return 0, _dense_strides(o.shape)

    def _addresses(self, arg: str) -> np.ndarray:
        off, st = self._layout(arg)
        addr = np.full((), off, dtype=np.int64)
        for ext, s in zip(self.operands[arg].shape, st):
            addr = np.add.outer(addr, np.arange(ext, dtype=np.int64) * s)
        return addr.ravel()

    def _covers_exactly(self, args: List[str], numel: int) -> bool:
        """Do the arguments together address every element of their buffer
        exactly once?"""
        if sum(int(np.prod(self.operands[a].shape)) for a in args) != numel:
            return False
        addr = np.concatenate([self._addresses(a) for a in args])
        if addr.size and (addr.min() < 0 or addr.max() >= numel):
            return False
        return bool(np.all(np.bincount(addr, minlength=numel) == 1))

    def _program(self, wanted: FrozenSet[str], numel: Dict[str, int]):
        """Per position with a wanted gradient: (pos, [(slot, buffer or None,
        offset, strides, accumulate)]), plus the buffers to zero first."""
        if wanted in self._programs:
            return self._programs[wanted]
        n = len(self.table[0])
        contrib: Dict[str, List[Tuple[int, str]]] = {s: [] for s in wanted}
        positions = []
        for pos in range(n):
            args = self._slot_args(pos)
            hits = [a for a in args if self.operands[a].kind in ("array", "view")
                    and self.operands[a].sources[0] in wanted]
            if not hits:
                continue
            positions.append((pos, args))
            for a in hits:
                contrib[self.operands[a].sources[0]].append((pos, a))
        overwrite = set()
        zero_first = []
        for s in sorted(wanted):
            cs = contrib[s]
            if not cs:
                zero_first.append(s)          # no argument reads it: zero gradient
                continue
            first_pos = cs[0][0]
            first = [a for p, a in cs if p == first_pos]
            if self._covers_exactly(first, numel[s]):
                overwrite.update((first_pos, a) for a in first)
            else:
                zero_first.append(s)
        prog = []
        for pos, args in positions:
            slots = []
            for k, a in enumerate(args):
                o = self.operands[a]
                src = o.sources[0] if o.kind in ("array", "view") else None
                if src in wanted:
                    off, st = self._layout(a)
                    slots.append((k, src, off, st, (pos, a) not in overwrite))
                else:
                    slots.append((k, None, 0, None, False))   # not wanted: scratch
            prog.append((pos, slots))
        self._programs[wanted] = (prog, zero_first)
        return self._programs[wanted]

    def __call__(self, buffers: Dict[str, torch.Tensor]) -> List[torch.Tensor]:
        tensors = [buffers[n] for n in self.buffer_names]
        return list(_BatchedEinsumFn.apply(self, *tensors))


class _BatchedEinsumFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, be: BatchedEinsum, *tensors):
        for k, nm in enumerate(be.buffer_names):
            if ctx.needs_input_grad[1 + k] and nm in be.nondiff_sources:
                raise ValueError(
                    f"buffer {nm!r} is a source of an element-wise or tetrahedron-Jacobian "
                    "operand; the library differentiates array and view operands only")
        bufs = {n: t.contiguous() for n, t in zip(be.buffer_names, tensors)}
        outs = [torch.empty(be.out_shape, dtype=be.dtype, device=tensors[0].device)
                for _ in be.table]
        be.plan.launch(bufs, outs)
        ctx.be = be
        ctx.save_for_backward(*[bufs[n] for n in be.buffer_names])
        return tuple(outs)

    @staticmethod
    def backward(ctx, *grads):
        be: BatchedEinsum = ctx.be
        saved = ctx.saved_tensors
        bufs = dict(zip(be.buffer_names, saved))
        wanted = frozenset(n for k, n in enumerate(be.buffer_names) if ctx.needs_input_grad[1 + k])
        if not wanted:
            return (None,) * (1 + len(be.buffer_names))
        dev = saved[0].device
        stream = int(torch.cuda.current_stream().cuda_stream)
        code = _CODE[be.dtype_name]
        G = []
        for g in grads:
            if g is None:                      # an output without gradient: zeros
                g = torch.empty(be.out_shape, dtype=be.dtype, device=dev)
                capi.bes_fill_zero(g.data_ptr(), g.numel(), code, stream)
            G.append(g.contiguous())
        src = [g.data_ptr() for g in G] + be.plan.src_ptrs(bufs)
        prog, zero_first = be._program(wanted, {n: bufs[n].numel() for n in wanted})
        gbuf = {n: torch.empty_like(bufs[n]) for n in wanted}
        for n in zero_first:
            capi.bes_fill_zero(gbuf[n].data_ptr(), gbuf[n].numel(), code, stream)
        keep = []
        for pos, slots in prog:
            adj = be.adjoint(pos)
            outs = []
            for k, srcname, off, st, acc in slots:
                if srcname is None:
                    shape = be.operands[be._slot_args(pos)[k]].shape
                    t = torch.empty(shape, dtype=be.dtype, device=dev)
                    keep.append(t)
                    capi.bes_plan_set_output(adj.h, k)
                    outs.append(t.data_ptr())
                else:
                    capi.bes_plan_set_output(adj.h, k, off, st, acc)
                    outs.append(gbuf[srcname].data_ptr())
            adj.launch_ptrs(src, outs, stream)
        return (None, *[gbuf.get(nm) for nm in be.buffer_names])
