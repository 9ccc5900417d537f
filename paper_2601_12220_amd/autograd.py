"""Differentiable batched einsums: torch.autograd.Function over the C ABI.

Forward launches the registered plan.  Backward launches, for every operand
position whose arguments need a gradient, the adjoint plan the library builds
for that position (bes_adjoint): a batched einsum over (G_i, the other
operands of member i) that is itself canonicalized, keyed and tuned, and that
sums the members sharing an argument.  The gradient of an ARRAY argument is
that output; the gradient of a VIEW argument is scattered into its source
buffer's gradient through the view's strides.
"""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence

import torch

from . import Context, Plan

_DT = {"float32": torch.float32, "float64": torch.float64}


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
        lhs, rhs = notation.split("->")
        ext = {}
        for labels, a in zip(lhs.split(","), self.table[0]):
            for ch, s in zip(labels, operands[a].shape):
                ext[ch] = s
        self.out_shape = tuple(ext[c] for c in rhs)
        self.dtype = _DT[operands[self.table[0][0]].dtype]
        self.buffer_names = sorted({s for a in self.operands for s in self.operands[a].sources})

    def adjoint(self, pos: int) -> Plan:
        if pos not in self._adjoints:
            self._adjoints[pos] = self.plan.adjoint(pos)
        return self._adjoints[pos]

    def __call__(self, buffers: Dict[str, torch.Tensor]) -> List[torch.Tensor]:
        tensors = [buffers[n] for n in self.buffer_names]
        return list(_BatchedEinsumFn.apply(self, *tensors))


class _BatchedEinsumFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, be: BatchedEinsum, *tensors):
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
        need = {n: ctx.needs_input_grad[1 + k] for k, n in enumerate(be.buffer_names)}
        dev = saved[0].device
        G = [g.contiguous() if g is not None else
             torch.zeros(be.out_shape, dtype=be.dtype, device=dev) for g in grads]
        src = [g.data_ptr() for g in G] + be.plan.src_ptrs(bufs)
        gbuf: Dict[str, Optional[torch.Tensor]] = {n: None for n in be.buffer_names}
        stream = int(torch.cuda.current_stream().cuda_stream)
        n = len(be.table[0])
        for pos in range(n):
            args: List[str] = []
            for row in be.table:
                if row[pos] not in args:
                    args.append(row[pos])
            wanted = [a for a in args
                      if be.operands[a].kind in ("array", "view") and need[be.operands[a].sources[0]]]
            if not wanted:
                continue
            adj = be.adjoint(pos)
            outs = [torch.empty(be.operands[a].shape, dtype=be.dtype, device=dev) for a in args]
            adj.launch_ptrs(src, [o.data_ptr() for o in outs], stream)
            for a, o in zip(args, outs):
                if a not in wanted:
                    continue
                op = be.operands[a]
                s = op.sources[0]
                if gbuf[s] is None:
                    gbuf[s] = torch.zeros_like(bufs[s])
                if op.kind == "array":
                    gbuf[s] += o.view_as(gbuf[s])
                else:  # view: scatter through the view's strides
                    gbuf[s].as_strided(op.shape, op.strides, op.offset).add_(o)
        return (None, *[gbuf[nm] for nm in be.buffer_names])
