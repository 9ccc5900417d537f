"""Batched Einstein summations on MI355X (gfx950), following arxiv 2601.12220.

Thin Python layer over the C ABI in ``include/bes.h`` (bound in
:mod:`paper_2601_12220_amd.capi`).  Every step of the path -- parsing,
canonicalization, tuning lookup, binding and the HIP kernels -- runs in the
native library; this module only marshals torch tensors and descriptors.

    ctx = Context("tuning.db")
    plan = ctx.register("er,rij,ej->ei", table, operands)
    plan.launch(buffers, outputs)          # on torch's current HIP stream
"""
from __future__ import annotations

import ctypes
from typing import Dict, List, Optional, Sequence

from . import capi
from .capi import BesError  # noqa: F401

__all__ = ["Context", "Plan", "Batch", "make_operand", "capi", "BesError"]


def make_operand(shape, dtype="float64", kind="array", sources=None, offset=0,
                 strides=None, op="id", alpha=1.0, beta=0.0, src_strides=None,
                 src_offsets=None) -> capi.bes_operand:
    """Build a bes_operand.  ``kind``: array | view | elementwise | tet_jacobian."""
    o = capi.bes_operand()
    o.kind = {"array": capi.BES_ARRAY, "view": capi.BES_VIEW,
              "elementwise": capi.BES_ELEMENTWISE,
              "tet_jacobian": capi.BES_TET_JACOBIAN, "expr": capi.BES_EXPR}[kind]
    o.dtype = capi.DTYPE_CODE[dtype]
    o.ndim = len(shape)
    for d, s in enumerate(shape):
        o.shape[d] = int(s)
    nsrc = len(sources) if sources else 1
    o.nsrc = nsrc
    if kind == "view":
        o.src_offset[0] = int(offset)
        for d, s in enumerate(strides):
            o.src_strides[0][d] = int(s)
    if src_strides:
        for k, st in enumerate(src_strides):
            if st is not None:
                for d, s in enumerate(st):
                    o.src_strides[k][d] = int(s)
    if src_offsets:
        for k, off in enumerate(src_offsets):
            o.src_offset[k] = int(off)
    o.op = capi.OP_CODE.get(op, 0)
    o.alpha = float(alpha)
    o.beta = float(beta)
    return o


def _operand_from_desc(d) -> capi.bes_operand:
    """From a duck-typed descriptor with name/shape/dtype/kind/sources/... .
    An element-wise operand with ``strides`` reads its first source through
    that view (offset and strides)."""
    strides = getattr(d, "strides", None)
    offset = getattr(d, "offset", 0)
    ew_view = d.kind in ("elementwise", "expr") and strides is not None
    return make_operand(d.shape, d.dtype, d.kind, d.sources, offset, strides,
                        getattr(d, "op", "id"), getattr(d, "alpha", 1.0), getattr(d, "beta", 0.0),
                        src_strides=[strides] if ew_view else None,
                        src_offsets=[offset] if ew_view else None)


def _stream_handle(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Context:
    """Owns the tuning database (None = no database file)."""

    def __init__(self, db_path: Optional[str] = None):
        capi.load()
        self.db_path = db_path
        self.h = capi.bes_ctx_create(db_path)

    def close(self):
        if self.h:
            capi.bes_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def register(self, notation: str, table: Sequence[Sequence[str]], operands: Dict[str, object],
                 arg_order: Optional[List[str]] = None) -> "Plan":
        """Register a batched einsum.  ``operands`` maps argument names to
        descriptors (objects with shape/dtype/kind/sources/... attributes, or
        bes_operand instances paired with a ``sources`` list)."""
        names = arg_order or sorted({a for row in table for a in row})
        idx = {nm: k for k, nm in enumerate(names)}
        descs, sources, exprs = [], [], []
        for nm in names:
            d = operands[nm]
            if isinstance(d, tuple):
                descs.append(d[0])
                sources.append(list(d[1]))
                exprs.append(d[2] if len(d) > 2 else None)
            else:
                descs.append(_operand_from_desc(d))
                sources.append(list(d.sources) if d.sources else [nm])
                exprs.append(getattr(d, "expr", None) if d.kind == "expr" else None)
        flat = [idx[a] for row in table for a in row]
        h, status = capi.bes_register(self.h, notation, len(table), len(table[0]), descs, flat,
                                      exprs)
        return Plan(self, h, notation, [list(r) for r in table], names, sources, status)

    def record(self, key: str, cfg: capi.bes_config, seconds: float, arch: str = "gfx950"):
        capi.bes_db_record(self.h, key, arch, cfg, seconds)

    def stats(self):
        return capi.bes_ctx_stats(self.h)


class Plan:
    def __init__(self, ctx: Context, h, notation, table, names, sources, status, n_out=None):
        self.ctx = ctx
        self.h = h
        self.notation = notation
        self.table = table
        self.names = names          # user argument order
        self.sources = sources      # per argument: source buffer names
        self.status = status        # BES_OK (record hit) or BES_W_NOTFOUND
        self.n_out = n_out if n_out is not None else len(table)

    def __del__(self):
        try:
            if self.h:
                capi.bes_plan_destroy(self.h)
                self.h = None
        except Exception:
            pass

    @property
    def key(self) -> str:
        return capi.bes_plan_key(self.h)

    @property
    def canonical(self) -> str:
        return capi.bes_plan_canonical(self.h)

    def maps(self):
        """(member_map, pos_map, arg_map as names, index_map) from canonical
        names to this registration's names."""
        b, n = len(self.table), len(self.table[0])
        mm, pm, am, im = capi.bes_plan_maps(self.h, b, n, len(self.names))
        return mm, pm, [self.names[a] for a in am], im

    def graph(self, which: int = 0):
        return capi.bes_plan_graph(self.h, which)

    @property
    def config(self) -> capi.bes_config:
        return capi.bes_plan_get_config(self.h)

    @property
    def template(self) -> str:
        return capi.TEMPLATE_NAME[self.config.template_id]

    def set_config(self, template_id: int, *params: int):
        c = capi.bes_config()
        c.template_id = template_id
        for k, v in enumerate(params):
            c.p[k] = int(v)
        capi.bes_plan_set_config(self.h, c)

    def lookup(self, arch: str = "gfx950") -> int:
        return capi.bes_plan_lookup(self.ctx.h, self.h, arch)

    def src_ptrs(self, buffers: Dict[str, object]) -> List[int]:
        ptrs = []
        for nm, srcs in zip(self.names, self.sources):
            for s in srcs:
                t = buffers[s]
                ptrs.append(t.data_ptr())
        return ptrs

    def launch(self, buffers: Dict[str, object], outputs: Sequence[object], stream=None):
        """Enqueue on ``stream`` (default: torch's current stream).  Device
        tensors only; outputs are overwritten."""
        capi.bes_launch(self.h, self.src_ptrs(buffers), [o.data_ptr() for o in outputs],
                        _stream_handle(stream))

    def launch_ptrs(self, src_ptrs: Sequence[int], out_ptrs: Sequence[int], stream: int = 0):
        capi.bes_launch(self.h, list(src_ptrs), list(out_ptrs), stream)

    def set_timing(self, start_event=None, stop_event=None):
        """Record torch.cuda.Event ``start_event`` / ``stop_event`` around the
        plan's evaluation kernel(s) on every later launch (None, None: off).
        The events must stay alive while they are in use."""
        import torch
        for ev in (start_event, stop_event):
            if ev is not None and not ev.cuda_event:   # torch creates events lazily
                ev.record(torch.cuda.current_stream())
        h0 = start_event.cuda_event if start_event is not None else 0
        h1 = stop_event.cuda_event if stop_event is not None else 0
        capi.bes_plan_set_timing(self.h, h0, h1)

    def adjoint(self, pos: int) -> "Plan":
        h, n_out, status = capi.bes_adjoint(self.ctx.h, self.h, pos)
        return Plan(self.ctx, h, None, None, None, None, status, n_out)


class Batch:
    """Persistent batched launch of many plans (hipGraph-captured)."""

    def __init__(self, ctx: Context, plans: Sequence[Plan]):
        self.ctx = ctx
        self.plans = list(plans)
        self.h = capi.bes_batch_create(ctx.h, [p.h for p in self.plans])

    def __del__(self):
        try:
            if self.h:
                capi.bes_batch_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def launch(self, buffers: Sequence[Dict[str, object]], outputs: Sequence[Sequence[object]],
               stream=None):
        srcs = [p.src_ptrs(b) for p, b in zip(self.plans, buffers)]
        outs = [[o.data_ptr() for o in os_] for os_ in outputs]
        capi.bes_batch_launch(self.h, srcs, outs, _stream_handle(stream))

    def launch_ptrs(self, srcs, outs, stream: int = 0):
        capi.bes_batch_launch(self.h, srcs, outs, stream)

    def bind_ptrs(self, srcs, outs, stream: int = 0):
        """Bind device pointers once (bes_batch_bind); replay() then launches
        on them without marshalling 256 pointer lists per launch."""
        capi.bes_batch_bind(self.h, srcs, outs, stream)

    def replay(self, stream: int = 0):
        capi.bes_batch_replay(self.h, stream)
