"""GPU-test helpers: run a workload through the library's C ABI and compute
the oracle's answer for the same seeded inputs.

Oracle side: every functional operand is materialized in FP64 by
oracle.functional from the very buffers the GPU reads (upcast from their
compute dtype), then the oracle's loop nest evaluates Eq. (1) per member.
"""
from __future__ import annotations

import numpy as np
import torch

import oracle
from oracle import functional as F


def materialize(w, name):
    """FP64 value array of operand ``name`` of workload ``w`` (oracle side)."""
    o = w.operands[name]
    src = [w.buffers[s].double().numpy() for s in o.sources]
    if o.kind == "array":
        return src[0].reshape(o.shape)
    if o.kind == "view":
        return F.strided_view(src[0], o.shape, o.strides, o.offset)
    if o.kind == "elementwise":
        s0 = src[0].reshape(o.shape)
        s1 = src[1].reshape(o.shape) if len(src) > 1 else None
        return F.elementwise(s0, o.op, o.alpha, o.beta, s1)
    if o.kind == "tet_jacobian":
        return F.tet_jacobian(src[0].reshape(-1, 4, 3))
    if o.kind == "expr":
        views = []
        for k, s in enumerate(src):
            if k == 0 and o.strides is not None:
                views.append(F.strided_view(s, o.shape, o.strides, o.offset))
            else:
                views.append(s.reshape(o.shape))
        return F.expression(o.expr, views[0], views[1] if len(views) > 1 else None)
    raise ValueError(o.kind)


def oracle_full(w):
    vals = {a: materialize(w, a) for a in w.operands}
    return oracle.batched_einsum(w.notation, w.table, vals)


def oracle_sampled(w, n_samples=2048, seed=0):
    """Sampled output positions per member and the oracle's values there."""
    vals = {a: materialize(w, a) for a in w.operands}
    size = int(np.prod(w.out_shape()))
    rng = np.random.default_rng(seed)
    pos = np.unique(np.concatenate([rng.integers(0, size, n_samples), [0, size - 1]]))
    res = [oracle.einsum_at(w.notation, [vals[a] for a in row], pos) for row in w.table]
    return pos, res


def device_buffers(w, device="cuda"):
    return {k: v.to(device) for k, v in w.buffers.items()}


def run(plan, w, bufs, stream=None):
    dt = {"float32": torch.float32, "float64": torch.float64}[w.dtype]
    outs = [torch.full(w.out_shape(), float("nan"), dtype=dt, device="cuda") for _ in range(w.b)]
    plan.launch(bufs, outs, stream)
    torch.cuda.synchronize()
    return outs


def rel_fro(x, ref):
    x = np.asarray(x, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    den = np.linalg.norm(ref)
    num = np.linalg.norm(x - ref)
    return float(num / den) if den > 0 else float(num)


TOL = {"float64": 1e-12, "float32": 1e-5}
