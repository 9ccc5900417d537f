"""Expression operands: arbitrary substitution-rule bodies (the "u = P*P,
v = 3 cos(Q) + 5, w = sin(R)" rules of the paper's retrieval listing) compiled
at run time into the generic template.

CPU tests pin the oracle's expression evaluator to values the mathematics
fixes and check the library's body grammar and keys; the GPU tests compare
the run-time built kernels with the oracle.
"""
import math

import numpy as np
import pytest
import torch

import workloads
from oracle import functional as F
from paper_2601_12220_amd import Context, capi
from tests.gpu_util import TOL, device_buffers, oracle_full, rel_fro, run


@pytest.mark.parametrize("body,s0,s1,want", [
    ("3*cos(s0)+5", [0.0, math.pi], None, [8.0, 2.0]),
    ("s0*s0", [3.0, -1.5], None, [9.0, 2.25]),
    ("sin(s0)+s1", [math.pi / 2, 0.0], [0.25, -1.0], [1.25, -1.0]),
    ("exp(-s0*s0)*s1", [0.0, 0.0], [7.0, -2.0], [7.0, -2.0]),
    ("pow(s0, 2) - fabs(s1)", [3.0, 0.5], [-4.0, 1.0], [5.0, -0.75]),
    ("fmax(s0, s1) / 2", [1.0, -3.0], [4.0, -8.0], [2.0, -1.5]),
    ("-(s0) + 2.5e1", [1.0, 25.0], None, [24.0, 0.0]),
])
def test_oracle_expression_known_values(body, s0, s1, want):
    got = F.expression(body, np.array(s0), None if s1 is None else np.array(s1))
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("body", ["s0**2", "__import__('os')", "s0.real", "s2", "abs(s0)",
                                  "[s0]", "s0 if s1 else s1"])
def test_oracle_expression_refuses_other_python(body):
    with pytest.raises((ValueError, SyntaxError)):
        F.expression(body, np.zeros(2))


def _expr_op(name, shape, body, sources, dtype="float64"):
    return workloads.Operand(name, tuple(shape), dtype, "expr", tuple(sources), expr=body)


def _paper_kernel_workload(dtype="float64", bodies=("s0*s0", "3*cos(s0)+5", "sin(s0)")):
    g = torch.Generator().manual_seed(2601_12220 + 991)
    t = torch.float64 if dtype == "float64" else torch.float32
    bufs = {"P": torch.randn(96, 4, generator=g, dtype=torch.float64).to(t),
            "Q": torch.randn(4, generator=g, dtype=torch.float64).to(t),
            "R": torch.randn(4, generator=g, dtype=torch.float64).to(t)}
    ops = {"u": _expr_op("u", (96, 4), bodies[0], ["P"], dtype),
           "v": _expr_op("v", (4,), bodies[1], ["Q"], dtype),
           "w": _expr_op("w", (4,), bodies[2], ["R"], dtype)}
    return workloads.Workload("retrieval_listing", "ij,j->i", [["u", "v"], ["u", "w"]],
                              ops, bufs, dtype)


def test_library_accepts_bodies_and_keeps_them_out_of_the_key():
    ctx = Context()
    w = _paper_kernel_workload()
    p = ctx.register(w.notation, w.table, w.operands)
    assert p.template == "generic"
    arrays = {k: workloads.Operand(k, o.shape, "float64", "array", (k,)) for k, o in
              w.operands.items()}
    assert ctx.register(w.notation, w.table, arrays).key == p.key


@pytest.mark.parametrize("body", ["s0; s1", "s2", "system(s0)", "s0 s1", "(s0", "s0)",
                                  "s0**2", "1e", ".", "sin s0", "", "s0,s1", "{s0}", "s0[0]",
                                  "sin()", "#define x", "s0 +"])
def test_library_rejects_other_text(body):
    ctx = Context()
    w = _paper_kernel_workload(bodies=(body, "s0", "s0"))
    with pytest.raises(capi.BesError):
        ctx.register(w.notation, w.table, w.operands)


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_retrieval_listing_bodies_on_the_gpu(dtype):
    ctx = Context()
    w = _paper_kernel_workload(dtype)
    p = ctx.register(w.notation, w.table, w.operands)
    outs = run(p, w, device_buffers(w))
    ref = oracle_full(w)
    for m in range(2):
        assert rel_fro(outs[m].double().cpu().numpy(), ref[m]) <= TOL[dtype]


@pytest.mark.gpu
@pytest.mark.parametrize("split", [1, 8])
def test_two_source_body_with_view_and_split(split):
    # u[e,j] = exp(-a*a)*b + pow(b,2) where a is a strided view, in a FEM-like
    # batch 'ij,ej->ei'; split > 1 runs the run-time build's zeroing kernel
    ctx = Context()
    g = torch.Generator().manual_seed(2601_12220 + 992)
    e, nj = 1031, 10
    A = torch.randn(e, 2 * nj, generator=g, dtype=torch.float64)
    bufs = {"A": A, "B": torch.randn(e, nj, generator=g, dtype=torch.float64)}
    ops = {"u": workloads.Operand("u", (e, nj), "float64", "expr", ("A", "B"), offset=1,
                                  strides=(2 * nj, 2), expr="exp(-s0*s0)*s1 + pow(s1, 2)")}
    for m in range(3):
        bufs[f"D{m}"] = torch.randn(nj, nj, generator=g, dtype=torch.float64)
        ops[f"D{m}"] = workloads.Operand(f"D{m}", (nj, nj), "float64", "array", (f"D{m}",))
    w = workloads.Workload("expr_fem", "ij,ej->ei", [["D0", "u"], ["D1", "u"], ["D2", "u"]],
                           ops, bufs, "float64")
    p = ctx.register(w.notation, w.table, w.operands)
    p.set_config(2, 256, 4, split)
    outs = run(p, w, device_buffers(w))
    ref = oracle_full(w)
    for m in range(3):
        assert rel_fro(outs[m].double().cpu().numpy(), ref[m]) <= TOL["float64"]
