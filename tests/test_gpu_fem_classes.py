"""Face mass and local divergence on the FEM-stream template's apply class
(needs an MI355X).

The two other DG-FEM classes of Section "Batched einsums in DG-FEM
Operators", at P1..P4 with ragged element counts and several members, are
compared element by element with the FP64 oracle (relative Frobenius
<= 1e-12 in FP64, <= 1e-5 in FP32); the paper's size (e = 10^5) on sampled
outputs; a functional streamed field sin(a) + b; and a registration with the
operands in another order, which must retrieve the same canonical key.
"""
import sys

import numpy as np
import pytest
import torch

import workloads
from paper_2601_12220_amd import Context
from tests.gpu_util import TOL, device_buffers, oracle_full, oracle_sampled, rel_fro, run

pytestmark = pytest.mark.gpu

CLASSES = {"face": workloads.face_mass, "div": workloads.local_divergence}


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    return Context()


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("cls", ["face", "div"])
def test_apply_class_parity_ragged(ctx, cls, p, dtype):
    w = CLASSES[cls](p=p, e=1000 + 37, b=3, dtype=dtype)
    plan = ctx.register(w.notation, w.table, w.operands)
    _say(f"[apply] {w.name} {dtype} e=1037 b=3 template={plan.template}")
    assert plan.template == "fem_stream"
    outs = run(plan, w, device_buffers(w))
    ref = oracle_full(w)
    for m in range(w.b):
        err = rel_fro(outs[m].double().cpu().numpy(), ref[m])
        assert err <= TOL[dtype], (w.name, m, err)


@pytest.mark.parametrize("p", [3, 4])
@pytest.mark.parametrize("cls", ["face", "div"])
def test_apply_class_paper_size_sampled(ctx, cls, p):
    w = CLASSES[cls](p=p, e=100_000, b=4)
    plan = ctx.register(w.notation, w.table, w.operands)
    _say(f"[apply] {w.name} e=1e5 b=4 template={plan.template}")
    outs = run(plan, w, device_buffers(w))
    pos, ref = oracle_sampled(w, n_samples=2048)
    idx = torch.as_tensor(pos, device="cuda")
    for m in range(w.b):
        got = outs[m].reshape(-1)[idx].double().cpu().numpy()
        assert rel_fro(got, ref[m]) <= TOL["float64"], (w.name, m)


def test_apply_class_functional_field(ctx):
    # F_k = sin(a_k) + b_k evaluated while staging, never materialized
    w = workloads.face_mass(p=3, e=777, b=2)
    for k in range(2):
        a = workloads._normal(6, 40 + k, (4, 777, 10), "float64")
        w.buffers[f"a{k}"] = a
        w.buffers[f"b{k}"] = w.buffers.pop(f"F{k}")
        w.operands[f"F{k}"] = workloads.Operand(f"F{k}", (4, 777, 10), "float64",
                                                "elementwise", (f"a{k}", f"b{k}"), op="sin")
    plan = ctx.register(w.notation, w.table, w.operands)
    assert plan.template == "fem_stream"
    outs = run(plan, w, device_buffers(w))
    ref = oracle_full(w)
    for m in range(2):
        assert rel_fro(outs[m].double().cpu().numpy(), ref[m]) <= TOL["float64"]


def test_apply_class_reordered_registration(ctx):
    # the same batch with operands listed (U, G, S) and indices renamed:
    # one canonical key, and the binding still routes every slot correctly
    w = workloads.local_divergence(p=2, e=515, b=2)
    plan = ctx.register(w.notation, w.table, w.operands)
    v = workloads.local_divergence(p=2, e=515, b=2)
    v.notation = "aeb,ace,cfb->ef"     # (U[x,e,j], J[x,r,e], D[r,i,j]) renamed
    v.table = [[r[2], r[0], r[1]] for r in v.table][::-1]
    vplan = ctx.register(v.notation, v.table, v.operands)
    assert vplan.key == plan.key and vplan.template == "fem_stream"
    outs = run(vplan, v, device_buffers(v))
    ref = oracle_full(v)
    for m in range(2):
        assert rel_fro(outs[m].double().cpu().numpy(), ref[m]) <= TOL["float64"]


@pytest.mark.parametrize("bpc", [1, 16])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("cls", ["face", "div"])
def test_apply_class_matrix_core(ctx, cls, p, bpc):
    """The FP64 matrix-core variant (p[2] = 3) at P1..P4: a ragged element
    count (a partial 16-element unit) and a multiple of 16, three members;
    one block per CU makes every wave walk several units."""
    from paper_2601_12220_amd import capi
    for e in (1000 + 37, 16 * 211):
        w = CLASSES[cls](p=p, e=e, b=3)
        plan = ctx.register(w.notation, w.table, w.operands)
        assert plan.template == "fem_stream"
        plan.set_config(capi.BES_T_FEM_STREAM, 64, bpc, 3)
        _say(f"[apply-mfma] {w.name} e={e} b=3 bpc={bpc}")
        outs = run(plan, w, device_buffers(w))
        ref = oracle_full(w)
        for m in range(w.b):
            err = rel_fro(outs[m].double().cpu().numpy(), ref[m])
            assert err <= TOL["float64"], (w.name, e, m, err)


@pytest.mark.parametrize("cls", ["face", "div"])
def test_apply_class_matrix_core_paper_size_and_fallbacks(ctx, cls):
    """Variant 3 at the paper's size (e = 10^5, P4, b = 8) on sampled
    outputs, and the batches it leaves to the other kernels: FP32 and a
    functional streamed field."""
    import dataclasses
    from paper_2601_12220_amd import capi
    w = CLASSES[cls](p=4, e=100_000, b=8)
    plan = ctx.register(w.notation, w.table, w.operands)
    plan.set_config(capi.BES_T_FEM_STREAM, 64, 8, 3)
    _say(f"[apply-mfma] {w.name} e=1e5 b=8")
    outs = run(plan, w, device_buffers(w))
    pos, ref = oracle_sampled(w, n_samples=2048)
    idx = torch.as_tensor(pos, device="cuda")
    for m in range(w.b):
        got = outs[m].reshape(-1)[idx].double().cpu().numpy()
        assert rel_fro(got, ref[m]) <= TOL["float64"], (w.name, m)
    w32 = CLASSES[cls](p=3, e=1037, b=2, dtype="float32")
    plan = ctx.register(w32.notation, w32.table, w32.operands)
    plan.set_config(capi.BES_T_FEM_STREAM, 64, 8, 3)
    outs = run(plan, w32, device_buffers(w32))
    ref = oracle_full(w32)
    for m in range(w32.b):
        assert rel_fro(outs[m].double().cpu().numpy(), ref[m]) <= TOL["float32"]
    wf = CLASSES[cls](p=3, e=1037, b=2)
    bufs = dict(wf.buffers)
    ops = dict(wf.operands)
    for k in range(wf.b):
        field = f"F{k}" if cls == "face" else f"U{k}"
        bufs[f"B{k}"] = torch.randn(bufs[field].shape, dtype=torch.float64,
                                    generator=torch.Generator().manual_seed(5 + k))
        ops[field] = dataclasses.replace(ops[field], kind="elementwise",
                                         sources=(field, f"B{k}"), op="sin")
    wf = workloads.Workload(wf.name + "_fn", wf.notation, wf.table, ops, bufs, wf.dtype, wf.info)
    plan = ctx.register(wf.notation, wf.table, wf.operands)
    plan.set_config(capi.BES_T_FEM_STREAM, 64, 8, 3)
    outs = run(plan, wf, device_buffers(wf))
    ref = oracle_full(wf)
    for m in range(wf.b):
        assert rel_fro(outs[m].double().cpu().numpy(), ref[m]) <= TOL["float64"]
