"""GETT template: binary contractions of any index grouping on the matrix
cores, with affine operands (alpha A + beta) as in Section "TCCG Benchmark
suite with Unmaterialized Operands" (needs an MI355X).

Random TCCG-like contractions (transposed operands and outputs, ragged
edges), degenerate groups (no contracted index, no free index on one side),
several members summed per output, accumulating outputs, and the full-size
stand-in suite on sampled outputs, all against the FP64 oracle (relative
Frobenius <= 1e-12 in FP64, <= 1e-5 in FP32).
"""
import sys

import numpy as np
import pytest
import torch

import workloads
from paper_2601_12220_amd import Context, capi
from tests.gpu_util import TOL, device_buffers, oracle_full, oracle_sampled, rel_fro, run

pytestmark = pytest.mark.gpu
T_GETT = 4


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    return Context()


def _check(plan, w, tol):
    outs = run(plan, w, device_buffers(w))
    ref = oracle_full(w)
    for m in range(w.b):
        err = rel_fro(outs[m].double().cpu().numpy(), ref[m])
        assert err <= tol, (w.notation, m, err)


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("case", range(8))
def test_gett_small_tccg_like(ctx, case, dtype):
    w = workloads.tccg_like(case, dtype=dtype, min_elems=1 << 9, max_elems=1 << 14)
    plan = ctx.register(w.notation, w.table, w.operands)
    plan.set_config(T_GETT, 64, 64)
    _say(f"[gett] {w.notation} {dtype}")
    _check(plan, w, TOL[dtype])


def _op(name, shape, dtype, kind="array", alpha=1.0, beta=0.0, src=None):
    return workloads.Operand(name, tuple(shape), dtype, kind, (src or name,), op="id",
                             alpha=alpha, beta=beta)


def _workload(notation, table, shapes, dtype="float64", affine=()):
    gen = torch.Generator().manual_seed(2601_12220 + 880)
    bufs, ops = {}, {}
    for nm, shp in shapes.items():
        bufs[nm] = torch.randn(*shp, generator=gen, dtype=torch.float64).to(
            torch.float64 if dtype == "float64" else torch.float32)
        if nm in affine:
            ops[nm] = _op(nm, shp, dtype, "elementwise", 1.5, -0.25)
        else:
            ops[nm] = _op(nm, shp, dtype)
    return workloads.Workload("gett_case", notation, table, ops, bufs, dtype)


@pytest.mark.parametrize("notation,shapes", [
    ("abc,cd->adb", {"A": (5, 7, 13), "B": (13, 33)}),       # ragged everywhere
    ("i,j->ij", {"A": (70,), "B": (45,)}),                    # no contracted index
    ("ij,j->i", {"A": (130, 17), "B": (17,)}),                # no free index of B
    ("kji,kl->lij", {"A": (9, 65, 66), "B": (9, 3)}),
])
def test_gett_edge_shapes(ctx, notation, shapes):
    w = _workload(notation, [["A", "B"]], shapes, affine=("A",))
    plan = ctx.register(w.notation, w.table, w.operands)
    plan.set_config(T_GETT, 64, 64)
    _check(plan, w, TOL["float64"])


@pytest.mark.parametrize("ksplit", [1, 3])
def test_gett_members_summed_and_accumulate(ctx, ksplit):
    # two members sharing B; then the same plan accumulating into a
    # pre-filled output through a permuted layout; with K split in ranges
    # whose partial tiles add atomically
    w = _workload("ik,kj->ij", [["A1", "B"], ["A2", "B"]],
                  {"A1": (100, 77), "A2": (100, 77), "B": (77, 70)}, affine=("B",))
    plan = ctx.register(w.notation, w.table, w.operands)
    plan.set_config(T_GETT, 64, 64, ksplit)
    _check(plan, w, TOL["float64"])
    ref = oracle_full(w)
    bufs = device_buffers(w)
    pre = torch.randn(70, 100, dtype=torch.float64, device="cuda")   # stored [j][i]
    out0 = pre.clone()
    out1 = torch.empty(100, 70, dtype=torch.float64, device="cuda")
    capi.bes_plan_set_output(plan.h, 0, 0, [1, 100], True)
    plan.launch(bufs, [out0, out1])
    torch.cuda.synchronize()
    got = (out0 - pre).t().double().cpu().numpy()
    assert rel_fro(got, ref[0]) <= TOL["float64"]
    assert rel_fro(out1.double().cpu().numpy(), ref[1]) <= TOL["float64"]


@pytest.mark.parametrize("case", range(6))
def test_gett_full_size_stand_in_sampled(ctx, case):
    w = workloads.tccg_like(case)
    plan = ctx.register(w.notation, w.table, w.operands)
    _say(f"[gett] full {w.notation} template={plan.template}")
    assert plan.template == "gett"
    outs = run(plan, w, device_buffers(w))
    pos, ref = oracle_sampled(w, n_samples=1024)
    got = outs[0].reshape(-1)[torch.as_tensor(pos, device="cuda")].double().cpu().numpy()
    assert rel_fro(got, ref[0]) <= TOL["float64"]


@pytest.mark.parametrize("shape", [1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("ksplit", [1, 3])
def test_gett_every_tile_shape(ctx, shape, ksplit):
    # each tile shape on ragged operands (rows and columns not multiples of
    # the tile), with and without a K split
    for notation, shapes in (("abc,cd->adb", {"A": (21, 7, 40), "B": (40, 150)}),
                             ("kji,kl->lij", {"A": (37, 13, 11), "B": (37, 290)})):
        w = _workload(notation, [["A", "B"]], shapes, affine=("A", "B"))
        plan = ctx.register(w.notation, w.table, w.operands)
        plan.set_config(T_GETT, 64, 64, ksplit, shape)
        _check(plan, w, TOL["float64"])


@pytest.mark.parametrize("shape", [0, 1, 2, 3, 4, 5, 6, 7])
def test_gett_many_k_ranges_summed_in_a_second_pass(ctx, shape):
    """K split into 64 ranges (partial tiles to the workspace, summed by a
    second kernel): two members summed per output, then the same plan
    accumulating into a pre-filled output through a permuted layout; long
    ragged K, every tile shape."""
    w = _workload("ik,kj->ij", [["A1", "B"], ["A2", "B"]],
                  {"A1": (100, 2011), "A2": (100, 2011), "B": (2011, 70)}, affine=("B",))
    plan = ctx.register(w.notation, w.table, w.operands)
    plan.set_config(T_GETT, 64, 64, 64, shape, 1)
    _check(plan, w, TOL["float64"])
    ref = oracle_full(w)
    bufs = device_buffers(w)
    pre = torch.randn(70, 100, dtype=torch.float64, device="cuda")   # stored [j][i]
    out0 = pre.clone()
    out1 = torch.empty(100, 70, dtype=torch.float64, device="cuda")
    capi.bes_plan_set_output(plan.h, 0, 0, [1, 100], True)
    plan.launch(bufs, [out0, out1])
    torch.cuda.synchronize()
    got = (out0 - pre).t().double().cpu().numpy()
    assert rel_fro(got, ref[0]) <= TOL["float64"]
    assert rel_fro(out1.double().cpu().numpy(), ref[1]) <= TOL["float64"]
