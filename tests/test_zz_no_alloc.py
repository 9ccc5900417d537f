"""The launch entry point that allocates nothing (bes_launch_noalloc) against
bes_launch on the same plans and buffers (needs an MI355X).

FEM-stream plans re-lay their shared operand into the library's fixed
per-GPU scratch array; the results must match bes_launch's to the
oracle-parity bar.  Two calls in a row, the second with a smaller input, show
that a call does not depend on what the previous one left in the array.
"""
import sys

import pytest
import torch

import workloads
from paper_2601_12220_amd import Context, capi
from tests.gpu_util import TOL, device_buffers, oracle_full, rel_fro

pytestmark = pytest.mark.gpu

_DT = {"float32": torch.float32, "float64": torch.float64}


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _permuted_s(w):
    """Give the FEM shared operand D[r,i,j] a non-dense layout (stored as
    D'[j,r,i]) so that the launch must re-lay it into the scratch array."""
    D = w.buffers["D"]
    w.buffers["D"] = D.permute(2, 0, 1).contiguous()
    nr, ni, nj = D.shape
    o = w.operands["D"]
    o.kind = "view"
    o.offset = 0
    o.strides = (ni, 1, nr * ni)
    return w


def _both(plan, w, bufs):
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    src = plan.src_ptrs(bufs)
    outs = []
    for fn in (capi.bes_launch, capi.bes_launch_noalloc):
        o = [torch.full(w.out_shape(), float("nan"), dtype=_DT[w.dtype], device="cuda")
             for _ in range(w.b)]
        fn(plan.h, src, [t.data_ptr() for t in o], sh)
        outs.append(o)
    torch.cuda.synchronize()
    return outs


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_noalloc_matches_launch_twice_second_smaller(dtype):
    ctx = Context()
    cases = [_permuted_s(workloads.config2(e=4099, dtype=dtype)),
             _permuted_s(workloads.config2(e=1000, ni=10, dtype=dtype))]
    for w in cases:
        plan = ctx.register(w.notation, w.table, w.operands)
        _say(f"[noalloc] {w.name} e={w.info['e']} ni={w.info['ni']} {dtype} "
             f"template={plan.template}")
        assert plan.template == "fem_stream"
        bufs = device_buffers(w)
        ref_launch, got = _both(plan, w, bufs)
        ref = oracle_full(w)
        for m in range(w.b):
            a = got[m].double().cpu().numpy()
            b = ref_launch[m].double().cpu().numpy()
            assert rel_fro(a, b) <= TOL[dtype], (w.name, m)
            assert rel_fro(a, ref[m]) <= TOL[dtype], (w.name, m)


def test_noalloc_mfma_plan_and_refusals():
    ctx = Context()
    w = workloads.config5(a=16, i=16)
    plan = ctx.register(w.notation, w.table, w.operands)
    assert plan.template == "mfma"
    ref_launch, got = _both(plan, w, device_buffers(w))
    for m in range(w.b):
        assert rel_fro(got[m].double().cpu().numpy(),
                       ref_launch[m].double().cpu().numpy()) <= TOL["float32"]
    # a generic-template plan is refused with a clear error
    g = workloads.config4(count=4, n_variants=0)[0]
    gp = ctx.register(g.notation, g.table, g.operands)
    gp.set_config(2, 256, 1, 1)
    with pytest.raises(capi.BesError, match="FEM-stream and MFMA"):
        capi.bes_launch_noalloc(gp.h, gp.src_ptrs(device_buffers(g)),
                                [0] * g.b, 0)
