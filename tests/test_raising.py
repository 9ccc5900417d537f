"""Raising torch.fx programs to functional batched einsums and Algorithm
"IdentifyAsEinsum" (host only: tracing, raising, canonicalization and the
map composition run without a GPU).

The paper's own example is the retrieval listing of Section "Integration ...":
a kernel with substitution rules u = P*P, v = 3 cos(Q) + 5, w = sin(R) and
two sums y1 = u.v, y2 = u.w, identified as the transformation writer's
reference batched einsum 'ij,j->i' with rows (A, B), (A, C).
"""
import pytest
import torch

import workloads
from paper_2601_12220_amd import Context, capi
from paper_2601_12220_amd.raising import compile_fx, identify_as_einsum, raise_fx


def _ops(shapes, dtype="float64"):
    return {k: workloads.Operand(k, tuple(v), dtype, "array", (k,)) for k, v in shapes.items()}


def _paper_kernel(P, Q, R):
    u = P * P
    v = 3 * torch.cos(Q) + 5
    w = torch.sin(R)
    y1 = torch.einsum("ij,j->i", u, v)
    y2 = torch.einsum("ij,j->i", u, w)
    return y1, y2


def _inputs():
    g = torch.Generator().manual_seed(2601_12220 + 990)
    return {"P": torch.randn(96, 4, generator=g, dtype=torch.float64),
            "Q": torch.randn(4, generator=g, dtype=torch.float64),
            "R": torch.randn(4, generator=g, dtype=torch.float64)}


def test_paper_retrieval_listing_raises_to_one_functional_batch(paper_examples):
    gm = torch.fx.symbolic_trace(_paper_kernel)
    batches = raise_fx(gm, _inputs())
    assert len(batches) == 1
    rb = batches[0]
    assert len(rb.table) == 2 and rb.table[0][0] == rb.table[1][0]    # u is shared
    u, v, w = (rb.operands[rb.table[0][0]], rb.operands[rb.table[0][1]],
               rb.operands[rb.table[1][1]])
    assert (u.kind, u.op, u.sources) == ("elementwise", "square", ("P",))
    assert (v.op, v.alpha, v.beta, v.sources) == ("cos", 3.0, 5.0, ("Q",))
    assert (w.op, w.alpha, w.beta, w.sources) == ("sin", 1.0, 0.0, ("R",))


def test_identify_as_the_reference_einsum(paper_examples):
    ref = paper_examples["transform_writer"]
    ctx = Context()
    ref_plan = ctx.register(ref["notation"], ref["table"], _ops(ref["shapes"]))
    rb = raise_fx(torch.fx.symbolic_trace(_paper_kernel), _inputs())[0]
    raised = ctx.register(rb.notation, rb.table, rb.operands)
    assert raised.key == ref_plan.key            # transformation transfers to the kernel
    sigma_a, sigma_i, mm, pm = identify_as_einsum(ref_plan, raised)
    # sigma maps the reference onto the raised einsum: every slot and every
    # index label agrees after substitution
    for i, row in enumerate(ref_plan.table):
        for j, a in enumerate(row):
            assert raised.table[mm[i]][pm[j]] == sigma_a[a]
    ref_ins = ref["notation"].split("->")[0].split(",")
    raised_ins = rb.notation.split("->")[0].split(",")
    for j, labels in enumerate(ref_ins):
        assert "".join(sigma_i[c] for c in labels) == raised_ins[pm[j]]
    assert sigma_a["A"] == rb.table[0][0]        # the shared operand maps to u


def test_identify_refuses_non_isomorphic():
    ctx = Context()
    a = ctx.register("ij,j->i", [["A", "B"], ["A", "C"]],
                     _ops({"A": (96, 4), "B": (4,), "C": (4,)}))
    b = ctx.register("ij,j->i", [["A", "B"], ["D", "C"]],          # nothing shared
                     _ops({"A": (96, 4), "B": (4,), "C": (4,), "D": (96, 4)}))
    with pytest.raises(capi.BesError, match="not isomorphic"):
        identify_as_einsum(a, b)


def _fem_gradient(J, D, u):
    # three einsums of one notation sharing D and u, reading views of J
    return tuple(torch.einsum("er,rij,ej->ei", J[:, x, :], D, u) for x in range(3))


def test_fem_gradient_views_raise_to_the_benchmark_batch():
    w = workloads.config2(e=256)
    ins = {k: w.buffers[k] for k in ("J", "D", "u")}
    rb = raise_fx(torch.fx.symbolic_trace(_fem_gradient), ins)[0]
    assert len(rb.table) == 3
    views = [rb.operands[r[0]] for r in rb.table]
    assert [(v.kind, v.offset, v.strides) for v in views] == \
        [("view", 3 * x, (9, 1)) for x in range(3)]
    ctx = Context()
    assert ctx.register(rb.notation, rb.table, rb.operands).key == \
        ctx.register(w.notation, w.table, w.operands).key


def test_calls_with_renamed_letters_batch_together():
    def f(A, x, y):
        return torch.einsum("ij,j->i", A, x), torch.einsum("ab,b->a", A, y)
    g = torch.Generator().manual_seed(3)
    ins = {"A": torch.randn(40, 8, generator=g, dtype=torch.float64),
           "x": torch.randn(8, generator=g, dtype=torch.float64),
           "y": torch.randn(8, generator=g, dtype=torch.float64)}
    batches = raise_fx(torch.fx.symbolic_trace(f), ins)
    assert len(batches) == 1 and len(batches[0].table) == 2


@pytest.mark.gpu
def test_compiled_fx_runs_batches_on_the_gpu():
    ins = {k: v.cuda() for k, v in _inputs().items()}
    cf = compile_fx(_paper_kernel, ins)
    assert len(cf.batches) == 1
    y1, y2 = cf(**ins)
    torch.cuda.synchronize()
    r1, r2 = _paper_kernel(**{k: v.cpu() for k, v in ins.items()})
    assert torch.allclose(y1.cpu(), r1, rtol=1e-12, atol=1e-12)
    assert torch.allclose(y2.cpu(), r2, rtol=1e-12, atol=1e-12)
    w = workloads.config2(e=1000)
    ins = {k: w.buffers[k].cuda() for k in ("J", "D", "u")}
    cf = compile_fx(_fem_gradient, ins)
    outs = cf(**ins)
    torch.cuda.synchronize()
    refs = _fem_gradient(**{k: v.cpu() for k, v in ins.items()})
    for o, r in zip(outs, refs):
        assert torch.allclose(o.cpu(), r, rtol=1e-11, atol=1e-11)
