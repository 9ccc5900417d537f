"""GPU parity of the evaluation path against the FP64 oracle (needs an MI355X).

Bar: relative Frobenius error per output <= 1e-12 (FP64) and <= 1e-5 (FP32).
Small cases are compared element by element over the whole output (sizes that
span many blocks plus a ragged tail); full-size cases on sampled outputs the
oracle computes one by one.
"""
import random
import sys

import numpy as np
import pytest
import torch

import workloads
from paper_2601_12220_amd import Context, capi
from tests.gpu_util import TOL, device_buffers, oracle_full, oracle_sampled, rel_fro, run

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    return Context()


def _check_full(plan, w, tmpl=None):
    _say(f"[parity] {w.name} dtype={w.dtype} template={plan.template} out={w.out_shape()}")
    bufs = device_buffers(w)
    outs = run(plan, w, bufs)
    ref = oracle_full(w)
    for m in range(w.b):
        err = rel_fro(outs[m].double().cpu().numpy(), ref[m])
        assert err <= TOL[w.dtype], (w.name, m, err)


def _check_sampled(plan, w):
    _say(f"[parity-sampled] {w.name} dtype={w.dtype} template={plan.template} out={w.out_shape()}")
    bufs = device_buffers(w)
    outs = run(plan, w, bufs)
    pos, ref = oracle_sampled(w)
    for m in range(w.b):
        got = outs[m].reshape(-1)[torch.as_tensor(pos, device="cuda")].double().cpu().numpy()
        err = rel_fro(got, ref[m])
        assert err <= TOL[w.dtype], (w.name, m, err)
        assert torch.isfinite(outs[m]).all()


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_config1(ctx, dtype):
    w = workloads.config1(dtype=dtype)
    p = ctx.register(w.notation, w.table, w.operands)
    assert p.template == "fem_stream"
    _check_full(p, w)
    p.set_config(capi.BES_T_GENERIC, 256, 1)
    _check_full(p, w)


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("e", [1, 63, 4099, 70001])
def test_config2_small(ctx, dtype, e):
    w = workloads.config2(e=e, dtype=dtype)
    p = ctx.register(w.notation, w.table, w.operands)
    # the stream index must be the largest extent for the FEM-stream template
    assert p.template == ("fem_stream" if e > 20 else "generic")
    _check_full(p, w)


def test_config2_generic_template(ctx):
    w = workloads.config2(e=1000)
    p = ctx.register(w.notation, w.table, w.operands)
    for lanes in (1, 4, 16):
        p.set_config(capi.BES_T_GENERIC, 128, lanes)
        _check_full(p, w)


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_config2_full_size(ctx, dtype):
    w = workloads.config2(dtype=dtype)
    p = ctx.register(w.notation, w.table, w.operands)
    _check_sampled(p, w)


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_config2_full_size_whole_output_every_candidate(ctx, dtype):
    """The P3 gradient batch at full size (e = 2^20), every output element
    against the oracle, in every FEM-stream configuration the tuner may
    record for it (the launch the benchmark times is one of them)."""
    from paper_2601_12220_amd import tune
    w = workloads.config2(dtype=dtype)
    p = ctx.register(w.notation, w.table, w.operands)
    assert p.template == "fem_stream"
    bufs = device_buffers(w)
    ref = oracle_full(w)
    tdt = torch.float64 if dtype == "float64" else torch.float32
    outs = [torch.empty(w.out_shape(), dtype=tdt, device="cuda") for _ in range(w.b)]
    for cand in tune.candidates(capi.BES_T_FEM_STREAM):
        _say(f"[parity-full] {w.name} {dtype} config={cand}")
        for o in outs:
            o.fill_(float("nan"))
        p.set_config(*cand)
        p.launch(bufs, outs)
        torch.cuda.synchronize()
        for m in range(w.b):
            err = rel_fro(outs[m].double().cpu().numpy(), ref[m])
            assert err <= TOL[dtype], (cand, m, err)


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("bpc", [1, 64])
def test_config2_kernel_variants(ctx, dtype, variant, bpc):
    """The lean kernel with two waves per tile (variant 0) and one (2), the
    descriptor-driven one (1) and the FP32 matrix-core one (3; FP64 falls
    back to the lean kernel), on the P3 gradient batch with a ragged tail;
    one block per CU makes every block walk several tiles."""
    w = workloads.config2(e=64 * 1093 + 29, dtype=dtype)
    p = ctx.register(w.notation, w.table, w.operands)
    p.set_config(capi.BES_T_FEM_STREAM, 64, bpc, variant)
    _check_full(p, w)


def _tet_one_member(ni, e, dt):
    """'rij,exr,ej->exi' with one member: G the tetrahedron Jacobian of V,
    u a plain array."""
    bufs = {"V": workloads._uniform(12, 0, (e, 4, 3), 0.0, 1.0, dt),
            "D": workloads._uniform(12, 1, (3, ni, ni), -1.0, 1.0, dt),
            "u": workloads._normal(12, 2, (e, ni), dt)}
    ops = {"D": workloads._dense("D", bufs["D"], dt), "u": workloads._dense("u", bufs["u"], dt),
           "J": workloads.Operand("J", (e, 3, 3), dt, "tet_jacobian", ("V",))}
    return workloads.Workload(f"tet_one_p{ni}", "rij,exr,ej->exi", [["D", "J", "u"]], ops, bufs,
                              dt, {"e": e, "ni": ni})


@pytest.mark.parametrize("case", ["p3_views", "p4_views", "p2_views", "p1_views", "p4_tet",
                                  "p2_tet"])
@pytest.mark.parametrize("bpc", [1, 64])
def test_fp32_matrix_core_variant(ctx, case, bpc):
    """The FP32 matrix-core variant (p[2] = 3): three members reading views
    of one Jacobian row (the P3 gradient batch at P1..P4 extents) and one
    member reading a tetrahedron Jacobian, ragged tails; one block per CU
    makes every wave walk several 16-element units."""
    e = 64 * 523 + 45
    ni = {"p1": 4, "p2": 10, "p3": 20, "p4": 35}[case[:2]]
    if case.endswith("views"):
        w = workloads.config2(e=e, ni=ni, dtype="float32")
    else:
        w = _tet_one_member(ni, e, "float32")
    p = ctx.register(w.notation, w.table, w.operands)
    assert p.template == "fem_stream"
    p.set_config(capi.BES_T_FEM_STREAM, 64, bpc, 3)
    _check_full(p, w)


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_lean_kernel_one_member_and_without_g(ctx, dtype):
    """The lean kernel's other instantiations: a batch of one member (no
    shared stage 1) and members without a per-element G."""
    w2 = workloads.config2(e=64 * 70 + 7, dtype=dtype)
    one = workloads.Workload("fem_grad_b1", w2.notation, [list(w2.table[1])],
                             {k: w2.operands[k] for k in ("J1", "D", "u")}, w2.buffers,
                             dtype, w2.info)
    e, nj = 64 * 70 + 7, 20
    bufs = {"u": workloads._normal(90, 0, (e, nj), dtype),
            "D": workloads._uniform(90, 1, (nj, nj), -1.0, 1.0, dtype)}
    ops = {k: workloads._dense(k, v, dtype) for k, v in bufs.items()}
    no_g = workloads.Workload("fem_matvec_shared", "ij,ej->ei", [["D", "u"], ["D", "u"]],
                              ops, bufs, dtype, {"e": e, "nj": nj})
    for w in (one, no_g):
        p = ctx.register(w.notation, w.table, w.operands)
        assert p.template == "fem_stream"
        for variant in (0, 1, 2, 3):
            p.set_config(capi.BES_T_FEM_STREAM, 64, 16, variant)
            _check_full(p, w)


@pytest.mark.parametrize("e", [5, 2049, 30011])
def test_config3_small(ctx, e):
    w = workloads.config3(e=e)
    p = ctx.register(w.notation, w.table, w.operands)
    assert p.template == ("fem_stream" if e > 35 else "generic")
    _check_full(p, w)


@pytest.mark.parametrize("op", ["sin", "cos"])
def test_functional_trig_ranges(ctx, op):
    """The P4 prologue's two trigonometric paths: the short reduction for
    waves whose arguments all stay below 2^20 in magnitude and the library
    routine for a wave holding a larger one (tile 3 gets |a| up to 1e9),
    for sin and cos, against the oracle."""
    import dataclasses
    w = workloads.config3(e=64 * 8 + 5)
    a0 = w.buffers["a0"].clone()
    a0[3 * 64 + 7, 11] = 1.0e9
    a0[3 * 64 + 40, :] *= 3.0e6
    a0[5 * 64:6 * 64, :] *= 40.0                     # |a| in the hundreds
    bufs = dict(w.buffers, a0=a0)
    ops = {k: (dataclasses.replace(v, op=op) if v.kind == "elementwise" else v)
           for k, v in w.operands.items()}
    w2 = workloads.Workload(w.name + "_" + op, w.notation, w.table, ops, bufs, w.dtype, w.info)
    p = ctx.register(w2.notation, w2.table, w2.operands)
    assert p.template == "fem_stream"
    _check_full(p, w2)


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("bpc", [8, 64])
def test_config3_matrix_core_mappings(ctx, variant, bpc):
    """The functional P4 batch on both matrix-core mappings ((r, i) on the M
    side: variant 0; i on the N side: variant 1) with a ragged tail, each
    wave walking several 16-element units and all four members."""
    w = workloads.config3(e=64 * 1093 + 29)
    p = ctx.register(w.notation, w.table, w.operands)
    assert p.template == "fem_stream"
    p.set_config(capi.BES_T_FEM_STREAM, 64, bpc, variant)
    _check_full(p, w)


@pytest.mark.parametrize("nx", [3, 1])
@pytest.mark.parametrize("variant,dt", [(0, "float64"), (1, "float64"), (3, "float32"),
                                        (0, "float32")])
def test_p4_matrix_core_plain_operands(ctx, nx, variant, dt):
    """P4 gradient batches whose operands are plain arrays (no element-wise
    prologue), with G[e, x, r] and with G[e, r] (x absent): FP64 on both
    matrix-core mappings, FP32 on its matrix-core variant (3) and on the
    default path; ragged tail."""
    e = 64 * 301 + 17
    gshape = (e, 3, 3) if nx == 3 else (e, 3)
    bufs = {"D": workloads._uniform(11, 0, (3, 35, 35), -1.0, 1.0, dt),
            "G": workloads._normal(11, 1, gshape, dt)}
    ops = {k: workloads._dense(k, v, dt) for k, v in bufs.items()}
    table = []
    for k in range(3):
        bufs[f"u{k}"] = workloads._normal(11, 2 + k, (e, 35), dt)
        ops[f"u{k}"] = workloads._dense(f"u{k}", bufs[f"u{k}"], dt)
        table.append(["D", "G", f"u{k}"])
    nota = "rij,exr,ej->exi" if nx == 3 else "rij,er,ej->ei"
    w = workloads.Workload(f"p4_plain_x{nx}", nota, table, ops, bufs, dt, {"e": e})
    p = ctx.register(w.notation, w.table, w.operands)
    assert p.template == "fem_stream"
    p.set_config(capi.BES_T_FEM_STREAM, 64, 16, variant)
    _check_full(p, w)


@pytest.mark.parametrize("mix", ["one_source", "one_and_two", "plain_and_two", "plain_and_one"])
@pytest.mark.parametrize("variant", [0, 1])
def test_p4_matrix_core_operand_mixes(ctx, mix, variant):
    """The P4 batch with its members' u in different forms: element-wise
    with one source (alpha*sin(a)+beta), mixed with two-source ones, and
    mixed with plain arrays -- the kernel's per-group prologue and the
    launcher's choice between the matrix-core mappings -- ragged tail."""
    import dataclasses
    w = workloads.config3(e=64 * 301 + 17)
    ops = dict(w.operands)
    for k in range(4):
        u = ops[f"u{k}"]
        one = dataclasses.replace(u, sources=(f"a{k}",), alpha=0.75, beta=-0.25)
        plain = workloads._dense(f"a{k}", w.buffers[f"a{k}"], w.dtype)
        if mix == "one_source" or (mix in ("one_and_two", "plain_and_one") and k >= 2):
            ops[f"u{k}"] = one
        if mix.startswith("plain") and k == 0:
            ops[f"u{k}"] = dataclasses.replace(plain, name="u0")
    w2 = workloads.Workload(w.name + "_" + mix, w.notation, w.table, ops, w.buffers, w.dtype,
                            w.info)
    p = ctx.register(w2.notation, w2.table, w2.operands)
    assert p.template == "fem_stream"
    p.set_config(capi.BES_T_FEM_STREAM, 64, 16, variant)
    _check_full(p, w2)


def test_config3_full_size(ctx):
    w = workloads.config3()
    p = ctx.register(w.notation, w.table, w.operands)
    _check_sampled(p, w)


def test_config3_generic_template(ctx):
    w = workloads.config3(e=777)
    p = ctx.register(w.notation, w.table, w.operands)
    p.set_config(capi.BES_T_GENERIC, 256, 1)
    _check_full(p, w)


def _permuted(w, seed):
    """A renamed, member- and position-permuted registration of w with the
    same buffers: the outputs must land in the right places."""
    rng = random.Random(seed)
    nota, table, shapes, _ = workloads.spec_structure(w)
    nn, nt, ns, pi, pj, imap, amap = workloads.variant_of(rng, nota, table, shapes, "z")
    ops = {}
    for old, new in amap.items():
        o = w.operands[old]
        ops[new] = workloads.Operand(new, o.shape, o.dtype, o.kind, o.sources, o.offset,
                                     o.strides, o.op, o.alpha, o.beta)
    v = workloads.Workload(w.name + "_variant", nn, nt, ops, w.buffers, w.dtype)
    return v, pi


@pytest.mark.parametrize("maker", [lambda: workloads.config2(e=3001),
                                   lambda: workloads.config3(e=1501),
                                   lambda: workloads.config1()])
def test_variants_bind_to_the_right_outputs(ctx, maker):
    w = maker()
    base = ctx.register(w.notation, w.table, w.operands)
    for seed in range(3):
        v, pi = _permuted(w, seed)
        p = ctx.register(v.notation, v.table, v.operands)
        assert p.key == base.key and p.template == base.template
        _check_full(p, v)


def test_empty_stream_and_determinism(ctx):
    w = workloads.config2(e=0)
    p = ctx.register(w.notation, w.table, w.operands)
    bufs = device_buffers(w)
    outs = [torch.empty(w.out_shape(), dtype=torch.float64, device="cuda") for _ in range(3)]
    p.launch(bufs, outs)
    torch.cuda.synchronize()
    w = workloads.config3(e=4097)
    p = ctx.register(w.notation, w.table, w.operands)
    bufs = device_buffers(w)
    a = run(p, w, bufs)
    b = run(p, w, bufs)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_functional_retrieval_listing(ctx, paper_examples):
    # Listing 'Computational scientist's view': u = P*P, v = 3 cos(Q) + 5,
    # w = sin(R), fused where read; checked against the oracle.
    from paper_2601_12220_amd import make_operand
    n0, n1 = 96, 4
    g = torch.Generator().manual_seed(5)
    P = torch.randn(n0, n1, generator=g, dtype=torch.float64)
    Q = torch.randn(n1, generator=g, dtype=torch.float64)
    R = torch.randn(n1, generator=g, dtype=torch.float64)
    ops = {"U": (make_operand((n0, n1), kind="elementwise", op="square"), ["P"]),
           "V": (make_operand((n1,), kind="elementwise", op="cos", alpha=3.0, beta=5.0), ["Q"]),
           "W": (make_operand((n1,), kind="elementwise", op="sin"), ["R"])}
    p = ctx.register("ij,j->i", [["U", "V"], ["U", "W"]], ops, arg_order=["U", "V", "W"])
    bufs = {"P": P.cuda(), "Q": Q.cuda(), "R": R.cuda()}
    outs = [torch.empty(n0, dtype=torch.float64, device="cuda") for _ in range(2)]
    p.launch(bufs, outs)
    torch.cuda.synchronize()
    pp = (P * P).numpy()
    y1 = (pp * (3 * np.cos(Q.numpy()) + 5)).sum(1)
    y2 = (pp * np.sin(R.numpy())).sum(1)
    assert rel_fro(outs[0].cpu().numpy(), y1) <= 1e-12
    assert rel_fro(outs[1].cpu().numpy(), y2) <= 1e-12


@pytest.mark.parametrize("nota,shapes", [
    ("ij,ij->", [(37, 5), (37, 5)]),
    ("ii,i->i", [(33, 33), (33,)]),
    ("ab,bc,cd->ad", [(7, 0), (0, 5), (5, 3)]),
    ("abc,cb->a", [(300, 17, 9), (9, 17)]),
])
def test_generic_edge_cases(ctx, nota, shapes):
    import oracle
    from paper_2601_12220_amd import make_operand
    g = torch.Generator().manual_seed(9)
    arrs = [torch.randn(*s, generator=g, dtype=torch.float64) for s in shapes]
    names = [f"X{k}" for k in range(len(shapes))]
    ops = {nm: (make_operand(s), [nm]) for nm, s in zip(names, shapes)}
    p = ctx.register(nota, [names], ops, arg_order=names)
    assert p.template == "generic"
    ref = oracle.einsum(nota, *[a.numpy() for a in arrs])
    out = torch.full(ref.shape, float("nan"), dtype=torch.float64, device="cuda")
    p.launch({nm: a.cuda() for nm, a in zip(names, arrs)}, [out])
    torch.cuda.synchronize()
    assert rel_fro(out.cpu().numpy(), ref) <= 1e-12


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("split", [1, 8, 64])
def test_generic_factored_and_split(ctx, dtype, split):
    """Few outputs, long contraction: indices carried by one operand only are
    summed inside it, the shared space is split into chunks that add into the
    zeroed outputs (two members, one sharing an argument)."""
    import oracle
    from paper_2601_12220_amd import make_operand
    nota = "vh,fht,ftv,hfv->v"
    shapes = [(16, 12), (9, 12, 7), (9, 7, 16), (12, 9, 16)]
    g = torch.Generator().manual_seed(77)
    names = ["A", "B", "C", "D", "E"]
    arrs = {nm: torch.randn(*(shapes[k] if k < 4 else shapes[3]), generator=g, dtype=torch.float64)
            for k, nm in enumerate(names)}
    if dtype == "float32":
        arrs = {k: v.float().double() for k, v in arrs.items()}    # FP32-exact inputs
    tdt = torch.float64 if dtype == "float64" else torch.float32
    ops = {nm: (make_operand(tuple(arrs[nm].shape), dtype), [nm]) for nm in names}
    table = [["A", "B", "C", "D"], ["A", "B", "C", "E"]]
    p = ctx.register(nota, table, ops, arg_order=names)
    p.set_config(capi.BES_T_GENERIC, 4, 16, split)
    refs = [oracle.einsum(nota, *[arrs[a].numpy() for a in row]) for row in table]
    outs = [torch.full(refs[0].shape, float("nan"), dtype=tdt, device="cuda") for _ in range(2)]
    for rep in range(2):          # twice: the zeroing of split outputs must repeat
        p.launch({k: v.to(tdt).cuda() for k, v in arrs.items()}, outs)
        torch.cuda.synchronize()
        for m in range(2):
            assert rel_fro(outs[m].double().cpu().numpy(), refs[m]) <= TOL[dtype], (split, m, rep)


@pytest.mark.parametrize("nota", ["ank,qfi,n->i", "ij,ij->i"])
@pytest.mark.parametrize("lanes", [1, 2, 8, 64])
def test_generic_fp32_ill_conditioned_sum_any_lanes(ctx, nota, lanes):
    """FP32 sums whose terms cancel to about 1/1000 of their absolute sum: the
    generic template carries sums in FP64 and rounds the result once, so
    every split of the sum across an output's lanes stays within a few FP32
    roundings of the oracle (1e-6, far inside the 1e-5 bound that naive FP32
    summation of such sums can miss).  In 'ank,qfi,n->i' the cancelling sum
    belongs to the operand without shared indices (summed once per output,
    dealt out across the lanes); in 'ij,ij->i' to the shared rows."""
    import oracle
    from paper_2601_12220_amd import make_operand
    g = torch.Generator().manual_seed(1234)
    if nota == "ank,qfi,n->i":
        shapes = [(4, 8, 4), (32, 32, 8), (8,)]
        x = torch.randn(32, 32, 8, generator=g, dtype=torch.float64)
        arrs = [torch.randn(4, 8, 4, generator=g, dtype=torch.float64),
                x - x.mean(dim=(0, 1), keepdim=True) + 1e-3,
                torch.randn(8, generator=g, dtype=torch.float64)]
    else:
        shapes = [(16, 2048), (16, 2048)]
        x = torch.randn(16, 2048, generator=g, dtype=torch.float64)
        arrs = [x - x.mean(dim=1, keepdim=True) + 1e-3, torch.ones(16, 2048, dtype=torch.float64)]
    arrs = [a.float().double() for a in arrs]         # FP32-exact inputs
    names = [f"X{k}" for k in range(len(shapes))]
    ops = {nm: (make_operand(s, "float32"), [nm]) for nm, s in zip(names, shapes)}
    p = ctx.register(nota, [names], ops, arg_order=names)
    p.set_config(capi.BES_T_GENERIC, 64, lanes, 1)
    ref = oracle.einsum(nota, *[a.numpy() for a in arrs])
    out = torch.full(ref.shape, float("nan"), dtype=torch.float32, device="cuda")
    p.launch({nm: a.float().cuda() for nm, a in zip(names, arrs)}, [out])
    torch.cuda.synchronize()
    err = rel_fro(out.double().cpu().numpy(), ref)
    assert err <= 1e-6, (nota, lanes, err)
