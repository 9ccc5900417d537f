"""Dense contraction pair sharing T on MFMA, and its hand-written adjoint.

'abij,cdab->cdij' with rows (T, V) and (T, W'), W'[c,d,a,b] = W[a,b,c,d] a
permuted view.  Forward and backward are compared with the FP64 oracle (the
backward with the oracle's definitional gradient); the FP64 4^6 instance is
checked against central finite differences with torch.autograd.gradcheck.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2601_12220_amd import Context
from paper_2601_12220_amd.autograd import BatchedEinsum
from tests.gpu_util import TOL, device_buffers, materialize, oracle_full, oracle_sampled, rel_fro, run

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    return Context()


def test_dense_pair_small_full_parity(ctx):
    w = workloads.config5(a=16, i=16)        # M = N = K = 256: MFMA tiles
    p = ctx.register(w.notation, w.table, w.operands)
    _say(f"[dense] small template={p.template}")
    assert p.template == "mfma"
    outs = run(p, w, device_buffers(w))
    ref = oracle_full(w)
    for m in range(2):
        assert rel_fro(outs[m].double().cpu().numpy(), ref[m]) <= TOL["float32"]


def test_dense_pair_full_size_forward(ctx):
    w = workloads.config5()
    p = ctx.register(w.notation, w.table, w.operands)
    _say(f"[dense] full template={p.template} key={p.key}")
    assert p.template == "mfma"
    outs = run(p, w, device_buffers(w))
    pos, ref = oracle_sampled(w, n_samples=1024)
    for m in range(2):
        got = outs[m].reshape(-1)[torch.as_tensor(pos, device="cuda")].double().cpu().numpy()
        assert rel_fro(got, ref[m]) <= TOL["float32"]


def _grad_samples(be, bufs, G, rng, n=512):
    """Oracle gradient entries of <G, R> for T, V and W at sampled positions."""
    vals = {a: materialize(be._w, a) for a in be._w.operands}
    g = [x.double().cpu().numpy() for x in G]
    nota = be.notation
    out = {}
    T, V, Wp = vals["T"], vals["V"], vals["Wp"]
    pos = rng.integers(0, T.size, n)
    out["T"] = (pos, oracle.einsum_grad_at(nota, [T, V], g[0], 0, pos) +
                oracle.einsum_grad_at(nota, [T, Wp], g[1], 0, pos))
    pos = rng.integers(0, V.size, n)
    out["V"] = (pos, oracle.einsum_grad_at(nota, [T, V], g[0], 1, pos))
    # W[a,b,c,d] = W'[c,d,a,b]: a flat W position maps to a W' position
    a_ = be._w.info["a"]
    posW = rng.integers(0, V.size, n)
    ia, ib, ic, id_ = np.unravel_index(posW, (a_, a_, a_, a_))
    posWp = np.ravel_multi_index((ic, id_, ia, ib), (a_, a_, a_, a_))
    out["W"] = (posW, oracle.einsum_grad_at(nota, [T, Wp], g[1], 1, posWp))
    return out


def test_dense_pair_full_size_adjoint(ctx):
    w = workloads.config5()
    be = BatchedEinsum(ctx, w.notation, w.table, w.operands)
    be._w = w
    _say(f"[adjoint] pos0 key={be.adjoint(0).key} template={be.adjoint(0).template}")
    _say(f"[adjoint] pos1 key={be.adjoint(1).key} template={be.adjoint(1).template}")
    assert be.adjoint(0).template == "mfma" and be.adjoint(1).template == "mfma"
    bufs = {k: v.cuda().requires_grad_(True) for k, v in w.buffers.items()}
    outs = be(bufs)
    gen = torch.Generator().manual_seed(2601_12220 + 505)
    G = [torch.randn(o.shape, generator=gen, dtype=torch.float64).float().cuda() for o in outs]
    loss = sum((o * g).sum() for o, g in zip(outs, G))
    loss.backward()
    torch.cuda.synchronize()
    samples = _grad_samples(be, bufs, G, np.random.default_rng(3))
    for name, (pos, ref) in samples.items():
        got = bufs[name].grad.reshape(-1)[torch.as_tensor(pos, device="cuda")].double().cpu().numpy()
        err = rel_fro(got, ref)
        _say(f"[adjoint] d{name} rel_fro={err:.2e}")
        assert err <= TOL["float32"], (name, err)


def test_adjoint_gradcheck_fp64_4pow6(ctx):
    # all extents 4, FP64: central finite differences (torch.autograd.gradcheck)
    w = workloads.config5(a=4, i=4, dtype="float64")
    be = BatchedEinsum(ctx, w.notation, w.table, w.operands)
    T = w.buffers["T"].cuda().requires_grad_(True)
    V = w.buffers["V"].cuda().requires_grad_(True)
    W = w.buffers["W"].cuda().requires_grad_(True)

    def f(T, V, W):
        return tuple(be({"T": T, "V": V, "W": W}))

    assert torch.autograd.gradcheck(f, (T, V, W), eps=1e-6, atol=1e-8, rtol=1e-6)
    # and against the oracle's definitional gradient, every entry
    outs = f(T, V, W)
    gen = torch.Generator().manual_seed(7)
    G = [torch.randn(o.shape, generator=gen, dtype=torch.float64).cuda() for o in outs]
    gT, gV, gW = torch.autograd.grad(outs, (T, V, W), G)
    Tn, Vn, Wn = (x.detach().cpu().numpy() for x in (T, V, W))
    Wp = Wn.transpose(2, 3, 0, 1)
    g = [x.cpu().numpy() for x in G]
    n = w.notation
    refT = oracle.einsum_grad(n, [Tn, Vn], g[0], 0) + oracle.einsum_grad(n, [Tn, Wp], g[1], 0)
    refV = oracle.einsum_grad(n, [Tn, Vn], g[0], 1)
    refW = oracle.einsum_grad(n, [Tn, Wp], g[1], 1).transpose(2, 3, 0, 1)
    for got, ref in ((gT, refT), (gV, refV), (gW, refW)):
        assert rel_fro(got.cpu().numpy(), ref) <= 1e-12


def test_fem_adjoint_matches_oracle(ctx):
    # the adjoint of the FEM gradient batch w.r.t. the shared field u and the
    # per-member Jacobian views (generic template; J views scatter into J)
    w = workloads.config2(e=513)
    be = BatchedEinsum(ctx, w.notation, w.table, w.operands)
    bufs = {k: v.cuda().requires_grad_(True) for k, v in w.buffers.items()}
    outs = be(bufs)
    gen = torch.Generator().manual_seed(11)
    G = [torch.randn(o.shape, generator=gen, dtype=torch.float64).cuda() for o in outs]
    gJ, gD, gu = torch.autograd.grad(outs, (bufs["J"], bufs["D"], bufs["u"]), G)
    J = w.buffers["J"].numpy()
    D = w.buffers["D"].numpy()
    u = w.buffers["u"].numpy()
    g = [x.cpu().numpy() for x in G]
    n = w.notation
    refJ = np.zeros_like(J)
    refD = np.zeros_like(D)
    refu = np.zeros_like(u)
    for x in range(3):
        ops = [J[:, x, :], D, u]
        refJ[:, x, :] = oracle.einsum_grad(n, ops, g[x], 0)
        refD += oracle.einsum_grad(n, ops, g[x], 1)
        refu += oracle.einsum_grad(n, ops, g[x], 2)
    for got, ref in ((gJ, refJ), (gD, refD), (gu, refu)):
        assert rel_fro(got.cpu().numpy(), ref) <= 1e-12


# ---------------------------------------------------------------------------
# Gradient sums and view scatters inside the library: a buffer read at two
# operand positions (the second adjoint adds into what the first wrote), a
# view covering part of its buffer (zeroed gradient, then added into), and
# views of one buffer that overlap inside one adjoint launch (atomic adds).
# ---------------------------------------------------------------------------

def _op(name, shape, dtype, kind="array", src=None, offset=0, strides=None):
    return workloads.Operand(name, tuple(shape), dtype, kind, (src or name,),
                             offset=offset, strides=strides)


def _oracle_grads(notation, table, operands, vals, G, buffers):
    """d<G, R>/d(buffer) from the oracle's definitional gradient, scattered
    through each argument's view (numpy, FP64)."""
    out = {b: np.zeros(buffers[b].numel()) for b in buffers}
    for i, row in enumerate(table):
        for pos, a in enumerate(row):
            o = operands[a]
            g = oracle.einsum_grad(notation, [vals[x] for x in row], G[i], pos)
            if o.kind == "view":
                idx = np.full((), o.offset, dtype=np.int64)
                for ext, st in zip(o.shape, o.strides):
                    idx = np.add.outer(idx, np.arange(ext) * st)
                np.add.at(out[o.sources[0]], idx.ravel(), g.ravel())
            else:
                out[o.sources[0]] += g.ravel()
    return out


@pytest.mark.parametrize("case", ["square_AA_mfma", "square_AA_fp64", "partial_view",
                                  "overlapping_views"])
def test_gradient_sums_and_scatters_in_library(ctx, case):
    gen = torch.Generator().manual_seed(2601_12220 + 900)
    if case.startswith("square_AA"):
        # R = A A (A at both positions): dA = G A^T + A^T G
        dt = "float32" if case.endswith("mfma") else "float64"
        n = 128 if dt == "float32" else 24
        bufs = {"A": torch.randn(n, n, generator=gen, dtype=torch.float64).to(
            torch.float32 if dt == "float32" else torch.float64)}
        operands = {"A": _op("A", (n, n), dt)}
        notation, table = "ik,kj->ij", [["A", "A"]]
    elif case == "partial_view":
        # two members read disjoint row blocks of X that leave rows uncovered
        dt = "float64"
        bufs = {"X": torch.randn(40, 6, generator=gen, dtype=torch.float64),
                "B": torch.randn(6, 5, generator=gen, dtype=torch.float64)}
        operands = {"X0": _op("X0", (8, 6), dt, "view", "X", 0, (6, 1)),
                    "X1": _op("X1", (8, 6), dt, "view", "X", 12 * 6, (6, 1)),
                    "B": _op("B", (6, 5), dt)}
        notation, table = "ik,kj->ij", [["X0", "B"], ["X1", "B"]]
    else:
        # overlapping views of one buffer at one position: one adjoint launch
        # adds both slots into the same memory
        dt = "float64"
        bufs = {"X": torch.randn(30, 4, generator=gen, dtype=torch.float64),
                "B": torch.randn(4, 7, generator=gen, dtype=torch.float64)}
        operands = {"X0": _op("X0", (20, 4), dt, "view", "X", 0, (4, 1)),
                    "X1": _op("X1", (20, 4), dt, "view", "X", 5 * 4, (4, 1)),
                    "B": _op("B", (4, 7), dt)}
        notation, table = "ik,kj->ij", [["X0", "B"], ["X1", "B"]]
    be = BatchedEinsum(ctx, notation, table, operands)
    _say(f"[grad-sum] {case}: adjoint templates "
         f"{[be.adjoint(p).template for p in range(2)]}")
    leaves = {k: v.cuda().requires_grad_(True) for k, v in bufs.items()}
    outs = be(leaves)
    G = [torch.randn(o.shape, generator=gen, dtype=torch.float64).to(o.dtype).cuda()
         for o in outs]
    grads = torch.autograd.grad(outs, [leaves[k] for k in sorted(leaves)], G)
    torch.cuda.synchronize()
    vals = {a: (F_view(bufs[o.sources[0]].double().numpy(), o)) for a, o in operands.items()}
    ref = _oracle_grads(notation, table, operands, vals,
                        [g.double().cpu().numpy() for g in G], bufs)
    tol = TOL[dt]
    for k, g in zip(sorted(leaves), grads):
        err = rel_fro(g.double().cpu().numpy().ravel(), ref[k])
        _say(f"[grad-sum] {case} d{k} rel_fro={err:.2e}")
        assert err <= tol, (case, k, err)


def F_view(buf, o):
    from oracle import functional as F
    if o.kind == "view":
        return F.strided_view(buf.ravel(), o.shape, o.strides, o.offset)
    return buf.reshape(o.shape)
