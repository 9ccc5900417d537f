"""Persistent batched launch of many uneven batched einsums, the autotuner and
canonical-key retrieval on the GPU (needs an MI355X).

Workload: random batched einsums with 2-4 operands, 3-6 indices, extents in
{4, 8, 16, 32, 64}, 1-8 members and FP32 N(0,1) data; a quarter of them are
renamed / permuted / re-named-argument copies of earlier ones.  Every output
of the persistent launch (one hipGraph replay) is checked against the FP64
oracle (relative Frobenius <= 1e-5) and against the plain path (one
``bes_launch`` per batched einsum).
"""
import sys

import numpy as np
import pytest
import torch

import workloads
from paper_2601_12220_amd import Batch, Context, capi, tune
from tests.gpu_util import TOL, device_buffers, oracle_full, rel_fro

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _nan_outputs(w):
    return [torch.full(w.out_shape(), float("nan"), dtype=torch.float32, device="cuda")
            for _ in range(w.b)]


@pytest.fixture(scope="module")
def batch_setup(tmp_path_factory):
    ws = workloads.config4(count=32, n_variants=8)
    ctx = Context(str(tmp_path_factory.mktemp("db") / "tuning.db"))
    plans = [ctx.register(w.notation, w.table, w.operands) for w in ws]
    bufs = [device_buffers(w) for w in ws]
    refs = [oracle_full(w) for w in ws]
    return ws, ctx, plans, bufs, refs


def test_tuner_records_are_retrieved_by_variants(batch_setup):
    ws, ctx, plans, bufs, _ = batch_setup
    _say(f"[batch] tuning {len(plans)} plans")
    work = [(p, b, _nan_outputs(w)) for p, b, w in zip(plans, bufs, ws)]
    results, hits = tune.tune_all(ctx, work, reps=3, warmup=1)
    torch.cuda.synchronize()
    variants = [k for k, w in enumerate(ws) if w.info["variant_of"] is not None]
    assert hits >= len(variants)
    for k in variants:
        src = ws[k].info["variant_of"]
        assert plans[k].key == plans[src].key
        assert plans[k].lookup() == capi.BES_OK
        a, b = plans[k].config, plans[src].config
        assert (a.template_id, list(a.p)) == (b.template_id, list(b.p))


def test_persistent_batch_matches_oracle_and_plain(batch_setup):
    ws, ctx, plans, bufs, refs = batch_setup
    _say(f"[batch] persistent launch of {len(plans)} plans")
    batch = Batch(ctx, plans)
    outs_b = [_nan_outputs(w) for w in ws]
    batch.launch(bufs, outs_b)
    outs_p = [_nan_outputs(w) for w in ws]
    for p, b, o in zip(plans, bufs, outs_p):
        p.launch(b, o)
    torch.cuda.synchronize()
    for k, w in enumerate(ws):
        for m in range(w.b):
            got_b = outs_b[k][m].double().cpu().numpy()
            got_p = outs_p[k][m].double().cpu().numpy()
            assert rel_fro(got_b, refs[k][m]) <= TOL["float32"], (w.name, w.notation, m)
            assert rel_fro(got_p, refs[k][m]) <= TOL["float32"], (w.name, w.notation, m)
            # each is within the oracle's FP32 bound: at most twice it apart
            assert rel_fro(got_b, got_p) <= 2 * TOL["float32"], (w.name, m)


def test_graph_replays_with_eager_work_between(batch_setup):
    """Every replay of the captured persistent launch is checked against the
    eager result, with the program's own eager work and synchronizations
    between replays (the counters the launch resets must be zero again)."""
    ws, ctx, plans, bufs, refs = batch_setup
    batch = Batch(ctx, plans)
    eager = [_nan_outputs(w) for w in ws]
    for p, b, o in zip(plans, bufs, eager):
        p.launch(b, o)
    torch.cuda.synchronize()
    outs = [_nan_outputs(w) for w in ws]
    for rep in range(4):
        for os_ in outs:
            for o in os_:
                o.fill_(float("nan"))
        junk = torch.randn(1 << 16, device="cuda").sum()     # unrelated eager work
        batch.launch(bufs, outs)
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for k, w in enumerate(ws):
            for m in range(w.b):
                err = rel_fro(outs[k][m].double().cpu().numpy(),
                              eager[k][m].double().cpu().numpy())
                assert err <= TOL["float32"], (rep, w.name, m, err)


def test_batch_with_new_output_buffers(batch_setup):
    """Pointers may change between launches: the descriptor upload follows."""
    ws, ctx, plans, bufs, refs = batch_setup
    batch = Batch(ctx, plans[:6])
    for rep in range(2):
        outs = [_nan_outputs(w) for w in ws[:6]]
        batch.launch(bufs[:6], outs)
        torch.cuda.synchronize()
        for k in range(6):
            for m in range(ws[k].b):
                assert rel_fro(outs[k][m].double().cpu().numpy(), refs[k][m]) <= TOL["float32"]


# ---------------------------------------------------------------------------
# The batch exactly as the benchmark times it: all 256 batched einsums (64 of
# them renamed / permuted variants), tuned with the benchmark's settings, then
# one persistent replay.  Every output is compared with the FP64 oracle and
# with one plain launch per batched einsum under the same tuned configs
# (including the split configs whose chunks add into zeroed outputs).
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def benched_batch(tmp_path_factory):
    ws = workloads.config4()
    ctx = Context(str(tmp_path_factory.mktemp("db256") / "tuning.db"))
    plans = [ctx.register(w.notation, w.table, w.operands) for w in ws]
    bufs = [device_buffers(w) for w in ws]
    _say(f"[batch256] oracle for {len(ws)} batched einsums")
    refs = [oracle_full(w) for w in ws]
    return ws, ctx, plans, bufs, refs


def test_benched_256_batch_matches_oracle_and_plain(benched_batch):
    ws, ctx, plans, bufs, refs = benched_batch
    assert len(ws) == 256
    stream = torch.cuda.Stream()
    _say("[batch256] tuning as the benchmark does (reps=3, warmup=1)")
    with torch.cuda.stream(stream):
        results, hits = tune.tune_all(ctx, [(p, b, _nan_outputs(w))
                                            for p, b, w in zip(plans, bufs, ws)],
                                      stream=stream, reps=3, warmup=1)
    torch.cuda.synchronize()
    n_var = sum(w.info["variant_of"] is not None for w in ws)
    assert n_var == 64 and hits >= n_var
    splits = sum(1 for p in plans if p.config.template_id == tune.T_GENERIC and p.config.p[2] > 1)
    _say(f"[batch256] {len(results)} tuned records, {hits} retrievals, {splits} split configs")
    batch = Batch(ctx, plans)
    outs_b = [_nan_outputs(w) for w in ws]
    outs_p = [_nan_outputs(w) for w in ws]
    sh = int(stream.cuda_stream)
    srcs = [p.src_ptrs(b) for p, b in zip(plans, bufs)]
    batch.launch_ptrs(srcs, [[o.data_ptr() for o in os_] for os_ in outs_b], sh)
    for p, s, os_ in zip(plans, srcs, outs_p):
        p.launch_ptrs(s, [o.data_ptr() for o in os_], sh)
    torch.cuda.synchronize()
    worst = 0.0
    for k, w in enumerate(ws):
        for m in range(w.b):
            got_b = outs_b[k][m].double().cpu().numpy()
            got_p = outs_p[k][m].double().cpu().numpy()
            eb = rel_fro(got_b, refs[k][m])
            worst = max(worst, eb)
            assert eb <= TOL["float32"], (k, w.notation, m, eb, plans[k].config.p[:3])
            assert rel_fro(got_p, refs[k][m]) <= TOL["float32"], (k, w.notation, m)
            # both are within the FP32 bound of the oracle; split einsums add
            # their chunks atomically in a run-dependent order, so the two
            # FP32 results differ by up to twice that bound
            assert rel_fro(got_b, got_p) <= 2 * TOL["float32"], (k, m)
    _say(f"[batch256] worst relative Frobenius error vs oracle {worst:.3e}")


def test_bind_once_then_replay(batch_setup):
    """bes_batch_bind + bes_batch_replay: pointers bound once, several
    replays, each checked against the oracle; a replay before any bind is
    refused."""
    ws, ctx, plans, bufs, refs = batch_setup
    batch = Batch(ctx, plans[:10])
    with pytest.raises(capi.BesError):
        batch.replay(0)
    outs = [_nan_outputs(w) for w in ws[:10]]
    batch.bind_ptrs([p.src_ptrs(b) for p, b in zip(plans[:10], bufs[:10])],
                    [[o.data_ptr() for o in os_] for os_ in outs], 0)
    for rep in range(3):
        for os_ in outs:
            for o in os_:
                o.fill_(float("nan"))
        batch.replay(0)
        torch.cuda.synchronize()
        for k in range(10):
            for m in range(ws[k].b):
                assert rel_fro(outs[k][m].double().cpu().numpy(), refs[k][m]) <= TOL["float32"]
