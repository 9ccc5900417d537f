"""Autotuner for batched-einsum plans.

The paper retrieves transformation choices for a batched einsum from a
database of performance facts keyed by its canonical form (Section
"Integration with a Code Transformation Framework"; the retrieval listing
there).  This module produces those facts on the GPU: it times every
candidate configuration of a plan's kernel template through the C ABI with
HIP events on the launching stream and appends the fastest one to the
context's tuning database under the plan's canonical key.  Because the key is
the canonical form, every renamed, permuted or re-shared registration of the
same batched einsum retrieves the same record (``Plan.lookup``).

Only the timing loop runs here; every evaluation is the library's own kernel.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

from . import capi

T_FEM_STREAM = 1
T_GENERIC = 2
T_MFMA = 3
T_GETT = 4


def candidates(template_id: int) -> List[Tuple[int, ...]]:
    """Parameter tuples (template id first) the tuner tries for a template.

    FEM stream: p[1] = blocks per compute unit in the grid, p[2] = kernel
                variant (0 lean with two waves per tile, 2 lean with one,
                1 descriptor-driven, 3 matrix cores: FP32 gradient class,
                FP64 face-mass / divergence class; as 0 elsewhere).
    Generic:    p[0] = outputs per tile, p[1] = lanes per output, p[2] = chunks
                of the shared contracted space (their sums add into the output).
    MFMA:       the single 128 x 128 tile shape the template implements.
    GETT:       p[2] = K ranges per output tile, p[3] = tile shape, p[4] = 1
                partial tiles of >= 8 ranges summed by a second kernel."""
    if template_id == T_FEM_STREAM:
        return [(T_FEM_STREAM, 64, b, v) for v in (0, 2, 1, 3) for b in (4, 8, 16, 32, 64)]
    if template_id == T_GENERIC:
        # p[2]: chunks of the shared contracted space per output (1: none)
        return ([(T_GENERIC, tile, lanes, 1) for tile in (64, 256, 1024) for lanes in (1, 4, 16, 64)]
                + [(T_GENERIC, 256, lanes, split) for lanes in (16, 64) for split in (8, 64)])
    if template_id == T_MFMA:
        return [(T_MFMA, 128, 128)]
    if template_id == T_GETT:   # p[2]: K ranges per tile (0: launcher's), p[3]: tile shape,
        # p[4] = 1: partial tiles of >= 8 ranges summed by a second kernel
        return ([(T_GETT, 64, 64, ks, 0) for ks in (0, 1, 4, 16, 64, 256)] +
                [(T_GETT, 64, 64, ks, sh) for sh in (1, 2, 3, 4, 5, 6, 7) for ks in (0, 256)] +
                [(T_GETT, 64, 64, ks, sh, 1) for sh in (0, 1, 2, 3, 4, 5) for ks in (64, 256)])
    return []


@dataclass
class TuneResult:
    key: str
    best: Tuple[int, ...]
    seconds: float
    timings: Dict[Tuple[int, ...], float] = field(default_factory=dict)


def time_launches(launch, stream, reps: int, warmup: int) -> float:
    """Mean seconds per call of ``launch(handle)`` on ``stream`` (a torch
    stream): after ``warmup`` eager calls (which also make every allocation
    a first launch needs), ``reps`` calls are captured in one HIP graph and
    the graph is replayed between HIP events, so host launch overhead does
    not blur the differences between candidates of short kernels."""
    import torch
    h = int(stream.cuda_stream)
    for _ in range(warmup):
        launch(h)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        hh = int(torch.cuda.current_stream().cuda_stream)
        for _ in range(reps):
            launch(hh)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        g.replay()
        start.record(stream)
        g.replay()
        end.record(stream)
    end.synchronize()
    del g
    return start.elapsed_time(end) * 1e-3 / reps


def tune(ctx, plan, buffers: Dict[str, object], outputs: Sequence[object], stream=None,
         reps: int = 20, warmup: int = 3, arch: str = "gfx950",
         record: bool = True, rounds: int = 1) -> Optional[TuneResult]:
    """Time every candidate of the plan's current template on ``buffers`` /
    ``outputs`` (device tensors), install the fastest in the plan and, with
    ``record``, append it to the context's database.  Returns None when the
    template has nothing to tune."""
    import torch
    stream = stream if stream is not None else torch.cuda.current_stream()
    if stream == torch.cuda.default_stream():
        # graphs are not captured on the legacy default stream: time on a
        # side stream, after everything queued so far has finished
        torch.cuda.synchronize()
        stream = torch.cuda.Stream()
    cands = candidates(plan.config.template_id)
    if not cands:
        return None
    src = plan.src_ptrs(buffers)
    outs = [o.data_ptr() for o in outputs]
    timings: Dict[Tuple[int, ...], float] = {}
    # every candidate is timed in `rounds` interleaved rounds and keeps its
    # best round, so that a transient slowdown of the device during one
    # candidate's turn does not decide the choice
    for _ in range(rounds):
        for c in cands:
            try:
                plan.set_config(*c)
            except capi.BesError:
                continue                      # the template rejects this shape
            t = time_launches(lambda h: plan.launch_ptrs(src, outs, h), stream, reps, warmup)
            timings[c] = min(t, timings.get(c, t))
    if not timings:
        return None
    best = min(timings, key=timings.get)
    plan.set_config(*best)
    if record:
        cfg = capi.bes_config()
        cfg.template_id = best[0]
        for k, v in enumerate(best[1:]):
            cfg.p[k] = int(v)
        ctx.record(plan.key, cfg, timings[best], arch)
    return TuneResult(plan.key, best, timings[best], timings)


def tune_all(ctx, work: Sequence[Tuple[object, Dict[str, object], Sequence[object]]],
             stream=None, reps: int = 10, warmup: int = 2,
             arch: str = "gfx950") -> Tuple[List[TuneResult], int]:
    """Tune a list of (plan, buffers, outputs).  A plan whose canonical key
    already has a record (an isomorphic plan tuned earlier in the list, or a
    previous session's database) is not re-tuned: it retrieves the record.
    Returns the new results and the number of retrievals."""
    results: List[TuneResult] = []
    hits = 0
    for plan, bufs, outs in work:
        if plan.lookup(arch) == capi.BES_OK:
            hits += 1
            continue
        r = tune(ctx, plan, bufs, outs, stream=stream, reps=reps, warmup=warmup, arch=arch)
        if r is not None:
            results.append(r)
    return results, hits
