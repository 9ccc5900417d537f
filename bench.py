"""Benchmark of the batched-einsum hot path on one MI355X.

Headline workload: 3-D FEM operator application (local-gradient class),
``out_x[e,i] = sum_{r,j} J[e,x,r] D[r,i,j] u[e,j]`` for x = 0..2, P3
tetrahedra (i = j = 20, r = 3), e = 2^20 elements, FP64, registered as one
batched einsum 'er,rij,ej->ei' with b = 3 that shares D and u.

A step is one pass of the path for that batch: bind the caller's buffers to
the canonical slots and launch the evaluation (registration -- parse,
induced graph, canonical labeling, key, tuning lookup -- happens once before
the timed region, as the paper does at compile time; its host time is
reported separately).  Inputs are resident in HBM before timing starts.  The
step enqueues two kernels on the caller's stream: a 9.6 KB re-layout of the
shared operand D and the stream kernel; both are inside the timed region.

Prints ONE JSON line.  ``value`` is achieved GB/s on algorithmic bytes (each
distinct source buffer read once, each output written once).  ``extra``
holds the other workloads: FP32, the functional P4 batch, the persistent
launch of 256 uneven batched einsums against one launch per einsum, and the
dense MFMA pair with its adjoint.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
PROFILES = os.path.join(ROOT, "profiles")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(w):
    """Each distinct source buffer read once plus each output written once."""
    item = 8 if w.dtype == "float64" else 4
    used = set()
    for row in w.table:
        for a in row:
            used.update(w.operands[a].sources)
    src = sum(w.buffers[s].numel() for s in used) * item
    out = 1
    for s in w.out_shape():
        out *= s
    return src + w.b * out * item


def fem_flops(w):
    """Factored FLOP count of the FEM-stream evaluation (per launch)."""
    if w.name.startswith("fem_grad_p3"):
        e, ni = w.info["e"], w.info["ni"]
        return e * (2 * 3 * ni * ni + 3 * 2 * 3 * ni)          # T once, 3 members
    if w.name.startswith("fem_grad_functional"):
        e, ni = w.info["e"], w.info["ni"]
        per = 4 * (2 * 3 * ni * ni + 2 * 3 * 3 * ni) + 4 * ni + 9   # + sin adds, V diffs
        return e * per
    return None


def definitional_flops(w):
    """2 x (product of all index extents) per member: the plain loop nest."""
    lhs, _ = w.notation.split("->")
    ext = {}
    for labels, a in zip(lhs.split(","), w.table[0]):
        for ch, s in zip(labels, w.operands[a].shape):
            ext[ch] = s
    space = 1
    for v in ext.values():
        space *= v
    return 2 * space * w.b * max(1, len(lhs.split(",")) - 1)


def fem_kernel_name(cfg, shape):
    """The stream kernel a FEM config runs on the plain P3 batch."""
    if cfg and cfg[0] == 1 and cfg[3] == 0:
        return f"fem_lean_kernel ({shape})"
    return f"fem_stream_kernel, descriptor-driven FAST ({shape})"


def time_launches(fn, steps, warmup, stream):
    """Mean ms per call of fn() between HIP events recorded on ``stream``
    (the stream the kernels are launched on)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps


def kernel_source_digest():
    h = hashlib.sha256()
    for rel in ("paper_2601_12220_amd/csrc/kernels/fem_stream.hip",
                "paper_2601_12220_amd/csrc/fem_shapes.h", "paper_2601_12220_amd/csrc/desc.h"):
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_name):
    """HBM bytes per step from committed rocprofv3 counter runs, if they were
    taken on the current kernel source; else None."""
    path = os.path.join(PROFILES, "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(workload_name)
    if not rec or rec.get("kernel_digest") != kernel_source_digest():
        return None
    return rec.get("bytes_per_launch")


_STREAM = None


def bench_stream():
    """One dedicated HIP stream for every timed launch (torch's default stream
    adds a synchronization point per launch)."""
    global _STREAM
    import torch
    if _STREAM is None:
        _STREAM = torch.cuda.Stream()
    return _STREAM


def run_fem(w, steps, warmup, tune_first=True):
    """Register the batch, tune it (the tuner appends the fastest config to the
    context's database under the canonical key), register it again -- the
    second registration retrieves that record by its key -- and time it."""
    import torch
    from paper_2601_12220_amd import Context, tune
    ctx = Context()
    t0 = time.perf_counter()
    plan = ctx.register(w.notation, w.table, w.operands)
    reg_s = time.perf_counter() - t0
    dt = {"float32": torch.float32, "float64": torch.float64}[w.dtype]
    bufs = {k: v.to("cuda") for k, v in w.buffers.items()}
    outs = [torch.empty(w.out_shape(), dtype=dt, device="cuda") for _ in range(w.b)]
    stream = bench_stream()
    tuned = None
    if tune_first:
        with torch.cuda.stream(stream):
            r = tune.tune(ctx, plan, bufs, outs, stream=stream, reps=30, warmup=3)
        plan = ctx.register(w.notation, w.table, w.operands)     # retrieves the record
        tuned = {"config": list(r.best) if r else None, "retrieved": plan.status}
    src = plan.src_ptrs(bufs)
    optr = [o.data_ptr() for o in outs]
    sh = int(stream.cuda_stream)
    ms = time_launches(lambda: plan.launch_ptrs(src, optr, sh), steps, warmup, stream)
    # The evaluation kernel alone: HIP events recorded by the library around
    # it on this stream, one pair per timed launch.
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
             for _ in range(steps)]
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        for ev0, ev1 in pairs:
            plan.set_timing(ev0, ev1)
            plan.launch_ptrs(src, optr, sh)
    torch.cuda.synchronize()
    plan.set_timing(None, None)
    kernel_ms = sum(a.elapsed_time(b) for a, b in pairs) / steps
    nbytes = algorithmic_bytes(w)
    cfg = plan.config
    res = {"ms": ms, "gbs": nbytes / (ms * 1e-3) / 1e9, "bytes": nbytes,
           "kernel_ms": kernel_ms, "kernel_gbs": nbytes / (kernel_ms * 1e-3) / 1e9,
           "template": plan.template, "register_ms": reg_s * 1e3, "key": plan.key,
           "config": [cfg.template_id] + [int(cfg.p[k]) for k in range(3)], "tuned": tuned}
    fl = fem_flops(w)
    if fl:
        res["tflops"] = fl / (ms * 1e-3) / 1e12
    del bufs, outs
    torch.cuda.empty_cache()
    return res


def run_batch(steps, warmup):
    """256 uneven FP32 batched einsums: one launch per batched einsum with the
    default config, then autotuned (records keyed by canonical form), then
    one persistent hipGraph-captured launch of all of them."""
    import torch
    import workloads
    from paper_2601_12220_amd import Batch, Context, tune
    ws = workloads.config4()
    with tempfile.TemporaryDirectory() as d:
        ctx = Context(os.path.join(d, "tuning.db"))
        t0 = time.perf_counter()
        plans = [ctx.register(w.notation, w.table, w.operands) for w in ws]
        reg_s = time.perf_counter() - t0
        bufs = [{k: v.to("cuda") for k, v in w.buffers.items()} for w in ws]
        outs = [[torch.empty(w.out_shape(), dtype=torch.float32, device="cuda")
                 for _ in range(w.b)] for w in ws]
        srcs = [p.src_ptrs(b) for p, b in zip(plans, bufs)]
        optrs = [[o.data_ptr() for o in os_] for os_ in outs]
        stream = bench_stream()
        sh = int(stream.cuda_stream)

        def plain():
            for p, s, o in zip(plans, srcs, optrs):
                p.launch_ptrs(s, o, sh)
        ms_plain = time_launches(plain, steps, warmup, stream)
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            results, hits = tune.tune_all(ctx, list(zip(plans, bufs, outs)), stream=stream,
                                          reps=3, warmup=1)
        tune_s = time.perf_counter() - t0
        ms_plain_tuned = time_launches(plain, steps, warmup, stream)
        batch = Batch(ctx, plans)
        ms_pers = time_launches(lambda: batch.launch_ptrs(srcs, optrs, sh), steps, warmup,
                                stream)
        n_var = sum(w.info["variant_of"] is not None for w in ws)
        var_hits = sum(1 for k, w in enumerate(ws) if w.info["variant_of"] is not None
                       and plans[k].key == plans[w.info["variant_of"]].key)
        nbytes = sum(algorithmic_bytes(w) for w in ws)
        flops = sum(definitional_flops(w) for w in ws)
        res = {"einsums": len(ws), "ms_plain": round(ms_plain, 4),
               "ms_plain_tuned": round(ms_plain_tuned, 4), "ms_persistent": round(ms_pers, 4),
               "speedup_vs_plain": round(ms_plain / ms_pers, 2),
               "GB/s_persistent": round(nbytes / (ms_pers * 1e-3) / 1e9, 1),
               "GFLOP/s_persistent": round(flops / (ms_pers * 1e-3) / 1e9, 1),
               "tuned_records": len(results), "db_hits": hits,
               "variants": n_var, "variants_sharing_key": var_hits,
               "register_ms_total": round(reg_s * 1e3, 1), "tune_s": round(tune_s, 2)}
        del batch, bufs, outs
    torch.cuda.empty_cache()
    return res


def run_dense(steps, warmup):
    """Dense pair sharing T on MFMA (FP32): forward and autograd backward."""
    import torch
    import workloads
    from paper_2601_12220_amd import Context
    from paper_2601_12220_amd.autograd import BatchedEinsum
    w = workloads.config5()
    ctx = Context()
    be = BatchedEinsum(ctx, w.notation, w.table, w.operands)
    bufs = {k: v.cuda() for k, v in w.buffers.items()}
    stream = bench_stream()
    torch.cuda.synchronize()
    fwd_flops = 2 * 2 * (64 ** 4) * (32 ** 2)          # 2 members x M N K x 2
    with torch.cuda.stream(stream):
        return _run_dense_on(be, bufs, stream, steps, warmup, fwd_flops)


def _run_dense_on(be, bufs, stream, steps, warmup, fwd_flops):
    import torch
    ms_f = time_launches(lambda: be(bufs), steps, warmup, stream)
    leaves = {k: v.clone().requires_grad_(True) for k, v in bufs.items()}
    G = [torch.randn(be.out_shape, device="cuda") for _ in range(2)]

    def fwd_bwd():
        outs = be(leaves)
        torch.autograd.backward(outs, G)
        for t in leaves.values():
            t.grad = None
    ms_fb = time_launches(fwd_bwd, max(20, steps // 2), 2, stream)
    ms_b = max(ms_fb - ms_f, 1e-6)
    res = {"template": be.plan.template, "ms_forward": round(ms_f, 4),
           "TFLOP/s_forward": round(fwd_flops / (ms_f * 1e-3) / 1e12, 1),
           "frac_fp32_peak_forward": round(fwd_flops / (ms_f * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 3),
           "ms_backward": round(ms_b, 4),
           "TFLOP/s_backward": round(2 * fwd_flops / (ms_b * 1e-3) / 1e12, 1)}
    del bufs, leaves
    torch.cuda.empty_cache()
    return res


def cpu_baseline(e_sample, reps=3):
    """The oracle (plain loop nest, FP64) on the headline workload with
    ``e_sample`` elements, timed on the host cores; GB/s on the same
    algorithmic bytes."""
    import oracle
    import workloads
    from tests.gpu_util import materialize
    w = workloads.config2(e=e_sample, dtype="float64")
    vals = {a: materialize(w, a) for a in w.operands}
    oracle.batched_einsum(w.notation, w.table, {a: v[:64] if v.shape[0] == e_sample else v
                                                for a, v in vals.items()})   # warm-up
    t0 = time.perf_counter()
    for _ in range(reps):
        oracle.batched_einsum(w.notation, w.table, vals)
    sec = (time.perf_counter() - t0) / reps
    return {"value": round(algorithmic_bytes(w) / sec / 1e9, 3), "unit": "GB/s",
            "cores": oracle.threads_used(), "kind": "oracle",
            "sample": f"fem_grad_p3 FP64 with e = {e_sample} elements, mean of {reps} "
                      f"evaluations ({sec:.2f} s each)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 20)
    ap.add_argument("--only", default="",
                    help="comma list of extra workloads: f32,p4,batch,dense (default: all)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 5 device-to-device copies of 1 GiB (the known-size "
                         "kernel that scales the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each": a.numel() * 8, "copies": 5}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the batched-einsum "
                                   "path has no multi-GPU mode (DESIGN.md says how it would "
                                   "shard)", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import workloads
    assert torch.cuda.is_available(), "needs a HIP device"
    only = set(args.only.split(",")) if args.only else {"f32", "p4", "batch", "dense"}

    extra = {}
    log("[bench] fem_grad_p3 FP64 e=2^20")
    head = run_fem(workloads.config2(dtype="float64"), args.steps, args.warmup)
    if "f32" in only:
        log("[bench] fem_grad_p3 FP32 e=2^20")
        r = run_fem(workloads.config2(dtype="float32"), args.steps, args.warmup)
        extra["fem_grad_p3_f32"] = {"GB/s": round(r["gbs"], 1), "ms": round(r["ms"], 5),
                                    "frac_hbm": round(r["gbs"] / HBM_PEAK_GBS, 4),
                                    "kernel_GB/s": round(r["kernel_gbs"], 1),
                                    "template": r["template"], "tuned_config": r["config"]}
    if "p4" in only:
        log("[bench] fem_grad_functional_p4 FP64 e=2^19")
        r = run_fem(workloads.config3(), max(5, args.steps // 5), 2)
        extra["fem_grad_functional_p4_f64"] = {
            "GB/s": round(r["gbs"], 1), "ms": round(r["ms"], 5),
            "frac_hbm": round(r["gbs"] / HBM_PEAK_GBS, 4),
            "kernel_GB/s": round(r["kernel_gbs"], 1),
            "TFLOP/s": round(r.get("tflops", 0.0), 2), "template": r["template"],
            "tuned_config": r["config"]}
    if "batch" in only:
        log("[bench] persistent batch of 256 uneven batched einsums (FP32)")
        extra["persistent_batch_256"] = run_batch(max(5, args.steps // 5), 2)
    if "dense" in only:
        log("[bench] dense pair sharing T on MFMA (FP32) + adjoint")
        extra["dense_pair_mfma"] = run_dense(max(4, args.steps // 5), 2)

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        cpu = cpu_baseline(args.cpu_sample)

    traffic = measured_traffic("fem_grad_p3_f64")
    line = {
        "metric": "batched-einsum GB/s & %HBM roofline; persistent/adjoint vs plain speedup",
        "value": round(head["gbs"], 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded; FEM-shaped: affine Jacobians, reference derivative "
                "matrix U[-1,1], N(0,1) fields)",
        "config": {"workload": "fem_grad_p3: 'er,rij,ej->ei', b=3, e=2^20, i=j=20, r=3, "
                               "shared D and u", "elements": 1 << 20,
                   "template": head["template"], "register_ms": round(head["register_ms"], 3),
                   "tuned_config": head["config"]},
        "roofline": {"bound": "hbm", "achieved": round(head["kernel_gbs"], 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(head["kernel_gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": fem_kernel_name(head["config"], "FP64, i=j=20, r=3, 3 members"),
                     "kernel_us": round(head["kernel_ms"] * 1e3, 2)},
        "cpu_baseline": cpu,
        "extra": dict(extra, fem_grad_p3_f64_tflops=round(head.get("tflops", 0.0), 2)),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
