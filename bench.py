#!/usr/bin/env python3
"""Benchmark of the pixel-array hot path on one MI355X.

Workload (the JSON line's `value`): the chain system -- 8 binary cubic
relations f_i(x_i, x_{i+1}) = 0 with N(0,1) coefficients, box [-3,3]^9 at 1024
cells per axis, x_1 and x_9 exposed, 7 latent variables (synthetic, seeded).
One step = one whole solve from device-resident coefficient and axis tables
to the device output bits: plotting of all 8 relations (FP32 with FP64
escalation) and the 7 Boolean 1024^3 contractions on int8 MFMA, replayed as
one hipGraph of level-grouped launches with autotuned tiles.

Beside it: the plain GPU path on the same system, the single persistent
launch, the batched workload (512 chains of 2-6 relations at 64..2048 cells
per axis in one graph replay vs one plain solve per system), the learned
contraction order on random relation hypergraphs (model trained on the GPU
from the library's own timings; every policy timed; learned order batched vs
plain), per-kernel durations and the roofline of the dominant kernel (HIP
events around back-to-back launches of each grouped kernel on the execution
stream), and the CPU oracle timed on a bounded sample of the chain workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

INT8_DENSE_PEAK_TOPS = 5000.0      # MI355X dense int8 MFMA, 5.0 POP/s
FP32_VECTOR_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0


def _progress(msg):
    """A progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _time_plan(plan, out, steps, warmup, stream=None):
    import torch
    for _ in range(warmup):
        plan.execute(out, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.execute(out, stream=stream)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def _step_percentiles(plan, out, stream, n):
    """Per-solve durations from an event pair around each graph replay."""
    import numpy as np
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for e0, e1 in evs:
        e0.record(stream)
        plan.execute(out, stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    ms = np.array([e0.elapsed_time(e1) for e0, e1 in evs])
    return {"p10": float(np.percentile(ms, 10)), "p50": float(np.percentile(ms, 50)),
            "p90": float(np.percentile(ms, 90))}


def _plot_flops(system):
    """Algorithmic plotting work: (r+1)^n corners per relation x 4d flop (d FMA
    for the value and d for its error bound)."""
    tot = 0.0
    for rel in system.relations:
        corners = 1
        for v in rel.vars:
            corners *= system.axes[v][2] + 1
        tot += corners * 4.0 * rel.degree
    return tot


TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "c2_chain8_r1024_traffic.json")


def _kernel_source_sha():
    import hashlib
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1609_00061_amd", "csrc", "pa_kernels.hip")
    with open(src, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _measured_traffic():
    """HBM bytes per launch per kernel from the committed FETCH_SIZE /
    WRITE_SIZE counter runs, if they were taken on the current kernel source
    (else {}: traffic is then reported as null)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return {}
    if t.get("kernel_source_sha256") != _kernel_source_sha():
        return {}
    return {k: v["hbm_bytes_per_launch"] for k, v in t.get("kernels", {}).items()}


def _kernel_table(plan, stream, system, reps):
    """Per grouped launch: kind, ms per launch (back-to-back repetitions
    between two events), algorithmic work; and a roofline entry per kind."""
    from paper_1609_00061_amd import pa
    groups = plan.time_groups(reps=reps, stream=stream)
    by = {}
    for kind, ms, macs in groups:
        a = by.setdefault(kind, {"ms": 0.0, "launches": 0, "macs": 0.0})
        a["ms"] += ms
        a["launches"] += 1
        a["macs"] += macs
    roof = {}
    g = by.get(pa.OPKIND_GEMM)
    if g:
        ops = 2.0 * g["macs"] / g["launches"]
        avg = g["ms"] / g["launches"]
        ach = ops / (avg * 1e-3) / 1e12
        roof["gemm"] = {"kernel": "k_group<1> (MFMA Boolean contraction tiles of one tree level)", "bound": "mfma",
                        "achieved": ach, "peak": INT8_DENSE_PEAK_TOPS, "unit": "TOP/s",
                        "frac": ach / INT8_DENSE_PEAK_TOPS, "traffic": None, "avg_launch_ms": avg,
                        "ops_per_launch": ops, "launches_per_step": g["launches"],
                        "ms_per_step": g["ms"]}
    p = by.get(pa.OPKIND_PLOT)
    if p:
        fl = _plot_flops(system) / p["launches"]
        avg = p["ms"] / p["launches"]
        ach = fl / (avg * 1e-3) / 1e12
        roof["plot"] = {"kernel": "k_group<0> (corner plotting of all relations)", "bound": "alu",
                        "achieved": ach, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": ach / FP32_VECTOR_PEAK_TFLOPS, "traffic": None, "avg_launch_ms": avg,
                        "flop_per_launch": fl, "launches_per_step": p["launches"], "ms_per_step": p["ms"]}
    for k, v in _measured_traffic().items():
        if k in roof:
            roof[k]["traffic"] = v
    per_kind = {str(k): {"ms_per_step": v["ms"], "launches_per_step": v["launches"]} for k, v in by.items()}
    return roof, per_kind, groups


def _calibration_copy(mib):
    """A plain device copy of `mib` MiB: FETCH_SIZE / WRITE_SIZE counter runs
    divide by what the counters read for it."""
    if mib <= 0:
        return
    import torch
    src = torch.ones(mib * 262144, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()


def _ternary(stream, steps=10, tuning=None):
    """The ternary workload (4 trivariate cubics over 6 variables at 256
    cells/axis, 2 exposed): solves/s, and per kernel kind the grouped
    launch's rate against its roofline.  Its two 65536 x 65536 x 256-bit
    contractions take sparse plotted operands (about 1% set bits): by
    default a sparse pass computes them (a row gather, HBM-bound: reported
    against HBM with its algorithmic bytes, and its dense-equivalent rate
    separately as effective TOP/s); the same contractions on the MFMA kernel
    (sparse pass off) are timed too and reported against the int8 peak.
    The word-streaming contraction reads both 512 MiB intermediates once."""
    from paper_1609_00061_amd import inputs, pa
    s = inputs.config3()
    if tuning is None:
        tuning, _ = pa.autotune([s], reps=3, stream=stream, order=pa.ORDER_EXHAUSTIVE, graph=True)
    tuning = {k: int(v) for k, v in tuning.items() if k != "ms"}
    plan = pa.Plan(s, order=pa.ORDER_EXHAUSTIVE, graph=True, **tuning)
    out = pa.empty_bits(plan.dims)
    dt = _time_plan(plan, out, steps, 2, stream)
    d = pa.describe_plan(s, order=pa.ORDER_EXHAUSTIVE, **tuning)
    words = [b["words"] for b in d["buffers"]]
    stream_bytes = sum(4.0 * (words[o["a"]] + (words[o["b"]] if o["b"] >= 0 else 0))
                       for o in d["ops"] if o["op"] in ("stream_k", "stream_w"))
    sparse_ops = [o for o in d["ops"] if o["op"] == "sparse_pass"]
    # algorithmic bytes of the sparse pass: every output word written, A and
    # the second plot of B read once
    sparse_bytes = sum(4.0 * (o["rows"] * o["Nw"] + words[o["a"]] + words[o["bt"]]) for o in sparse_ops)
    # the two r^5 contractions' MACs, whichever kernel computes them
    macs = d["total_macs"] - sum(o["macs"] for o in d["ops"] if o["op"] in ("stream_k", "stream_w"))
    kplan = plan
    if tuning.get("single_launch"):
        kplan = pa.Plan(s, order=pa.ORDER_EXHAUSTIVE, graph=True, **dict(tuning, single_launch=0))
        kplan.execute(pa.empty_bits(kplan.dims), stream=stream)
    groups = kplan.time_groups(reps=3, stream=stream)
    res = {"workload": "4 random trivariate cubics over 6 variables, N(0,1) coefficients, [-3,3]^6 at 256 "
                       "cells/axis, 2 exposed", "value": steps / dt, "unit": "solves/s", "ms_per_solve": 1e3 * dt / steps,
           "tuning": tuning}
    sp = [ms for kind, ms, _ in groups if kind == pa.OPKIND_GATHER]
    if sp and sparse_bytes:
        t = sum(sp)
        gbs = sparse_bytes / (t * 1e-3) / 1e9
        res["contraction_sparse"] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                     "frac": gbs / HBM_PEAK_GBS, "ms": t, "algorithmic_bytes": sparse_bytes,
                                     "effective_tops": 2.0 * macs / (t * 1e-3) / 1e12,
                                     "count_ms": sum(ms for kind, ms, _ in groups if kind == pa.OPKIND_COUNT)}
    # the same contractions on the MFMA kernel
    mplan = pa.Plan(s, order=pa.ORDER_EXHAUSTIVE, graph=True, **dict(tuning, sparse_pass=-1, gemm_path=0))
    mout = pa.empty_bits(mplan.dims)
    mdt = _time_plan(mplan, mout, max(2, steps // 2), 1, stream)
    res["mfma_only"] = {"value": max(2, steps // 2) / mdt, "unit": "solves/s",
                        "same_bits": bool((mout == out).all().item())}
    mgroups = mplan.time_groups(reps=3, stream=stream)
    gm = [(ms, macs) for kind, ms, macs in mgroups if kind == pa.OPKIND_GEMM]
    if gm:
        ops = sum(2.0 * m for _, m in gm) / len(gm)
        avg = sum(ms for ms, _ in gm) / len(gm)
        ach = ops / (avg * 1e-3) / 1e12
        res["contraction_mfma"] = {"bound": "mfma", "achieved": ach, "peak": INT8_DENSE_PEAK_TOPS, "unit": "TOP/s",
                                   "frac": ach / INT8_DENSE_PEAK_TOPS, "avg_launch_ms": avg, "launches": len(gm),
                                   "ops_per_launch": ops, "plan": "sparse pass off, default operand path"}
    st = [ms for kind, ms, _ in groups if kind in (pa.OPKIND_STREAM_K, pa.OPKIND_STREAM_W)]
    if st and stream_bytes:
        gbs = stream_bytes / (sum(st) * 1e-3) / 1e9
        res["contraction_stream"] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                     "frac": gbs / HBM_PEAK_GBS, "ms": sum(st), "operand_bytes": stream_bytes}
    return res


def _batched(stream, K, W):
    """512 chains of uneven resolution: one graph replay of the batch (level-
    grouped launches, autotuned tiles) vs the plain path solving each system."""
    import torch
    from paper_1609_00061_amd import inputs, pa
    systems = inputs.config4()
    t0 = time.perf_counter()
    b = pa.Batch(systems, graph=True, autotune=True)
    create_s = time.perf_counter() - t0
    outs = b.alloc_outputs()
    for _ in range(W):
        b.execute(outs, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        b.execute(outs, stream=stream)
    torch.cuda.synchronize()
    bdt = (time.perf_counter() - t0) / K
    plans = [pa.Plan(s, order=pa.ORDER_GREEDY, plain=True) for s in systems]
    pouts = [pa.empty_bits(p.dims) for p in plans]
    for p, o in zip(plans, pouts):
        p.execute(o)
    torch.cuda.synchronize()
    reps = max(1, K // 20)
    t0 = time.perf_counter()
    for _ in range(reps):
        for p, o in zip(plans, pouts):
            p.execute(o)
    torch.cuda.synchronize()
    pdt = (time.perf_counter() - t0) / reps
    same = all(bool(torch.equal(a, c)) for a, c in zip(outs, pouts))
    groups = b.time_groups(reps=5, stream=stream)
    kinds = {}
    for kind, ms, _ in groups:
        kinds[str(kind)] = kinds.get(str(kind), 0.0) + ms
    return {"workload": "512 independent chains of 2-6 binary cubic relations, N(0,1) coefficients, [-3,3], "
                        "per-axis resolution log-uniform in [64, 2048]",
            "value": len(systems) / bdt, "unit": "solves/s", "ms_per_batch": 1e3 * bdt,
            "executor": "one hipGraph replay of level-grouped launches over all systems, autotuned tiles",
            "batch_create_s": create_s,
            "plain_gpu": {"value": len(systems) / pdt, "unit": "solves/s", "ms_per_batch": 1e3 * pdt,
                          "path": "one plain plan per system, greedy order, one launch per plot and step"},
            "speedup_vs_plain": pdt / bdt, "same_bits_as_plain": same, "group_kernel_ms": kinds}


def _learned(stream, n_train=32, n_eval=48, res=128):
    """Random relation hypergraphs (8-14 variables, arity 2-3, 2-4 exposed,
    128 cells/axis): the step-time model trained on the GPU from the
    library's own timings on training graphs, then every policy timed on
    disjoint evaluation graphs (one graph replay per solve), and the learned
    order batched into one replay vs one plain solve per system."""
    import torch
    from paper_1609_00061_amd import inputs, learn, pa
    t0 = time.perf_counter()
    model, X, T = learn.train_order_model(inputs.config5(n_graphs=n_train, index=1000, res=res), rounds=2,
                                         log=_progress)
    train_s = time.perf_counter() - t0
    import numpy as np
    pred = model.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    r2 = float(1.0 - np.mean((pred - T) ** 2) / np.var(T))
    evals = inputs.config5(n_graphs=n_eval, index=0, res=res)
    _progress(f"trained in {train_s:.1f} s on {len(T)} samples; timing policies")
    pol = learn.time_policies(evals, model, policies=("greedy", "exhaustive", "learned", "learned_verified"),
                              steps=3, stream=stream, log=_progress)
    out = {"workload": f"{n_eval} random relation hypergraphs (8-14 variables, arity 2-3, 2-4 exposed, "
                       f"{res} cells/axis, [-3,3]); model trained on {n_train} disjoint graphs",
           "train_s": train_s, "train_samples": int(len(T)), "fit_r2": r2,
           "same_bits_all_policies": pol["same_bits"], "systems": pol["systems"],
           "skipped_enomem": pol["skipped_enomem"]}
    for p in ("greedy", "exhaustive", "learned", "learned_verified"):
        out[p] = {"total_ms": pol[p]["total_ms"], "plan_ms_mean": pol[p]["plan_ms_mean"]}
    out["learned_vs_exhaustive"] = pol["exhaustive"]["total_ms"] / pol["learned"]["total_ms"]
    out["learned_vs_greedy"] = pol["greedy"]["total_ms"] / pol["learned"]["total_ms"]
    out["learned_verified_vs_exhaustive"] = pol["exhaustive"]["total_ms"] / pol["learned_verified"]["total_ms"]
    # learned order + batched graph replay vs the plain path, on the systems
    # every policy could plan
    # (systems whose greedy plan exceeds the workspace, or whose naive cost
    # is beyond 1e12 and would take seconds per plain solve, are left out)
    ok = []
    for s in evals:
        d = pa.describe_plan(s, order=pa.ORDER_GREEDY, plain=True)
        if "error" not in d and d["cost"] <= 1e12:
            ok.append(s)
    out["batched_systems_excluded"] = len(evals) - len(ok)
    try:
        b = pa.Batch(ok, order=pa.ORDER_LEARNED, model=model, graph=True, autotune=True)
        outs = b.alloc_outputs()
        b.execute(outs, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            b.execute(outs, stream=stream)
        torch.cuda.synchronize()
        bdt = (time.perf_counter() - t0) / 3
        plain_ms = []
        for s in ok:
            try:
                p = pa.Plan(s, order=pa.ORDER_GREEDY, plain=True)
            except pa.PaError:       # workspace cap
                plain_ms = None
                break
            o = pa.empty_bits(p.dims)
            p.execute(o)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            p.execute(o)
            torch.cuda.synchronize()
            plain_ms.append(1e3 * (time.perf_counter() - t1))
        out["learned_batched"] = {"value": len(ok) / bdt, "unit": "solves/s", "systems": len(ok)}
        if plain_ms:
            out["plain_gpu"] = {"value": len(ok) / (1e-3 * sum(plain_ms)), "unit": "solves/s",
                                "path": "greedy order, one launch per plot and step, per system"}
            out["speedup_vs_plain"] = out["learned_batched"]["value"] / out["plain_gpu"]["value"]
    except pa.PaError as e:
        out["learned_batched"] = {"error": str(e)}
    return out


def _cpu_baseline(system, budget_s, gpu_bits):
    """The oracle (plain C, pthreads for plotting) solving the same instance:
    corner plots of every relation, then the chain multiplied pairwise."""
    import numpy as np
    import oracle
    res = {v: system.axes[v][2] for v in range(len(system.axes))}
    n = len(system.relations)
    merges = [(0, 1)] + [(n + t, t + 2) for t in range(n - 2)]
    t0 = time.perf_counter()
    solves = 0
    ref = None
    while True:
        plots = [oracle.plot(r, system.axes)[0] for r in system.relations]
        ref = oracle.solve_pairwise(res, [r.vars for r in system.relations], plots, system.exposed, merges)
        solves += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    exact = bool(np.array_equal(ref, gpu_bits))
    return {"value": solves / dt, "unit": "solves/s", "cores": oracle.DEFAULT_THREADS, "kind": "oracle",
            "sample": f"{solves} full solves of the same chain instance ({dt:.1f} s): 8 corner plots at "
                      f"1024^2 ({oracle.DEFAULT_THREADS} threads) + 7 pairwise contractions (1 thread)",
            "bit_exact_vs_gpu": exact}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-ternary", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--ternary-only", action="store_true",
                    help="run only the ternary workload (--steps solves) and print its JSON line (for profiling)")
    ap.add_argument("--tuning", type=str, default="",
                    help="JSON executor settings to use instead of autotuning (e.g. for counter runs, whose "
                         "serialization distorts timings)")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="after the run, copy a buffer of this size 3 times (scales HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              f"(independent systems would shard round-robin across GPUs without communication)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1609_00061_amd import inputs, pa

    torch.cuda.set_device(0)
    system = inputs.config2()
    K, W = args.steps, args.warmup

    stream = torch.cuda.Stream()
    if args.ternary_only:
        _progress("ternary workload")
        given = {k: int(v) for k, v in json.loads(args.tuning).items()} if args.tuning else None
        res = _ternary(stream, steps=K, tuning=given)
        _calibration_copy(args.calibration_copy_mib)
        print(json.dumps(res), flush=True)
        return
    _progress("planning and autotuning the chain workload")
    t0 = time.perf_counter()
    if args.tuning:
        tuning = {k: int(v) for k, v in json.loads(args.tuning).items()}
    else:
        tuning, _ = pa.autotune([system], reps=5, stream=stream, order=pa.ORDER_EXHAUSTIVE, graph=True)
        tuning = {k: int(v) for k, v in tuning.items() if k != "ms"}
    plan = pa.Plan(system, order=pa.ORDER_EXHAUSTIVE, precision=pa.PLOT_FP32_ESCALATE, graph=True, **tuning)
    plan_s = time.perf_counter() - t0
    out = pa.empty_bits(plan.dims)
    dt = _time_plan(plan, out, K, W, stream)
    _, rep, _ = plan.execute(out, stream=stream, report=True)
    gpu_bits = pa.unpack_bits(out.cpu().numpy(), plan.dims)
    pct = _step_percentiles(plan, out, stream, min(K, 200))

    result = {
        "metric": "pixel-array solves/sec + bool-contraction TOPS vs plain GPU path, bit-exact",
        "value": K / dt,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * dt / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8",
        "data": "synthetic",
        "config": {"workload": "chain of 8 binary cubic relations, N(0,1) coefficients (seed 160900061), "
                               "[-3,3]^9 at 1024 cells/axis, x1 and x9 exposed, 7 latent",
                   "plotting": "fp32 + fp64 escalation", "contraction": "int8 MFMA, int32 accumulation, count>0",
                   "order": "exhaustive (balanced tree on cost ties)",
                   "executor": ("one persistent launch per solve, hipGraph replay" if tuning.get("single_launch")
                                else "one grouped launch per tree level and kernel kind, hipGraph replay") +
                               (", tiles " + ("given" if args.tuning else "autotuned")),
                   "global_batch": 1},
        "step_ms_events": pct,
        "plan_and_tune_s": plan_s,
        "tuning": tuning,
        "nnz_out": rep["nnz_out"],
        "escalated_corners": rep["corners_flagged"],
        "corners": rep["corners"],
    }

    _progress(f"timed {K} solves: {1e3 * dt / K:.4f} ms each")
    # per-kernel durations and the roofline of the dominant kernel
    kplan = plan
    if tuning.get("single_launch"):
        # per-launch durations need the grouped executor (same tiles)
        kplan = pa.Plan(system, order=pa.ORDER_EXHAUSTIVE, graph=True, **dict(tuning, single_launch=0))
        kplan.execute(pa.empty_bits(kplan.dims), stream=stream)
    roof, per_kind, _ = _kernel_table(kplan, stream, system, reps=20)
    dom = max(roof.values(), key=lambda r: r["ms_per_step"]) if roof else None
    if dom:
        result["roofline"] = {k: dom[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")}
        result["roofline"]["kernel"] = dom["kernel"]
        result["roofline"]["avg_launch_ms"] = dom["avg_launch_ms"]
    result["roofline_by_kernel"] = roof
    result["group_kernel_ms"] = per_kind
    g = roof.get("gemm")
    if g:
        result["contraction_tops"] = g["achieved"]

    if not args.no_plain:
        _progress("plain path")
        plain = pa.Plan(system, order=pa.ORDER_GREEDY, plain=True)
        pout = pa.empty_bits(plain.dims)
        pdt = _time_plan(plain, pout, K, W)
        torch.cuda.synchronize()
        result["plain_gpu"] = {"value": K / pdt, "unit": "solves/s", "ms_per_step": 1e3 * pdt / K,
                               "path": "greedy order, one plotting launch per relation, one launch per step, "
                                       "no split K, no graph",
                               "same_bits": bool(torch.equal(pout, out))}
        result["speedup_vs_plain"] = (K / dt) / (K / pdt)

    # one persistent launch per solve (tiles wait on dependency counters)
    _progress("single-launch executor")
    splan = pa.Plan(system, order=pa.ORDER_EXHAUSTIVE, graph=True, single_launch=True)
    sout = pa.empty_bits(splan.dims)
    sdt = _time_plan(splan, sout, K, W, stream)
    torch.cuda.synchronize()
    result["single_launch"] = {"value": K / sdt, "unit": "solves/s", "ms_per_step": 1e3 * sdt / K,
                               "same_bits": bool(torch.equal(sout, out))}

    if not args.no_ternary:
        _progress("ternary workload")
        result["ternary"] = _ternary(stream)

    if not args.no_batched:
        _progress("batched workload")
        result["batched"] = _batched(stream, max(5, K // 10), 3)

    if not args.no_learned:
        _progress("learned order")
        result["learned_order"] = _learned(stream)

    if not args.no_cpu_baseline:
        _progress("cpu baseline (oracle)")
        result["cpu_baseline"] = _cpu_baseline(system, args.cpu_budget, gpu_bits)
        result["bit_exact_vs_oracle"] = result["cpu_baseline"]["bit_exact_vs_gpu"]

    _calibration_copy(args.calibration_copy_mib)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
