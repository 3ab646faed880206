#!/usr/bin/env python3
"""Benchmark of the pixel-array hot path on one MI355X.

Workload (the JSON line's `value`): the ternary system -- 4 random
trivariate cubic relations over 6 variables, R1(v1,v2,v3) R2(v3,v4,v5)
R3(v5,v6,v1) R4(v2,v4,v6), N(0,1) coefficients (seed 160900061), box
[-3,3]^6 at 256 cells per axis, (v1, v4) exposed, 4 latent variables
(synthetic, seeded).  One step = one whole solve from device-resident
coefficient and axis tables to the device output bits: FP32 corner plotting
with FP64 escalation of all relations, the two 65536 x 65536 x 256-bit
Boolean contractions and the word-streamed contraction of both 512 MiB
intermediates, replayed as one hipGraph of level-grouped launches with
autotuned tiles.

Beside it: the same system on the plain GPU path and on the MFMA kernel
alone, the solve rate with host planning included, the roofline of every
grouped kernel (HIP events around back-to-back launches on the execution
stream), the chain system (8 binary cubics at 1024 cells per axis) with its
own roofline and its single persistent launch, the batch of 512 uneven
chains, the learned contraction order on 256 random hypergraphs, FP32/FP64
escalation and disagreement counts per workload (audit mode), the CPU
oracle timed on the host cores, and the paper's own timing quoted with its
hardware.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP4_DENSE_PEAK_TOPS = 10100.0      # MI355X dense fp4 MFMA, 10.1 PFLOP/s (the Boolean contraction's MFMA type)
INT8_DENSE_PEAK_TOPS = 5000.0      # MI355X dense int8 MFMA, 5.0 POP/s (for comparison only)
FP32_VECTOR_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0
# LDS read bandwidth: 64 banks of 4 bytes per CU, 256 bytes per clock (a
# 16-lane pass of 16-byte reads per clock), 256 CUs at 2.4 GHz; the fused
# step's roofline also reports the rate pa.lds_read_rate() measures
LDS_PEAK_GBS = 256 * 256 * 2.4
METRIC = "pixel-array solves/sec + bool-contraction TOPS vs plain GPU path, bit-exact"
TERNARY = ("4 random trivariate cubics over 6 variables (every pair sharing one), N(0,1) coefficients "
           "(seed 160900061), [-3,3]^6 at 256 cells/axis, (v1, v4) exposed, 4 latent")
CHAIN = ("chain of 8 binary cubic relations, N(0,1) coefficients (seed 160900061), [-3,3]^9 at 1024 "
         "cells/axis, x1 and x9 exposed, 7 latent")
PAPER_CONTEXT = {
    "what": "the paper's only timing: the whole pixel array method in Julia on its transcendental 'butterfly' "
            "system at resolution 50 per variable, about 1.5 s, against Julia's NLsolve (one Newton solve per "
            "pixel centre) which did not finish in more than 3 hours (over 7,200x); Mathematica's NSolve fails "
            "on the system",
    "hardware": "'a Dell laptop' (CPU model, cores and threads not stated)",
    "note": "context only: a different system, method variant and machine; not a target",
}


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


def _plot_flops(system, rel_ids=None):
    """Algorithmic plotting work: (r+1)^n corners per relation x 4d flop (d FMA
    for the value and d for its error bound)."""
    tot = 0.0
    for i, rel in enumerate(system.relations):
        if rel_ids is not None and i not in rel_ids:
            continue
        corners = 1
        for v in rel.vars:
            corners *= system.axes[v][2] + 1
        tot += corners * 4.0 * rel.degree
    return tot


def _kernel_source_sha():
    src = os.path.join(ROOT, "paper_1609_00061_amd", "csrc", "pa_kernels.hip")
    with open(src, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _measured_traffic(name):
    """HBM bytes per launch per kernel from a committed FETCH_SIZE / WRITE_SIZE
    counter summary, if it was taken on the current kernel source (else {}:
    traffic is then reported as null)."""
    try:
        with open(os.path.join(ROOT, "profiles", name)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return {}
    if t.get("kernel_source_sha256") != _kernel_source_sha():
        return {}
    return {k: v["hbm_bytes_per_launch"] for k, v in t.get("kernels", {}).items()}


def _set_bits(system, rel):
    """Set cells of a relation's plot (on the device; counted with a byte
    table on the host)."""
    import numpy as np
    from paper_1609_00061_amd import pa
    r = system.relations[rel]
    t, dims, _ = pa.plot_relation(r, [system.axes[v] for v in r.vars])
    table = np.array([bin(i).count("1") for i in range(256)], dtype=np.int64)
    return int(table[t.cpu().numpy().view(np.uint8)].sum())


def _work_of(system, d):
    """Algorithmic work per op of a plan description: bytes for the HBM-bound
    kernels (streamed operands; sparse-pass output words written plus A and the
    second plot of B read once; row lists: A read, heads and meta words
    written), Boolean ops (2 per MAC) for MFMA contractions, and for a fused
    pass pair the LDS bytes it gathers (one 256-byte row per set bit of an A
    row and 8-wide block of the other output variable)."""
    words = [b["words"] for b in d["buffers"]]
    out = {"stream_bytes": 0.0, "sparse_bytes": 0.0, "gemm_ops": 0.0, "sparse_macs": 0.0, "list_bytes": 0.0,
           "fused_lds_bytes": 0.0, "fused_macs": 0.0}
    rel_of_buf = {p["buf"]: p["rel"] for p in d["plots"]}
    lists = [o for o in d["ops"] if o["op"] == "row_list"]
    for o in d["ops"]:
        if o["op"] == "row_list":
            groups = o["rows"] // 8
            # A read; per list row its 8-entry head (16 bytes), per group its
            # meta word written
            out["list_bytes"] += 4.0 * (words[o["a"]] + groups * (8 * 4 + 1))
        elif o["op"] == "fused_pass_pair":
            lx = [l for l in lists if l["c"] == o["lists"] and l["lbase"] == 0][0]
            ly = [l for l in lists if l["c"] == o["lists"] and l["lbase"] == o["kx"]][0]
            bx, by = _set_bits(system, rel_of_buf[lx["a"]]), _set_bits(system, rel_of_buf[ly["a"]])
            out["fused_lds_bytes"] += 256.0 * (bx * ((o["n_p"] + 7) // 8) + by * ((o["n_q"] + 7) // 8))
            out["fused_macs"] += o["dense_macs"]
        if o["op"] in ("stream_k", "stream_w"):
            out["stream_bytes"] += 4.0 * (words[o["a"]] + (words[o["b"]] if o["b"] >= 0 else 0))
        elif o["op"] == "sparse_pass":
            out["sparse_bytes"] += 4.0 * (o["rows"] * o["Nw"] + words[o["a"]] + words[o["bt"]])
            out["sparse_macs"] += o["dense_macs"]
        elif o["op"] == "gemm_mfma":
            out["gemm_ops"] += 2.0 * o["macs"]
    return out


def _rooflines(plan, system, d, stream, reps, traffic):
    """Per grouped-launch kind: the average launch duration (back-to-back
    launches between two HIP events on the execution stream) against the
    kernel's roofline, with its algorithmic work per launch."""
    from paper_1609_00061_amd import pa
    groups = plan.time_groups(reps=reps, stream=stream)
    by = {}
    for kind, ms, macs in groups:
        a = by.setdefault(kind, {"ms": 0.0, "launches": 0, "macs": 0.0})
        a["ms"] += ms
        a["launches"] += 1
        a["macs"] += macs
    w = _work_of(system, d)
    plotted = set(p["rel"] for p in d["plots"])
    names = {pa.OPKIND_PLOT: ("plot", "k_group<0> (corner plotting, FP32 + FP64 escalation)", "alu"),
             pa.OPKIND_GATHER: ("sparse_pass", "k_group<4> (sparse pass: row gather)", "hbm"),
             pa.OPKIND_GEMM: ("gemm", "k_group<1|11|21|31> (fp4-MFMA Boolean contraction tiles)", "mfma"),
             pa.OPKIND_STREAM_K: ("stream", "k_group<12> (word-streamed contraction)", "hbm"),
             pa.OPKIND_STREAM_W: ("stream_w", "k_group<22> (word-streamed contraction, broadcast)", "hbm"),
             pa.OPKIND_COUNT: ("count", "k_group<5> (set-bit count of A)", None),
             pa.OPKIND_ROWLIST: ("row_list", "k_group<6> (row lists of the set bits of A)", "hbm"),
             pa.OPKIND_FUSED: ("fused", "k_fused_group (fused pass pair: LDS row gathers)", "lds")}
    roof = {}
    for kind, a in by.items():
        if kind not in names:
            continue
        key, kernel, bound = names[kind]
        avg = a["ms"] / a["launches"]
        ent = {"kernel": kernel, "bound": bound, "avg_launch_ms": avg, "launches_per_step": a["launches"],
               "ms_per_step": a["ms"], "traffic": traffic.get(key)}
        if kind == pa.OPKIND_PLOT:
            # the plots of one solve: every relation plotted (second plots of B included)
            fl = sum(_plot_flops(system, {p["rel"]}) for p in d["plots"]) / a["launches"]
            ach = fl / (avg * 1e-3) / 1e12
            ent.update(achieved=ach, peak=FP32_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                       frac=ach / FP32_VECTOR_PEAK_TFLOPS, flop_per_launch=fl, relations_plotted=len(plotted))
        elif kind == pa.OPKIND_GEMM:
            ops = 2.0 * a["macs"] / a["launches"]
            ach = ops / (avg * 1e-3) / 1e12
            # Boolean ops (2 per MAC) against the dense peak of the MFMA type
            # the kernel runs on (fp4 e2m1, fp32 accumulation)
            ent.update(achieved=ach, peak=FP4_DENSE_PEAK_TOPS, unit="TOP/s", frac=ach / FP4_DENSE_PEAK_TOPS,
                       mfma_dtype="fp4", frac_of_int8_peak=ach / INT8_DENSE_PEAK_TOPS, ops_per_launch=ops)
        elif kind == pa.OPKIND_GATHER:
            b = w["sparse_bytes"] / a["launches"]
            ach = b / (avg * 1e-3) / 1e9
            ent.update(achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS, bytes_per_launch=b,
                       effective_tops=2.0 * w["sparse_macs"] / (a["ms"] * 1e-3) / 1e12)
        elif kind == pa.OPKIND_ROWLIST:
            b = w["list_bytes"] / a["launches"]
            ach = b / (avg * 1e-3) / 1e9
            ent.update(achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS, bytes_per_launch=b)
        elif kind == pa.OPKIND_FUSED:
            b = w["fused_lds_bytes"] / a["launches"]
            ach = b / (avg * 1e-3) / 1e9
            meas = pa.lds_read_rate(stream) / 1e9
            ent.update(achieved=ach, peak=LDS_PEAK_GBS, unit="GB/s", frac=ach / LDS_PEAK_GBS, lds_bytes_per_launch=b,
                       lds_read_rate_measured=meas, frac_of_measured=ach / meas,
                       effective_tops=2.0 * w["fused_macs"] / (a["ms"] * 1e-3) / 1e12)
        elif kind in (pa.OPKIND_STREAM_K, pa.OPKIND_STREAM_W):
            b = w["stream_bytes"] / a["launches"]
            ach = b / (avg * 1e-3) / 1e9
            ent.update(achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS, bytes_per_launch=b)
        roof[key] = ent
    return roof


def _roofline_line(entry):
    r = {k: entry.get(k) for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")}
    r["kernel"] = entry["kernel"]
    r["avg_launch_ms"] = entry["avg_launch_ms"]
    return r


def _tuning(args_tuning, systems, stream):
    from paper_1609_00061_amd import pa
    if args_tuning:
        return {k: int(v) for k, v in json.loads(args_tuning).items()}
    best, _ = pa.autotune(systems, reps=3, stream=stream, order=pa.ORDER_EXHAUSTIVE, graph=True)
    return {k: int(v) for k, v in best.items() if k != "ms"}


def _ternary(stream, K, W, tuning_arg=None, quick=False):
    """The headline workload: the optimised path (autotuned, graph replay),
    its rooflines, the MFMA-only and plain plans, and planning-inclusive
    rates."""
    import torch
    from paper_1609_00061_amd import inputs, pa
    s = inputs.config3()
    _progress("ternary: autotuning")
    t0 = time.perf_counter()
    tuning = _tuning(tuning_arg, [s], stream)
    tune_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    plan = pa.Plan(s, order=pa.ORDER_EXHAUSTIVE, graph=True, **tuning)
    create_s = time.perf_counter() - t0
    out = pa.empty_bits(plan.dims)
    torch.cuda.synchronize()
    _progress(f"ternary: timing {K} solves")
    dt = _time_plan(plan, out, K, W, stream)
    _, rep, _ = plan.execute(out, stream=stream, report=True)
    pct = _step_percentiles(plan, out, stream, min(max(K, 10), 100))
    d = pa.describe_plan(s, order=pa.ORDER_EXHAUSTIVE, **tuning)
    res = {"value": K / dt, "ms_per_step": 1e3 * dt / K, "step_ms_events": pct, "tuning": tuning,
           "autotune_s": tune_s, "plan_create_s": create_s, "nnz_out": rep["nnz_out"],
           "corners": rep["corners"], "escalated_corners": rep["corners_flagged"],
           "kernels": [o["op"] for o in d["ops"]], "out": out, "dims": plan.dims, "system": s}
    _progress("ternary: per-kernel rooflines")
    roof = _rooflines(plan, s, d, stream, reps=5, traffic=_measured_traffic("c3_ternary_r256_traffic.json"))
    res["roofline_by_kernel"] = roof
    # host planning alone (no device work), and whole solves that create a
    # plan each time (planning, workspace allocation, upload, execution)
    t0 = time.perf_counter()
    for _ in range(5):
        pa.describe_plan(s, order=pa.ORDER_EXHAUSTIVE, **tuning)
    res["host_plan_ms"] = 1e3 * (time.perf_counter() - t0) / 5
    n_pl = 3 if quick else 5
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_pl):
        p2 = pa.Plan(s, order=pa.ORDER_EXHAUSTIVE, **tuning)
        o2 = pa.empty_bits(p2.dims)
        p2.execute(o2, stream=stream)
        torch.cuda.synchronize()
        del p2, o2
    res["with_planning"] = {"value": n_pl / (time.perf_counter() - t0), "unit": "solves/s",
                            "what": "pa_plan_create (host planning, workspace allocation, table upload) + one "
                                    "execution + destroy per solve, synchronized"}
    # the same contractions on the MFMA kernel (sparse pass off)
    _progress("ternary: MFMA-only plan")
    mplan = pa.Plan(s, order=pa.ORDER_EXHAUSTIVE, graph=True, **dict(tuning, sparse_pass=-1, gemm_path=0))
    mout = pa.empty_bits(mplan.dims)
    torch.cuda.synchronize()
    nm = max(3, K // 4)
    mdt = _time_plan(mplan, mout, nm, 1, stream)
    md = pa.describe_plan(s, order=pa.ORDER_EXHAUSTIVE, **dict(tuning, sparse_pass=-1, gemm_path=0))
    mroof = _rooflines(mplan, s, md, stream, reps=3, traffic={})
    res["mfma_only"] = {"value": nm / mdt, "unit": "solves/s", "same_bits": bool(torch.equal(mout, out)),
                        "plan": "sparse pass off, default MFMA operand path", "roofline_by_kernel": mroof}
    del mplan, mout
    # the plain GPU path (the metric's baseline)
    _progress("ternary: plain GPU path")
    pplan = pa.Plan(s, order=pa.ORDER_GREEDY, plain=True)
    pout = pa.empty_bits(pplan.dims)
    torch.cuda.synchronize()
    npl = max(3, K // 4)
    pdt = _time_plan(pplan, pout, npl, 1)
    res["plain_gpu"] = {"value": npl / pdt, "unit": "solves/s", "ms_per_step": 1e3 * pdt / npl,
                        "path": "greedy order, one plotting launch per relation, one launch per contraction step "
                                "(MFMA, no split K, no sparse pass), no graph, default tiles",
                        "same_bits": bool(torch.equal(pout, out))}
    del pplan, pout
    return res


def _chain(stream, K, W, tuning_arg=None):
    """The chain workload: autotuned (or given) graph replay, its rooflines,
    the plain path and the single persistent launch."""
    import torch
    from paper_1609_00061_amd import inputs, pa
    s = inputs.config2()
    tuning = _tuning(tuning_arg, [s], stream)
    plan = pa.Plan(s, order=pa.ORDER_EXHAUSTIVE, graph=True, **tuning)
    out = pa.empty_bits(plan.dims)
    torch.cuda.synchronize()
    dt = _time_plan(plan, out, K, W, stream)
    _, rep, _ = plan.execute(out, stream=stream, report=True)
    kplan = plan
    if tuning.get("single_launch"):
        kplan = pa.Plan(s, order=pa.ORDER_EXHAUSTIVE, graph=True, **dict(tuning, single_launch=0))
        kplan.execute(pa.empty_bits(kplan.dims), stream=stream)
    d = pa.describe_plan(s, order=pa.ORDER_EXHAUSTIVE, **tuning)
    roof = _rooflines(kplan, s, d, stream, reps=20, traffic=_measured_traffic("c2_chain8_r1024_traffic.json"))
    res = {"workload": CHAIN, "value": K / dt, "unit": "solves/s", "ms_per_step": 1e3 * dt / K, "tuning": tuning,
           "nnz_out": rep["nnz_out"], "escalated_corners": rep["corners_flagged"], "roofline_by_kernel": roof}
    pplan = pa.Plan(s, order=pa.ORDER_GREEDY, plain=True)
    pout = pa.empty_bits(pplan.dims)
    torch.cuda.synchronize()
    pdt = _time_plan(pplan, pout, K, W)
    res["plain_gpu"] = {"value": K / pdt, "unit": "solves/s", "same_bits": bool(torch.equal(pout, out))}
    splan = pa.Plan(s, order=pa.ORDER_EXHAUSTIVE, graph=True, single_launch=True)
    sout = pa.empty_bits(splan.dims)
    torch.cuda.synchronize()
    sdt = _time_plan(splan, sout, K, W, stream)
    res["single_launch"] = {"value": K / sdt, "unit": "solves/s", "same_bits": bool(torch.equal(sout, out))}
    res["out"] = out
    res["dims"] = plan.dims
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
    torch.cuda.synchronize()
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
    torch.cuda.synchronize()
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
    return {"workload": "512 independent chains of 2-6 binary cubic relations, N(0,1) coefficients, [-3,3], "
                        "per-axis resolution log-uniform in [64, 2048]",
            "value": len(systems) / bdt, "unit": "solves/s", "ms_per_batch": 1e3 * bdt,
            "executor": "one hipGraph replay of level-grouped launches over all systems, autotuned tiles",
            "batch_create_s": create_s,
            "with_planning": {"value": len(systems) / (create_s + bdt), "unit": "solves/s",
                              "what": "batch creation (autotune cache hit, planning, allocation, upload) + one "
                                      "replay"},
            "plain_gpu": {"value": len(systems) / pdt, "unit": "solves/s", "ms_per_batch": 1e3 * pdt,
                          "path": "one plain plan per system, greedy order, one launch per plot and step"},
            "speedup_vs_plain": pdt / bdt, "same_bits_as_plain": same}


def _learned(stream, n_train=128, n_eval=256, res=128):
    """Random relation hypergraphs (8-14 variables, arity 2-3, 2-4 exposed,
    128 cells/axis): the step-time model trained on the GPU from the
    library's own timings on training graphs, then every policy timed on
    the disjoint evaluation graphs (one graph replay per solve; planning
    time reported apart), and the learned order batched into one replay vs
    one plain solve per system."""
    import numpy as np
    import torch
    from paper_1609_00061_amd import inputs, learn, pa
    t0 = time.perf_counter()
    model, X, T = learn.train_order_model(inputs.config5(n_graphs=n_train, index=1000, res=res), rounds=2,
                                         n_random=4, steps=4000, log=_progress, measure_density=True)
    train_s = time.perf_counter() - t0
    pred = model.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    r2 = float(1.0 - np.mean((pred - T) ** 2) / np.var(T))
    evals = inputs.config5(n_graphs=n_eval, index=0, res=res)
    _progress(f"trained in {train_s:.1f} s on {len(T)} samples; timing policies on {len(evals)} graphs")
    pol = learn.time_policies(evals, model, policies=("greedy", "exhaustive", "learned"), steps=3, stream=stream,
                              measure_density=True)
    out = {"workload": f"{n_eval} random relation hypergraphs (8-14 variables, arity 2-3, 2-4 exposed, "
                       f"{res} cells/axis, [-3,3], at most 4 variables kept and 6 ranged over per merge of some "
                       f"tree); model trained on {n_train} disjoint graphs; density features from the plot "
                       f"densities each plan measures",
           "train_s": train_s, "train_samples": int(len(T)), "fit_r2": r2,
           "same_bits_all_policies": pol["same_bits"], "systems": pol["systems"],
           "skipped_enomem": pol["skipped_enomem"]}
    for p in ("greedy", "exhaustive", "learned"):
        out[p] = {"total_ms": pol[p]["total_ms"], "plan_ms_mean": pol[p]["plan_ms_mean"],
                  "total_with_planning_ms": pol[p]["total_ms"] + pol[p]["plan_ms_mean"] * pol["systems"]}
    ex, le = np.array(pol["exhaustive"]["per_system_ms"]), np.array(pol["learned"]["per_system_ms"])
    out["learned_vs_exhaustive"] = pol["exhaustive"]["total_ms"] / pol["learned"]["total_ms"]
    out["learned_vs_exhaustive_with_planning"] = (out["exhaustive"]["total_with_planning_ms"] /
                                                  out["learned"]["total_with_planning_ms"])
    out["learned_vs_exhaustive_geomean"] = float(np.exp(np.mean(np.log(ex / le))))
    out["learned_wins_losses_1p2x"] = [int(np.sum(ex / le > 1.2)), int(np.sum(ex / le < 1 / 1.2))]
    out["learned_vs_greedy"] = pol["greedy"]["total_ms"] / pol["learned"]["total_ms"]
    # the plain path (greedy order) cannot run every graph: some greedy trees
    # need more memory than the GPU has, or take minutes; the comparison runs
    # on the graphs whose greedy plan fits and costs at most 1e13 MACs
    ok = []
    for s in evals:
        d = pa.describe_plan(s, order=pa.ORDER_GREEDY, plain=True)
        if "error" not in d and d["cost"] <= 1e13 and d["workspace_bytes"] <= 2 ** 35:
            ok.append(s)
    out["vs_plain_graphs"] = len(ok)
    try:
        b = pa.Batch(ok, order=pa.ORDER_LEARNED, model=model, graph=True, autotune=True, measure_density=True)
        outs = b.alloc_outputs()
        torch.cuda.synchronize()
        b.execute(outs, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            b.execute(outs, stream=stream)
        torch.cuda.synchronize()
        bdt = (time.perf_counter() - t0) / 3
        plain_s = 0.0
        for s in ok:
            p = pa.Plan(s, order=pa.ORDER_GREEDY, plain=True)
            o = pa.empty_bits(p.dims)
            torch.cuda.synchronize()
            p.execute(o)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            p.execute(o)
            torch.cuda.synchronize()
            plain_s += time.perf_counter() - t1
            del p, o
        out["learned_batched"] = {"value": len(ok) / bdt, "unit": "solves/s", "systems": len(ok)}
        out["plain_gpu"] = {"value": len(ok) / plain_s, "unit": "solves/s",
                            "path": "greedy order, one launch per plot and step, per system"}
        out["speedup_vs_plain"] = out["learned_batched"]["value"] / out["plain_gpu"]["value"]
    except pa.PaError as e:
        out["learned_batched"] = {"error": str(e)}
    return out


def _audit(stream):
    """Escalated corners and FP32/FP64 sign disagreements (all corners also
    evaluated in FP64) per workload; every disagreement must be among the
    escalated corners."""
    from paper_1609_00061_amd import inputs, pa
    out = {}
    for name, s in (("tiny", inputs.config1()), ("chain", inputs.config2()), ("ternary", inputs.config3())):
        _, _, rep = pa.solve_system(s, audit=True)
        out[name] = {k: rep[k] for k in ("corners", "corners_flagged", "corners_disagree",
                                         "corners_disagree_unflagged")}
    for name, systems in (("batch_512_chains", inputs.config4()),
                          ("hypergraphs_256", inputs.config5(n_graphs=256, index=0, res=128))):
        b = pa.Batch(systems, audit=True)
        _, rep, _ = b.execute(stream=stream, report=True)
        out[name] = {k: rep[k] for k in ("corners", "corners_flagged", "corners_disagree",
                                         "corners_disagree_unflagged")}
        del b
    return out


def _cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        visible = len(os.sched_getaffinity(0))
    except AttributeError:
        visible = os.cpu_count()
    return model, visible


def _cpu_baseline(system, gpu_bits):
    """The oracle (plain C: corner plots, then the cluster tree
    {{R1, R2}, {R3, R4}} multiplied pairwise as i-k-j loops) solving the same
    instance, once with a thread per available core (at most 16, the box's
    CPU share) and once with one thread."""
    import numpy as np
    import oracle
    model, visible = _cpu_info()
    nthreads = max(1, min(16, visible or 1))
    res = {v: system.axes[v][2] for v in range(len(system.axes))}
    rel_vars = [r.vars for r in system.relations]
    merges = [(0, 1), (2, 3), (4, 5)]

    def one(nt):
        t0 = time.perf_counter()
        plots = [oracle.plot(r, system.axes, nthreads=nt)[0] for r in system.relations]
        t1 = time.perf_counter()
        ref = oracle.solve_pairwise(res, rel_vars, plots, system.exposed, merges, nthreads=nt)
        return ref, t1 - t0, time.perf_counter() - t1

    ref, tp, tc = one(nthreads)
    _progress(f"oracle with {nthreads} threads: plot {tp:.1f} s, contract {tc:.1f} s")
    exact = bool(np.array_equal(ref, gpu_bits))
    del ref
    _, tp1, tc1 = one(1)
    _progress(f"oracle with 1 thread: plot {tp1:.1f} s, contract {tc1:.1f} s")
    return {"value": 1.0 / (tp + tc), "unit": "solves/s", "cores": nthreads, "kind": "oracle",
            "sample": f"one full solve of the ternary instance: 4 corner plots at 257^3 corners ({tp:.1f} s) + 3 "
                      f"pairwise contractions ({tc:.1f} s), {nthreads} threads",
            "cpu_model": model, "host_cpus_visible": visible,
            "one_thread": {"value": 1.0 / (tp1 + tc1), "unit": "solves/s", "plot_s": tp1, "contract_s": tc1},
            "bit_exact_vs_gpu": exact}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-chain", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-audit", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline workload and its rooflines (for profiling)")
    ap.add_argument("--chain-only", action="store_true", help="only the chain workload (for profiling)")
    ap.add_argument("--tuning", type=str, default="",
                    help="JSON executor settings to use instead of autotuning (e.g. for counter runs, whose "
                         "serialization distorts timings)")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="after the run, copy a buffer of this size 3 times (scales HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              f"(independent systems would shard round-robin across GPUs without communication)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1609_00061_amd import pa

    torch.cuda.set_device(0)
    K, W = args.steps, args.warmup
    stream = torch.cuda.Stream()

    if args.chain_only:
        res = _chain(stream, K, W, args.tuning or None)
        res.pop("out"), res.pop("dims")
        _calibration_copy(args.calibration_copy_mib)
        print(json.dumps(res), flush=True)
        return

    t = _ternary(stream, K, W, tuning_arg=args.tuning or None, quick=args.headline_only)
    roof = t["roofline_by_kernel"]
    dom = max(roof.values(), key=lambda r: r["ms_per_step"])
    result = {
        "metric": METRIC,
        "value": t["value"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": t["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": TERNARY, "plotting": "fp32 + fp64 escalation",
                   "contraction": "bit-packed Boolean, as the autotuner plans it: the two r^5 contractions and "
                                  "the final one fused (row lists of set bits, LDS-staged row gathers, u32 word "
                                  "AND/OR), or sparse row-gather passes with a word-streamed final step, or fp4-MFMA "
                                  "(fp32 accumulation, sum>0)",
                   "order": "exhaustive naive-cost cluster tree",
                   "executor": "one grouped launch per tree level and kernel kind, hipGraph replay, tiles " +
                               ("given" if args.tuning else "autotuned"),
                   "global_batch": 1},
        "roofline": _roofline_line(dom),
        "roofline_by_kernel": roof,
        "step_ms_events": t["step_ms_events"],
        "tuning": t["tuning"],
        "kernels": t["kernels"],
        "nnz_out": t["nnz_out"],
        "corners": t["corners"],
        "escalated_corners": t["escalated_corners"],
        "host_plan_ms": t["host_plan_ms"],
        "with_planning": t["with_planning"],
        "autotune_s": t["autotune_s"],
        "mfma_only": t["mfma_only"],
        "plain_gpu": t["plain_gpu"],
        "speedup_vs_plain": t["value"] / t["plain_gpu"]["value"],
        "paper_context": PAPER_CONTEXT,
    }
    g = t["mfma_only"]["roofline_by_kernel"].get("gemm")
    if g:
        result["contraction_tops_mfma"] = g["achieved"]
    sp = roof.get("sparse_pass")
    if sp:
        result["contraction_effective_tops"] = sp["effective_tops"]
    _progress(f"ternary: {t['value']:.1f} solves/s, plain {t['plain_gpu']['value']:.1f}")
    gpu_bits = pa.unpack_bits(t["out"].cpu().numpy(), t["dims"])
    system = t["system"]
    del t

    if not args.headline_only:
        if not args.no_chain:
            _progress("chain workload")
            c = _chain(stream, K, W)
            c.pop("out"), c.pop("dims")
            result["chain"] = c
        if not args.no_batched:
            _progress("batched workload")
            result["batched"] = _batched(stream, max(5, K // 10), 3)
        if not args.no_learned:
            _progress("learned order")
            result["learned_order"] = _learned(stream)
        if not args.no_audit:
            _progress("audit counts")
            result["fp32_fp64_audit"] = _audit(stream)
        if not args.no_cpu_baseline:
            _progress("cpu baseline (oracle)")
            result["cpu_baseline"] = _cpu_baseline(system, gpu_bits)
            result["bit_exact_vs_oracle"] = result["cpu_baseline"]["bit_exact_vs_gpu"]

    _calibration_copy(args.calibration_copy_mib)
    print(json.dumps(result), flush=True)


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


if __name__ == "__main__":
    main()
