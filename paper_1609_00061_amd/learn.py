"""Training and evaluation of the learned contraction order.

Samples are the library's own measurements: every pairwise step of a timed
plan (per-op launches, HIP events) gives the step's features and log2 of its
duration in microseconds.  Trees come from the greedy and exhaustive
policies and from random merge orders of connected clusters, over training
systems drawn from a seed range disjoint from the evaluation systems.  The
model (forward, backward and Adam in the library's kernels) is fitted to
them, and the learned policy is then compared with the others by measured
solve time on held-out systems, with identical output bits required.
"""
from __future__ import annotations

import time
from typing import Dict, List, Sequence

import numpy as np

from . import inputs, pa


def random_connected_merges(system, rng: inputs.SplitMix64) -> List[int]:
    """A uniformly drawn sequence of merges of two current clusters that share
    a variable (any two clusters once none do), in the PA_ORDER_GIVEN format."""
    n = len(system.relations)
    alive = list(range(n))
    vars_of = {i: set(system.relations[i].vars) for i in range(n)}
    merges, nxt = [], n
    while len(alive) > 1:
        pairs = [(a, b) for i, a in enumerate(alive) for b in alive[i + 1:] if vars_of[a] & vars_of[b]]
        if not pairs:
            pairs = [(a, b) for i, a in enumerate(alive) for b in alive[i + 1:]]
        a, b = pairs[rng.randint(0, len(pairs) - 1)]
        merges += [a, b]
        vars_of[nxt] = vars_of[a] | vars_of[b]
        alive = [x for x in alive if x not in (a, b)] + [nxt]
        nxt += 1
    return merges


def _feasible(system, merges, max_out_log2=33.0) -> bool:
    """Every intermediate of the tree fits a bit budget (2^33 bits = 1 GiB)."""
    n = len(system.relations)
    leaves = [1 << i for i in range(n)]
    for t in range(n - 1):
        a, b = merges[2 * t], merges[2 * t + 1]
        f = pa.step_features(system, leaves[a], leaves[b])
        if f[5] * 8 > max_out_log2 or f[6] * 8 > max_out_log2 or f[7] * 8 > max_out_log2:
            return False
        leaves.append(leaves[a] | leaves[b])
    return True


def collect_samples(systems: Sequence, n_random: int = 3, reps: int = 3, seed: int = 1, stream=None,
                    log=None, model=None, base_policies: bool = True, max_cost_ratio: float = 128.0,
                    measure_density: bool = False):
    """(X [k, F] float32, T [k] float32 log2 microseconds) from timed plans.
    Trees: greedy and exhaustive (base_policies), n_random random connected
    merge orders, and the learned order of `model` when given; a tree whose
    naive cost exceeds max_cost_ratio times the optimum is not timed (one
    such solve can take seconds; slow trees within the ratio stay, so the
    model sees the slow regime it must avoid).  Each tree is executed `reps` times after one warm-up; a step's
    sample is its fastest repetition.  With measure_density the plans measure their plots' densities and
    the samples' density features start from them (as the learned order then does)."""
    rng = inputs.SplitMix64(seed)
    Xs, Ts = [], []
    for si, s in enumerate(systems):
        if len(s.relations) < 2:
            continue
        trees = [dict(order=pa.ORDER_GREEDY), dict(order=pa.ORDER_EXHAUSTIVE)] if base_policies else []
        if model is not None:
            trees.append(dict(order=pa.ORDER_LEARNED, model=model))
        for _ in range(n_random):
            m = random_connected_merges(s, rng)
            if _feasible(s, m):
                trees.append(dict(order=pa.ORDER_GIVEN, given=m))
        best_cost = pa.describe_plan(s, order=pa.ORDER_EXHAUSTIVE).get("cost")
        kept = []
        if model is not None and measure_density:
            trees[-1] = dict(trees[-1], measure_density=True)
        for kw in trees:
            d = pa.describe_plan(s, **kw)
            if "error" in d or (best_cost and d["cost"] > max_cost_ratio * best_cost):
                continue
            kept.append(kw)
        for kw in kept:
            try:
                plan = pa.Plan(s, per_op=True, timing=2, **dict(kw, measure_density=measure_density))
            except pa.PaError as e:          # a tree whose intermediates exceed the workspace cap
                if e.code in (pa.PA_ENOMEM, pa.PA_EUNSUPPORTED):   # or the kernels' 32-bit indexing
                    continue
                raise
            out = pa.empty_bits(plan.dims)
            plan.execute(out, stream=stream)
            best = None
            for _ in range(reps):
                plan.execute(out, stream=stream)
                X, T = pa.plan_step_samples(plan)
                best = T if best is None else np.minimum(best, T)
            Xs.append(X)
            Ts.append(best)
            del plan
        if log:
            log(f"samples: {si + 1}/{len(systems)} systems, {sum(len(t) for t in Ts)} steps")
    return np.concatenate(Xs).astype(np.float32), np.concatenate(Ts).astype(np.float32)


def train(model: "pa.Model", X: np.ndarray, T: np.ndarray, steps: int = 3000, lr: float = 2e-3,
          batch: int = 1024, seed: int = 0, log=None) -> float:
    """Adam on minibatches drawn without replacement per epoch; returns the
    final full-batch loss."""
    import torch
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    Td = torch.from_numpy(np.ascontiguousarray(T)).cuda()
    n = Xd.shape[0]
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    perm = torch.randperm(n, generator=g).cuda()
    pos = 0
    for step in range(steps):
        if pos + batch > n:
            perm = torch.randperm(n, generator=g).cuda()
            pos = 0
        idx = perm[pos:pos + min(batch, n)]
        pos += min(batch, n)
        xb, tb = Xd.index_select(0, idx).contiguous(), Td.index_select(0, idx).contiguous()
        # cosine decay of the step size
        lr_t = lr * 0.5 * (1.0 + np.cos(np.pi * step / steps))
        model.train_step(xb, tb, lr=max(lr_t, lr * 0.02))
        if log and (step + 1) % 1000 == 0:
            _, loss = model.gradient(Xd, Td)
            log(f"train: step {step + 1} loss {loss:.4f}")
    _, loss = model.gradient(Xd, Td)
    return loss


def train_order_model(systems: Sequence, rounds: int = 2, n_random: int = 3, reps: int = 2, steps: int = 3000,
                      seed: int = 1, stream=None, log=None, measure_density: bool = False):
    """Fit the step-time model on the training systems' own timings, then
    (rounds > 1) add the steps of the trees the model itself picks on those
    systems and refit, so its training data covers the region it searches.
    Returns (model, X, T)."""
    X, T = collect_samples(systems, n_random=n_random, reps=reps, seed=seed, stream=stream, log=log,
                           measure_density=measure_density)
    model = pa.Model(seed=seed)
    train(model, X, T, steps=steps, log=log)
    for r in range(1, rounds):
        Xl, Tl = collect_samples(systems, n_random=0, reps=reps, seed=seed + r, stream=stream, log=log, model=model,
                                 base_policies=False, measure_density=measure_density)
        X, T = np.concatenate([X, Xl]), np.concatenate([T, Tl])
        model = pa.Model(seed=seed + r)
        train(model, X, T, steps=steps, log=log)
    return model, X, T


def time_policies(systems: Sequence, model, policies=("greedy", "exhaustive", "learned"), steps: int = 10,
                  warmup: int = 2, stream=None, check_bits: bool = True, log=None,
                  measure_density: bool = False) -> Dict[str, dict]:
    """Measured solve time of every system under each ordering policy (the
    default grouped executor replayed as a hipGraph), plan times, and whether
    all policies produced identical bits.  "learned_verified" is the learned
    order with the exhaustive tree as a measured judge (verify_order)."""
    import torch
    order = {"greedy": pa.ORDER_GREEDY, "exhaustive": pa.ORDER_EXHAUSTIVE, "learned": pa.ORDER_LEARNED,
             "learned_verified": pa.ORDER_LEARNED}
    stream = stream or torch.cuda.Stream()
    res = {p: {"ms": [], "plan_ms": []} for p in policies}
    same = True
    skipped = 0
    for s in systems:
        outs = {}
        plans = {}
        try:
            for p in policies:
                t0 = time.perf_counter()
                learned = p.startswith("learned")
                plans[p] = pa.Plan(s, order=order[p], model=model if learned else None, graph=True,
                                   verify_order=(p == "learned_verified"), measure_density=measure_density and learned)
                res[p]["plan_ms"].append(1e3 * (time.perf_counter() - t0))
        except pa.PaError as e:              # some policy's tree does not fit the workspace cap
            if e.code not in (pa.PA_ENOMEM, pa.PA_EUNSUPPORTED):   # or the kernels' 32-bit indexing
                raise
            for p in plans:
                res[p]["plan_ms"].pop()
            skipped += 1
            continue
        for p in policies:
            plan = plans.pop(p)
            out = pa.empty_bits(plan.dims)
            for _ in range(warmup):
                plan.execute(out, stream=stream)
            stream.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                plan.execute(out, stream=stream)
            stream.synchronize()
            res[p]["ms"].append(1e3 * (time.perf_counter() - t0) / steps)
            outs[p] = out
            del plan
        if check_bits:
            first = outs[policies[0]]
            same = same and all(bool(torch.equal(first, outs[p])) for p in policies[1:])
        if log:
            log(f"timed {s.name}: " + ", ".join(f"{p} {res[p]['ms'][-1]:.3f} ms" for p in policies))
    summary = {p: {"total_ms": float(np.sum(v["ms"])), "per_system_ms": v["ms"],
                   "plan_ms_mean": float(np.mean(v["plan_ms"]))} for p, v in res.items()}
    summary["same_bits"] = same
    summary["systems"] = len(systems) - skipped
    summary["skipped_enomem"] = skipped
    return summary
