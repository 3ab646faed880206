"""GPU parity of the other plotting rules against the oracle, bit-exact, in
FP64 mode and in FP32 mode with FP64 escalation (with audit counts): the
epsilon-tolerance sample-in-center plot (Def. sample_in_center) for the
targets f = 0, f <= 0 and f < 0, the corner plot of inequalities, and whole
solves built from them on every executor."""
import numpy as np
import pytest

import oracle
from paper_1609_00061_amd import inputs, pa
from gpu_util import note, random_relation, to_host

pytestmark = pytest.mark.gpu

MODES = [pa.PLOT_FP64, pa.PLOT_FP32_ESCALATE]
SHAPES = [
    (1, [(-3.0, 3.0, 1000)]),
    (1, [(-1.0, 2.5, 65)]),
    (2, [(-3.0, 3.0, 64), (-3.0, 3.0, 64)]),
    (2, [(-3.0, 3.0, 100), (-2.0, 1.0, 33)]),
    (2, [(-1.5, 3.0, 129), (-3.0, 3.0, 257)]),
    (2, [(-3.0, 3.0, 2), (-3.0, 3.0, 200)]),
    (3, [(-3.0, 3.0, 16), (-3.0, 3.0, 16), (-3.0, 3.0, 16)]),
    (3, [(-3.0, 3.0, 30), (-2.0, 2.5, 65), (-3.0, 3.0, 31)]),
]


def _with_target(rel, target):
    return inputs.Relation(rel.vars, rel.degree, rel.coef, target)


def _plot(rel, axes, precision, audit=False, **kw):
    note("plot", rel.vars, [a[2] for a in axes], "target", rel.target, "precision", precision, kw)
    t, dims, rep = pa.plot_relation(rel, axes, precision=precision, audit=audit, **kw)
    return to_host(t, dims), rep


@pytest.mark.parametrize("precision", MODES)
@pytest.mark.parametrize("case", range(len(SHAPES)))
def test_center_rule_random_cubics(case, precision):
    arity, axes = SHAPES[case]
    for seed in range(2):
        base = random_relation(7500 + 31 * case + seed, arity)
        for target in (0, 1, 2):
            for eps in (0.0, 0.05, 0.7):
                rel = _with_target(base, target)
                got, rep = _plot(rel, axes, precision, audit=(precision == pa.PLOT_FP32_ESCALATE),
                                 plot_rule=pa.RULE_CENTER, tolerance=eps)
                ref = oracle.plot_center(rel, axes, eps, target)
                assert np.array_equal(got, ref), (case, seed, target, eps)
                assert rep["corners"] == int(np.prod([a[2] for a in axes]))
                if precision == pa.PLOT_FP32_ESCALATE:
                    assert rep["corners_disagree_unflagged"] == 0
                    assert rep["corners_flagged"] < max(64, rep["corners"] // 20)


@pytest.mark.parametrize("precision", MODES)
def test_center_rule_exact_ties(precision):
    """The circle on [-2, 2]^2 at 64 with eps = 258/1024: centre values are
    exact in FP32 and some equal eps exactly, so the FP32 pass cannot decide
    them and the canonical value does (set for f = 0 and f <= 0, unset for
    f < 0)."""
    for target in (0, 1, 2):
        rel = inputs.Relation((0, 1), 2, np.array([-1.0, 0, 0, 1.0, 0, 1.0]), target)
        axes = [(-2.0, 2.0, 64)] * 2
        got, rep = _plot(rel, axes, precision, audit=True, plot_rule=pa.RULE_CENTER, tolerance=258 / 1024)
        ref = oracle.plot_center(rel, axes, 258 / 1024, target)
        assert np.array_equal(got, ref), target
        if precision == pa.PLOT_FP32_ESCALATE:
            assert rep["corners_flagged"] >= 8
            assert rep["corners_disagree_unflagged"] == 0


def test_center_rule_appendix_sample():
    """App. A's sample relations y - x^2 and y + z^2 - 1 on [-1.2, 1.2] at 50,
    tolerance 0.05, and their product (the sample's M1 * M2)."""
    ax = (-1.2, 1.2, 50)
    s = inputs.System([ax] * 3, [inputs.Relation((0, 1), 2, np.array([0, 0, 1.0, -1.0, 0, 0])),
                                 inputs.Relation((1, 2), 2, np.array([-1.0, 1.0, 0, 0, 0, 1.0]))], (0, 2),
                      name="appendix")
    plots = [oracle.plot_center(r, s.axes, 0.05) for r in s.relations]
    for r, ref in zip(s.relations, plots):
        got, _ = _plot(r, [ax, ax], pa.PLOT_FP32_ESCALATE, plot_rule=pa.RULE_CENTER, tolerance=0.05)
        assert np.array_equal(got, ref)
    ref = oracle.solve([50] * 3, [r.vars for r in s.relations], plots, s.exposed)
    assert np.array_equal(ref.astype(bool), (plots[0].astype(np.int64) @ plots[1].astype(np.int64)) > 0)
    out, dims, rep = pa.solve_system(s, plot_rule=pa.RULE_CENTER, tolerance=0.05)
    assert np.array_equal(to_host(out, dims), ref)


@pytest.mark.parametrize("precision", MODES)
@pytest.mark.parametrize("case", range(len(SHAPES)))
def test_inequality_corner_rule(case, precision):
    arity, axes = SHAPES[case]
    for seed in range(2):
        base = random_relation(7700 + 31 * case + seed, arity)
        for target in (1, 2):
            rel = _with_target(base, target)
            got, rep = _plot(rel, axes, precision, audit=(precision == pa.PLOT_FP32_ESCALATE))
            ref = oracle.plot_ineq(rel, axes, target)
            assert np.array_equal(got, ref), (case, seed, target)
            if precision == pa.PLOT_FP32_ESCALATE:
                assert rep["corners_disagree_unflagged"] == 0


def test_inequality_planted_zero_corners():
    """f = (x - x_k) q(x, y) with x_k a grid line of x: on that line |f| is at
    the level of the coefficients' rounding, so the FP32 pass escalates those
    corners and the canonical FP64 values decide f = 0, f <= 0 and f < 0."""
    rng = inputs.SplitMix64(7800)
    q = rng.normals(6)                  # quadratic q on (x, y): 1, x, y, x2, xy, y2
    xk = -3.0 + 11 * 0.125              # a corner coordinate of [-3, 3] at 48 cells
    # (x - xk) * q as a cubic in graded-lex order 1, x, y, x2, xy, y2, x3, x2y, xy2, y3
    c = np.zeros(10)
    c[0] = -xk * q[0]
    c[1] = q[0] - xk * q[1]
    c[2] = -xk * q[2]
    c[3] = q[1] - xk * q[3]
    c[4] = q[2] - xk * q[4]
    c[5] = -xk * q[5]
    c[6] = q[3]
    c[7] = q[4]
    c[8] = q[5]
    axes = [(-3.0, 3.0, 48), (-3.0, 3.0, 40)]
    for target in (0, 1, 2):
        rel = inputs.Relation((0, 1), 3, c, target)
        for precision in MODES:
            got, rep = _plot(rel, axes, precision, audit=True)
            ref = oracle.plot_relation(rel, axes)
            assert np.array_equal(got, ref), (target, precision)
            if precision == pa.PLOT_FP32_ESCALATE:
                assert rep["corners_disagree_unflagged"] == 0


def _mixed_system(seed, res_lo=6, res_hi=28):
    rng = inputs.SplitMix64(seed)
    g = inputs.random_hypergraph(rng, res=rng.randint(res_lo, res_hi))
    g.axes = [(-3.0, 3.0, rng.randint(3, 30)) for _ in g.axes]
    g.relations = [_with_target(r, rng.randint(0, 2)) for r in g.relations]
    g.name = f"mixed{seed}"
    return g


EXECUTORS = [dict(), dict(plain=True, order=pa.ORDER_GREEDY), dict(per_op=True), dict(graph=True),
             dict(single_launch=True), dict(sparse_pass=2), dict(precision=pa.PLOT_FP64)]


@pytest.mark.parametrize("rule", ["corner", "center"])
@pytest.mark.parametrize("seed", range(4))
def test_solves_with_rules_and_targets(rule, seed):
    """Random hypergraphs whose relations are equations and inequalities,
    plotted by either rule, solved on every executor: the oracle's bits."""
    s = _mixed_system(7900 + seed)
    eps = 0.4
    plots = [oracle.plot_relation(r, s.axes, rule=rule, eps=eps) for r in s.relations]
    ref = oracle.solve([a[2] for a in s.axes], [r.vars for r in s.relations], plots, s.exposed)
    kw_rule = dict(plot_rule=pa.RULE_CENTER, tolerance=eps) if rule == "center" else {}
    for kw in EXECUTORS:
        note("solve", s.name, rule, kw)
        out, dims, rep = pa.solve_system(s, **kw_rule, **kw)
        assert np.array_equal(to_host(out, dims), ref), (rule, kw)
        assert rep["nnz_out"] == int(ref.sum())


@pytest.mark.parametrize("rule", ["corner", "center"])
def test_batch_with_rules_and_targets(rule):
    import torch
    systems = [_mixed_system(8000 + i) for i in range(8)]
    eps = 0.3
    kw_rule = dict(plot_rule=pa.RULE_CENTER, tolerance=eps) if rule == "center" else {}
    refs = []
    for s in systems:
        plots = [oracle.plot_relation(r, s.axes, rule=rule, eps=eps) for r in s.relations]
        refs.append(oracle.solve([a[2] for a in s.axes], [r.vars for r in s.relations], plots, s.exposed))
    for kw in (dict(graph=True), dict(single_launch=True)):
        b = pa.Batch(systems, **kw_rule, **kw)
        outs, rep, nnz = b.execute(stream=torch.cuda.Stream(), report=True)
        for i, (o, d, ref) in enumerate(zip(outs, b.dims, refs)):
            assert np.array_equal(to_host(o, d), ref), (rule, kw, i)


def test_center_rule_full_size_chain_and_ternary():
    """The chain (1024 per axis) and the ternary system (256^3) plotted by the
    centre rule with eps = 0.05 and solved: whole outputs against the oracle's
    pairwise multiplication."""
    for s, merges in ((inputs.config2(), [(0, 1)] + [(8 + t, t + 2) for t in range(6)]),
                      (inputs.config3(), [(0, 1), (2, 3), (4, 5)])):
        note("centre rule full size", s.name)
        plots = [oracle.plot_center(r, s.axes, 0.05) for r in s.relations]
        res = {v: s.axes[v][2] for v in range(len(s.axes))}
        ref = oracle.solve_pairwise(res, [r.vars for r in s.relations], plots, s.exposed, merges, log=note)
        del plots
        for kw in (dict(), dict(sparse_pass=-1)):
            out, dims, rep = pa.solve_system(s, plot_rule=pa.RULE_CENTER, tolerance=0.05, audit=True, **kw)
            assert np.array_equal(to_host(out, dims), ref), (s.name, kw)
            assert rep["corners_disagree_unflagged"] == 0
            note(s.name, kw, "nnz", int(ref.sum()), "flagged", rep["corners_flagged"], "of", rep["corners"])
