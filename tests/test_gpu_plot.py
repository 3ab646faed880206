"""GPU parity of plotting (Sec. 3.2, corner rule): bit-exact against the
oracle, in FP64 mode and in FP32 mode with FP64 escalation."""
import numpy as np
import pytest

import oracle
from paper_1609_00061_amd import inputs, pa
from gpu_util import note, random_relation, to_host

pytestmark = pytest.mark.gpu

MODES = [pa.PLOT_FP64, pa.PLOT_FP32_ESCALATE]


def _plot(rel, axes, precision, audit=False):
    note("plot", rel.vars, [a[2] for a in axes], "precision", precision, "audit", audit)
    t, dims, rep = pa.plot_relation(rel, axes, precision=precision, audit=audit)
    return to_host(t, dims), rep


@pytest.mark.parametrize("precision", MODES)
def test_c1_plots(precision):
    """The tiny system's two plots; the 4 + 5 exact-zero corners are the only
    ones an FP32 bound can flag (every other |f| >= 1/4096)."""
    s = inputs.config1()
    for rel, nz_expect in zip(s.relations, (4, 5)):
        axes = [s.axes[v] for v in rel.vars]
        got, rep = _plot(rel, axes, precision)
        ref, nz = oracle.plot(rel, s.axes)
        assert nz == nz_expect
        assert np.array_equal(got, ref)
        if precision == pa.PLOT_FP32_ESCALATE:
            assert rep["corners_flagged"] == nz_expect
        else:
            assert rep["corners_flagged"] == 0


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


@pytest.mark.parametrize("precision", MODES)
@pytest.mark.parametrize("case", range(len(SHAPES)))
def test_random_cubics(case, precision):
    arity, axes = SHAPES[case]
    for seed in range(3):
        rel = random_relation(7000 + 31 * case + seed, arity)
        got, rep = _plot(rel, axes, precision, audit=(precision == pa.PLOT_FP32_ESCALATE))
        full_axes = list(axes)
        ref, _ = oracle.plot(rel, full_axes)
        assert np.array_equal(got, ref), (case, seed)
        if precision == pa.PLOT_FP32_ESCALATE:
            # no FP32 sign may differ from FP64 outside the escalated set
            assert rep["corners_disagree_unflagged"] == 0
            assert rep["corners_flagged"] <= max(8, rep["corners"] // 1000)


def test_planted_corner_roots():
    """Adversarial: f = (x - x_k)(y - y_j) q(x, y) vanishes exactly on whole grid
    lines; every such corner must be escalated and decided in FP64."""
    r = 48
    axes = [(-3.0, 3.0, r), (-3.0, 3.0, r)]
    xk, yj = oracle.axis(-3.0, 3.0, r)[17], oracle.axis(-3.0, 3.0, r)[30]
    # (x - xk)(y - yj)(1 + x/4) expanded in graded-lex order 1, x, y, x^2, xy, y^2, x^3, x^2y, xy^2, y^3
    c = np.zeros(10)
    # (x - a)(y - b) = xy - b x - a y + ab ; times (1 + x/4)
    a, b = xk, yj
    c[0] = a * b
    c[1] = -b + a * b / 4
    c[2] = -a
    c[3] = -b / 4
    c[4] = 1.0 - a / 4
    c[7] = 0.25
    rel = inputs.Relation((0, 1), 3, c)
    for precision in MODES:
        got, rep = _plot(rel, axes, precision, audit=(precision == pa.PLOT_FP32_ESCALATE))
        ref, nz = oracle.plot(rel, axes)
        assert np.array_equal(got, ref)
        if precision == pa.PLOT_FP32_ESCALATE:
            assert rep["corners_disagree_unflagged"] == 0
            assert rep["corners_flagged"] >= nz


@pytest.mark.parametrize("which", ["c2", "c3"])
def test_full_size_relations(which):
    """Every relation of the chain (1024^2) and ternary (256^3) workloads at
    full size, FP32 with escalation, bit-exact; then again in audit mode
    (every corner also evaluated in FP64): the same bits, the same escalated
    corners, and every FP32/FP64 sign disagreement among them."""
    s = inputs.config2() if which == "c2" else inputs.config3()
    flagged = disagree = 0
    for rel in s.relations:
        axes = [s.axes[v] for v in rel.vars]
        got, rep = _plot(rel, axes, pa.PLOT_FP32_ESCALATE)
        ref, _ = oracle.plot(rel, s.axes)
        assert np.array_equal(got, ref), rel.vars
        flagged += rep["corners_flagged"]
        got_a, rep_a = _plot(rel, axes, pa.PLOT_FP32_ESCALATE, audit=True)
        assert np.array_equal(got_a, ref), rel.vars
        assert rep_a["corners_disagree_unflagged"] == 0, rel.vars
        assert rep_a["corners_disagree"] <= rep_a["corners_flagged"]
        assert rep_a["corners_flagged"] == rep["corners_flagged"]
        disagree += rep_a["corners_disagree"]
    note(which, "flagged corners", flagged, "FP32/FP64 disagreements", disagree)


EXTREMES = [
    ("huge", 1e36, [(-3.0, 3.0, 40), (-3.0, 3.0, 70)]),         # S > 2^126: every corner escalated
    ("tiny", 1e-30, [(-3.0, 3.0, 40), (-3.0, 3.0, 70)]),        # values near the 2^-100 underflow term
    ("wide", 1.0, [(-1e9, 1e9, 65), (-2e8, 3e9, 66)]),          # |x|^3 ~ 1e27
    ("mixed", 1.0, [(-3.0, 3.0, 50), (-3.0, 3.0, 50)]),         # one coefficient 1e37, the rest N(0,1)
]


@pytest.mark.parametrize("case", range(len(EXTREMES)))
def test_extreme_magnitudes(case):
    """The FP32 bound at its edges: coefficients so large that FP32 could
    overflow (the line bound is +inf and FP64 decides every corner), values
    down at the underflow term, wide axes; bit-exact in both precisions and
    no unflagged FP32/FP64 sign disagreement."""
    name, scale, axes = EXTREMES[case]
    rel = random_relation(9100 + case, 2)
    rel.coef[:] = np.asarray(rel.coef) * scale
    if name == "huge":
        rel.coef[0] = 1e38           # every line's magnitude bound S >= |c_0| > 2^126
    if name == "mixed":
        rel.coef[4] = 1e37
    ref, _ = oracle.plot(rel, axes)
    for precision in MODES:
        got, rep = _plot(rel, axes, precision, audit=(precision == pa.PLOT_FP32_ESCALATE))
        assert np.array_equal(got, ref), (name, precision)
        if precision == pa.PLOT_FP32_ESCALATE:
            assert rep["corners_disagree_unflagged"] == 0
            if name == "huge":
                assert rep["corners_flagged"] == rep["corners"]
