"""Pins for the oracle's epsilon-tolerance sample-in-center plot (Def.
sample_in_center, Cor. guarantees) and its corner plot of inequalities
(relations f <= 0 and f < 0, Sec. 3.2), against exact rational arithmetic:
pixel centres, the App. A sample's two relations, the three bullets of
Def. accurate_plot on relations whose range over a cell has a closed form,
and brute force over corners."""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from paper_1609_00061_amd import inputs


def _exact_centers(lo, hi, r):
    lo, hi = Fr(lo), Fr(hi)
    return [lo + (k + Fr(1, 2)) * (hi - lo) / r for k in range(r)]


def test_centers_dyadic_exact():
    """On a dyadic box every centre is exact in FP64."""
    c = oracle.centers(-2.0, 2.0, 64)
    assert [Fr(x) for x in c] == _exact_centers(-2.0, 2.0, 64)
    c = oracle.centers(-3.0, 5.0, 8)
    assert list(c) == [-2.5, -1.5, -0.5, 0.5, 1.5, 2.5, 3.5, 4.5]


def test_centers_within_rounding():
    """Non-dyadic box (App. A's [-1.2, 1.2] at 50): the step, product and sum
    are each rounded once, so a centre is within 3 ulp of the box bound's
    magnitude of the exact one."""
    c = oracle.centers(-1.2, 1.2, 50)
    ex = _exact_centers(-1.2, 1.2, 50)
    ulp = Fr(np.spacing(1.2))
    for x, e in zip(c, ex):
        assert abs(Fr(x) - e) <= 3 * ulp


def _exact_plot(f, axes_lo_hi_r, eps, target):
    """A(e) from exact rational centres (the definition with exact arithmetic)."""
    grids = [_exact_centers(lo, hi, r) for lo, hi, r in axes_lo_hi_r]
    out = np.zeros(tuple(r for _, _, r in axes_lo_hi_r), dtype=np.uint8)
    margin = None
    for idx in np.ndindex(*out.shape):
        v = f(*[g[i] for g, i in zip(grids, idx)])
        d = abs(v) if target == 0 else v
        on = d <= eps if target in (0, 1) else d < eps
        out[idx] = on
        m = abs(d - Fr(eps))
        margin = m if margin is None else min(margin, m)
    return out, margin


@pytest.mark.parametrize("which", ["M1", "M2"])
def test_appendix_sample(which):
    """App. A plots y - x^2 = 0 on (x, y) and y + z^2 - 1 = 0 on (y, z), both on
    [-1.2, 1.2] at 50 pixels per axis with tolerance 0.05 (the appendix code
    tests |f| < tol; Def. sample_in_center's 'achieves' is |f| <= tol: the two
    agree unless some centre value equals the tolerance, checked below)."""
    ax = (-1.2, 1.2, 50)
    if which == "M1":     # variables (x, y); monomials 1, x, y, x^2, xy, y^2
        rel = inputs.Relation((0, 1), 2, np.array([0, 0, 1.0, -1.0, 0, 0]))
        f = lambda x, y: y - x * x
    else:                 # variables (y, z)
        rel = inputs.Relation((0, 1), 2, np.array([-1.0, 1.0, 0, 0, 0, 1.0]))
        f = lambda y, z: y + z * z - 1
    got = oracle.plot_center(rel, [ax, ax], 0.05, 0)
    ref, margin = _exact_plot(f, [ax, ax], Fr(0.05), 0)
    assert margin > Fr(1, 10 ** 9)        # no centre near the threshold: rounding cannot flip a cell
    assert np.array_equal(got, ref)
    assert 40 < got.sum() < 400


def _circle_range(a, b, c, d):
    """Exact [min, max] of x^2 + y^2 - 1 over the closed cell [a,b] x [c,d]."""
    def sq(lo, hi):
        lo2, hi2 = lo * lo, hi * hi
        return (Fr(0) if lo <= 0 <= hi else min(lo2, hi2)), max(lo2, hi2)
    (x0, x1), (y0, y1) = sq(a, b), sq(c, d)
    return x0 + y0 - 1, x1 + y1 - 1


@pytest.mark.parametrize("target", [0, 1, 2])
def test_accuracy_bullets_circle(target):
    """Cor. guarantees: with a valid tolerance the sample-in-center plot is an
    epsilon-accurate plot (Def. accurate_plot).  f = x^2 + y^2 - 1 on
    [-2, 2]^2 at 64: a point within the pixel radius 1/32 (l_inf) of a centre
    changes f by less than 2 * 4 * (1/32) = 1/4, so every eps >= 1/4 is valid;
    eps = 258/1024 is one that some centre values equal exactly (centre values
    are (a^2 + b^2 - 1024)/1024 with a, b odd).  The pixel errors come from f's
    exact range over each closed cell: distance to {0} (target 0) or to
    (-inf, 0] (targets 1, 2)."""
    rel = inputs.Relation((0, 1), 2, np.array([-1.0, 0, 0, 1.0, 0, 1.0]), target)
    eps = 258 / 1024
    A = oracle.plot_relation(rel, [(-2.0, 2.0, 64)] * 2, rule="center", eps=eps)
    edges = [Fr(-2) + Fr(k, 16) for k in range(65)]
    e = Fr(eps)
    n_on = 0
    for i in range(64):
        for j in range(64):
            lo, hi = _circle_range(edges[i], edges[i + 1], edges[j], edges[j + 1])
            if target == 0:
                dmin = Fr(0) if lo <= 0 <= hi else min(abs(lo), abs(hi))
                dmax = max(abs(lo), abs(hi))
            else:
                dmin, dmax = max(lo, Fr(0)), max(hi, Fr(0))
            if dmin == 0:
                assert A[i, j] == 1, (i, j)               # the pixel error achieves 0
            if dmin > e:
                assert A[i, j] == 0, (i, j)               # always above eps
            if A[i, j]:
                assert dmax <= 2 * e, (i, j)              # bounded by 2 eps
            n_on += int(A[i, j])
    assert n_on > 100
    # centres where the distance equals eps exactly (dyadic values): the
    # closed interval of "achieves" sets them; for f < 0 the distances to the
    # open target form the open ray (f(c), inf), which misses eps
    cs = _exact_centers(-2.0, 2.0, 64)
    ties = [(i, j) for i in range(64) for j in range(64)
            if (abs(cs[i] ** 2 + cs[j] ** 2 - 1) if target == 0 else cs[i] ** 2 + cs[j] ** 2 - 1) == e]
    assert ties
    assert all(A[t] == (1 if target < 2 else 0) for t in ties)


def test_accuracy_bullets_sphere():
    """The same bullets for x^2 + y^2 + z^2 - 1 = 0 on [-2, 2]^3 at 16 (pixel
    radius 1/8, valid eps = 3 * 4 * (1/8) = 3/2)."""
    c = np.zeros(inputs.n_monomials(3, 2))
    c[0] = -1.0
    c[4] = c[7] = c[9] = 1.0         # x^2, y^2, z^2 (graded-lex: 1, x, y, z, x2, xy, xz, y2, yz, z2)
    rel = inputs.Relation((0, 1, 2), 2, c)
    eps = 1.5
    A = oracle.plot_center(rel, [(-2.0, 2.0, 16)] * 3, eps)
    edges = [Fr(-2) + Fr(k, 4) for k in range(17)]

    def sq(lo, hi):
        return (Fr(0) if lo <= 0 <= hi else min(lo * lo, hi * hi)), max(lo * lo, hi * hi)
    for idx in np.ndindex(16, 16, 16):
        rs = [sq(edges[i], edges[i + 1]) for i in idx]
        lo, hi = sum(r[0] for r in rs) - 1, sum(r[1] for r in rs) - 1
        dmin = Fr(0) if lo <= 0 <= hi else min(abs(lo), abs(hi))
        dmax = max(abs(lo), abs(hi))
        if dmin == 0:
            assert A[idx] == 1
        if dmin > Fr(eps):
            assert A[idx] == 0
        if A[idx]:
            assert dmax <= 2 * Fr(eps)


def test_center_plot_random_cubics_against_exact_centres():
    """Random cubics on a dyadic grid (centres exact): the plot equals the
    definition evaluated with exact rationals wherever no centre value lies
    within the FP64 evaluation error (1e-9 here) of the threshold; targets
    f <= eps and f < eps differ only where f(c) == eps."""
    for seed in range(3):
        rng = inputs.SplitMix64(7000 + seed)
        coef = rng.normals(10)
        rel = inputs.Relation((0, 1), 3, coef)
        ax = [(-3.0, 3.0, 24), (-3.0, 3.0, 40)]
        grids = [_exact_centers(*a) for a in ax]
        exps = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (3, 0), (2, 1), (1, 2), (0, 3)]
        cf = [Fr(x) for x in coef]
        for target in (0, 1, 2):
            eps = 0.3
            got = oracle.plot_center(rel, ax, eps, target)
            for i in range(24):
                for j in range(40):
                    x, y = grids[0][i], grids[1][j]
                    v = sum(c * x ** a * y ** b for c, (a, b) in zip(cf, exps))
                    d = abs(v) if target == 0 else v
                    if abs(d - Fr(eps)) < Fr(1, 10 ** 9):
                        continue
                    assert got[i, j] == (d <= Fr(eps) if target < 2 else d < Fr(eps)), (seed, target, i, j)


@pytest.mark.parametrize("target", [1, 2])
def test_inequality_corner_plot_brute_force(target):
    """Corner plot of the disk x^2 + y^2 <= 1 (target 1) and < 1 (target 2) on
    [-2, 2]^2 at 64: every corner value is exact, so the plot equals brute
    force over exact corners; the two differ exactly at cells whose only
    satisfying corners lie on the circle (the four points (+-1, 0), (0, +-1)),
    and every set cell's closure meets the region (exact range)."""
    rel = inputs.Relation((0, 1), 2, np.array([-1.0, 0, 0, 1.0, 0, 1.0]), target)
    A = oracle.plot_relation(rel, [(-2.0, 2.0, 64)] * 2)
    edges = [Fr(-2) + Fr(k, 16) for k in range(65)]
    ref = np.zeros((64, 64), dtype=np.uint8)
    for i in range(64):
        for j in range(64):
            hit = False
            for di in (0, 1):
                for dj in (0, 1):
                    v = edges[i + di] ** 2 + edges[j + dj] ** 2 - 1
                    hit = hit or (v <= 0 if target == 1 else v < 0)
            ref[i, j] = hit
            if hit:
                assert _circle_range(edges[i], edges[i + 1], edges[j], edges[j + 1])[0] <= 0
    assert np.array_equal(A, ref)
    if target == 2:
        le = oracle.plot_ineq(inputs.Relation((0, 1), 2, rel.coef), [(-2.0, 2.0, 64)] * 2, 1)
        diff = np.argwhere(le != A)
        # cells touching the disk only at one of the four exact-zero corners
        assert len(diff) == 8 and np.all(le >= A)


def test_inequality_contains_equation_plot():
    """A cell where f changes sign (corner plot of f = 0) has a corner with
    f <= 0, so the plot of f <= 0 contains it; f < 0 contains every sign-change
    cell with a strictly negative corner."""
    for seed in range(4):
        rng = inputs.SplitMix64(7100 + seed)
        rel = inputs.Relation((0, 1, 2), 3, rng.normals(20))
        ax = [(-3.0, 3.0, 12), (-3.0, 3.0, 10), (-3.0, 3.0, 14)]
        eq = oracle.plot(rel, ax)[0]
        le = oracle.plot_ineq(rel, ax, 1)
        lt = oracle.plot_ineq(rel, ax, 2)
        assert np.all(le >= eq) and np.all(le >= lt)
        assert eq.sum() > 0 and lt.sum() < le.sum() + 1
