"""Pins for the oracle's plotting (Sec. 3.2): closed forms, exact arithmetic
and special cases, each independent of the oracle's own code."""
from fractions import Fraction as Fr
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_1609_00061_amd import inputs

U64 = 2.0 ** -53


# ------------------------------------------------------------------- axes
@pytest.mark.parametrize("lo,hi,r", [(-2.0, 2.0, 64), (-3.0, 3.0, 1024), (-3.0, 3.0, 256), (0.0, 1.0, 7)])
def test_axis_step_form(lo, hi, r):
    """eqn Pixel_def: pixel boundaries a + delta*k with delta = (b-a)/r."""
    x = oracle.axis(lo, hi, r)
    assert x[0] == lo
    exact = [Fr(lo) + Fr(k) * (Fr(hi) - Fr(lo)) / r for k in range(r + 1)]
    for k in range(r + 1):
        err = abs(Fr(x[k]) - exact[k])
        # two roundings (delta, then k*delta and the add): a few ulps of the span
        assert err <= Fr(4) * Fr(U64) * (abs(Fr(lo)) + abs(Fr(hi)) + 1)
    if (hi - lo) / r == 2.0 ** round(math.log2((hi - lo) / r)):      # dyadic step: exact
        assert all(Fr(x[k]) == exact[k] for k in range(r + 1))
    assert np.all(np.diff(x) > 0)


# -------------------------------------------------------- monomial order
BIVARIATE_D3 = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (3, 0), (2, 1), (1, 2), (0, 3)]
TRIVARIATE_D2 = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (1, 1, 0), (1, 0, 1),
                 (0, 2, 0), (0, 1, 1), (0, 0, 2)]


@pytest.mark.parametrize("arity,degree,exps", [(2, 3, BIVARIATE_D3), (3, 2, TRIVARIATE_D2)])
def test_graded_lex_basis(arity, degree, exps):
    """Coefficient m multiplies the m-th monomial of the graded-lex list."""
    assert oracle.n_monomials(arity, degree) == len(exps)
    pt = [1.5, -0.75, 2.25][:arity]
    for m, e in enumerate(exps):
        c = np.zeros(len(exps))
        c[m] = 1.0
        expect = 1.0
        for xi, ei in zip(pt, e):
            expect *= xi ** ei          # exact: short dyadic operands
        assert oracle.eval_poly(arity, degree, c, pt) == expect


def _exact_poly(arity, degree, coef, pt):
    """Sum of c_m x^m over the graded-lex monomials, in exact rationals, plus
    the sum of |c_m x^m|.  Monomials are enumerated independently here."""
    exps = []
    for D in range(degree + 1):
        for e in itertools.product(range(D, -1, -1), repeat=arity):
            if sum(e) == D:
                exps.append(e)
    # product(range(D..0)) gives lexicographically descending tuples
    total, absum = Fr(0), Fr(0)
    for c, e in zip(coef, exps):
        t = Fr(c)
        for xi, ei in zip(pt, e):
            t *= Fr(xi) ** ei
        total += t
        absum += abs(t)
    return total, absum


@pytest.mark.parametrize("arity", [1, 2, 3])
def test_canonical_value_within_fp64_bound(arity):
    """The canonical FP64 value differs from the exact polynomial by at most
    gamma_K * sum|c_m x^m| (Higham's Horner bound, K = 2d + n roundings)."""
    degree = 3
    rng = inputs.SplitMix64(1234 + arity)
    K = 2 * degree + arity
    gamma = Fr(K) * Fr(U64) / (1 - Fr(K) * Fr(U64))
    for _ in range(200):
        coef = rng.normals(oracle.n_monomials(arity, degree))
        pt = [rng.uniform() * 6 - 3 for _ in range(arity)]
        f = oracle.eval_poly(arity, degree, coef, pt)
        exact, absum = _exact_poly(arity, degree, coef, pt)
        assert abs(Fr(f) - exact) <= gamma * absum


def test_canonical_value_exact_for_short_dyadics():
    """With small dyadic data every fma is exact, so the value equals the
    polynomial exactly."""
    rng = inputs.SplitMix64(99)
    for arity in (1, 2, 3):
        for _ in range(50):
            n = oracle.n_monomials(arity, 3)
            coef = [rng.randint(-8, 8) / 4 for _ in range(n)]
            pt = [rng.randint(-12, 12) / 4 for _ in range(arity)]
            exact, _ = _exact_poly(arity, 3, coef, pt)
            assert Fr(oracle.eval_poly(arity, 3, np.array(coef), pt)) == exact


# ---------------------------------------------------------- closed forms
def _grid(lo, hi, r):
    return [Fr(lo) + Fr(k) * (Fr(hi) - Fr(lo)) / r for k in range(r + 1)]


def _sq_range(a, b):
    """Range of t^2 over [a, b]."""
    lo = Fr(0) if a <= 0 <= b else min(a * a, b * b)
    return lo, max(a * a, b * b)


def circle_cells(r=64, lo=-2, hi=2):
    """Closed cells of [lo,hi]^2 meeting x^2 + y^2 = 1 (exact)."""
    g = _grid(lo, hi, r)
    out = np.zeros((r, r), dtype=np.uint8)
    for i in range(r):
        xl, xh = _sq_range(g[i], g[i + 1])
        for j in range(r):
            yl, yh = _sq_range(g[j], g[j + 1])
            out[i, j] = (xl + yl <= 1 <= xh + yh)
    return out


def _cubic_g(z):
    return z ** 3 - z / 2


class _Q:
    """Numbers q + s*sqrt(1/54) with q rational and s in {-1, 0, 1}, exactly
    comparable with rationals (the critical values of z^3 - z/2 are
    -+1/(3 sqrt 6) = -+sqrt(1/54))."""

    def __init__(self, q=Fr(0), s=0):
        self.q, self.s = Fr(q), s

    def le(self, t):      # self <= t for rational t
        d = Fr(t) - self.q     # need s*sqrt(1/54) <= d
        if self.s == 0:
            return d >= 0
        if self.s > 0:
            return d >= 0 and d * d >= Fr(1, 54)
        return d >= 0 or d * d <= Fr(1, 54)

    def ge(self, t):      # self >= t
        d = Fr(t) - self.q     # need s*sqrt(1/54) >= d
        if self.s == 0:
            return d <= 0
        if self.s > 0:
            return d <= 0 or d * d <= Fr(1, 54)
        return d <= 0 and d * d >= Fr(1, 54)


def _contains_crit(a, b, sign):
    """Is sign/sqrt(6) in [a, b]?"""
    if sign > 0:
        return (a <= 0 or a * a <= Fr(1, 6)) and b >= 0 and b * b >= Fr(1, 6)
    return a <= 0 and a * a >= Fr(1, 6) and (b >= 0 or b * b <= Fr(1, 6))


def cubic_cells(r=64, lo=-2, hi=2):
    """Closed cells [y_i,y_i+1] x [z_j,z_j+1] meeting y = z^3 - z/2 (exact)."""
    g = _grid(lo, hi, r)
    out = np.zeros((r, r), dtype=np.uint8)
    for j in range(r):
        a, b = g[j], g[j + 1]
        cands = [_Q(_cubic_g(a)), _Q(_cubic_g(b))]
        if _contains_crit(a, b, +1):
            cands.append(_Q(0, -1))          # g(1/sqrt6) = -sqrt(1/54)
        if _contains_crit(a, b, -1):
            cands.append(_Q(0, +1))
        for i in range(r):
            yl, yh = g[i], g[i + 1]
            # range [min, max] of g meets [yl, yh] iff min <= yh and max >= yl
            has_low = any(c.le(yh) for c in cands)
            has_high = any(c.ge(yl) for c in cands)
            out[i, j] = has_low and has_high
    return out


def projection_cells(r=64, lo=-2, hi=2):
    """Closed (x, z) cells meeting {x^2 + g(z)^2 = 1}, the exact solution set of
    C1 on the exposed variables (exact rationals)."""
    grid = _grid(lo, hi, r)
    out = np.zeros((r, r), dtype=np.uint8)
    for k in range(r):
        a, b = grid[k], grid[k + 1]
        vals = [_cubic_g(a) ** 2, _cubic_g(b) ** 2]
        if a <= 0 <= b:
            vals.append(Fr(0))
        if (a <= 0 or a * a <= Fr(1, 2)) and b >= 0 and b * b >= Fr(1, 2):
            vals.append(Fr(0))                 # root +1/sqrt2
        if a <= 0 and a * a >= Fr(1, 2) and (b >= 0 or b * b <= Fr(1, 2)):
            vals.append(Fr(0))                 # root -1/sqrt2
        if _contains_crit(a, b, +1) or _contains_crit(a, b, -1):
            vals.append(Fr(1, 54))
        g2lo, g2hi = min(vals), max(vals)
        if g2lo > 1:
            continue
        need_lo, need_hi = 1 - min(g2hi, Fr(1)), 1 - g2lo     # range of x^2
        for i in range(r):
            sl, sh = _sq_range(grid[i], grid[i + 1])
            out[i, k] = (sl <= need_hi and sh >= need_lo)
    return out


@pytest.fixture(scope="module")
def c1():
    return inputs.config1()


def test_c1_circle_plot_equals_closed_cells(c1):
    """Corner rule = 'closed cell meets the circle' (x^2 + y^2 is monotone on
    each cell because 0 is a grid line): 132 cells."""
    A, nz = oracle.plot(c1.relations[0], c1.axes)
    ref = circle_cells()
    assert ref.sum() == 132
    assert np.array_equal(A, ref)
    assert nz == 4                          # (+-1, 0), (0, +-1)


def test_c1_cubic_plot_equals_closed_cells(c1):
    """Corner rule = 'closed cell meets y = z^3 - z/2' (the extrema at
    z = -+1/sqrt6 stay inside their y-cells): 124 cells."""
    B, nz = oracle.plot(c1.relations[1], c1.axes)
    ref = cubic_cells()
    assert ref.sum() == 124
    assert np.array_equal(B, ref)
    assert nz == 5                          # z in {0, +-1/2, +-1} with y = g(z) a grid value


def test_c1_solution_closed_form(c1):
    """Whole C1 solve: the output equals the Boolean product of the two exact
    cell sets (numpy integer matmul > 0, fn. to Sec. 2.2: N-semiring counts),
    and contains every cell of the exact projection x^2 + g(z)^2 = 1 (no false
    negatives, proof of Thm 'extended', first bullet)."""
    A, _ = oracle.plot(c1.relations[0], c1.axes)
    B, _ = oracle.plot(c1.relations[1], c1.axes)
    out = oracle.solve([64, 64, 64], [(0, 1), (1, 2)], [A, B], (0, 2))
    ref = (circle_cells().astype(np.int64) @ cubic_cells().astype(np.int64)) > 0
    assert out.sum() == 180
    assert np.array_equal(out.astype(bool), ref)
    proj = projection_cells()
    assert proj.sum() == 144
    assert np.all(out[proj.astype(bool)] == 1)


def test_ellipsoid_closed_form():
    """Trivariate: x^2 + 2y^2 + 4z^2 = 1 on [-2,2]^3 at r=16 (0 a grid line, so
    the function is monotone on every cell); asymmetric, so a transposed axis
    fails."""
    coef = np.array([-1.0, 0, 0, 0, 1.0, 0, 0, 2.0, 0, 4.0])
    rel = inputs.Relation((0, 1, 2), 2, coef)
    r = 16
    axes = [(-2.0, 2.0, r)] * 3
    P, nz = oracle.plot(rel, axes)
    g = _grid(-2, 2, r)
    ref = np.zeros((r, r, r), dtype=np.uint8)
    for i in range(r):
        xl, xh = _sq_range(g[i], g[i + 1])
        for j in range(r):
            yl, yh = _sq_range(g[j], g[j + 1])
            for k in range(r):
                zl, zh = _sq_range(g[k], g[k + 1])
                ref[i, j, k] = (xl + 2 * yl + 4 * zl <= 1 <= xh + 2 * yh + 4 * zh)
    assert np.array_equal(P, ref)
    # exact zero corners: grid points with x^2 + 2y^2 + 4z^2 = 1, quarter steps
    zc = sum(1 for a in g for b in g for c in g if a * a + 2 * b * b + 4 * c * c == 1)
    assert nz == zc


def test_plot_uneven_axes_graph():
    """A graph y = x^2/4 - 1/2 on a non-square grid with different boxes per
    axis: corner rule = closed cell meets the graph (g monotone on each cell
    because 0 is an x grid line)."""
    rel = inputs.Relation((0, 1), 2, np.array([-0.5, 0, -1.0, 0.25, 0, 0]))
    axes = [(-2.0, 2.0, 8), (-1.0, 1.0, 16)]
    P, _ = oracle.plot(rel, axes)
    gx, gy = _grid(-2, 2, 8), _grid(-1, 1, 16)
    ref = np.zeros((8, 16), dtype=np.uint8)
    for i in range(8):
        sl, sh = _sq_range(gx[i], gx[i + 1])
        for j in range(16):
            ref[i, j] = (sl / 4 - Fr(1, 2) <= gy[j + 1] and sh / 4 - Fr(1, 2) >= gy[j])
    assert np.array_equal(P, ref)


def test_plot_nan_corner_counts_as_neither():
    """A corner whose value is NaN turns on no pixel by itself (Sec. 2.4, the
    plotting function refrains where the relation is undefined)."""
    # 1e308*x^3 - 1e308*y^3 overflows to inf - inf = NaN where both cubes are big
    coef = np.zeros(10)
    coef[6], coef[9] = 1e308, -1e308
    rel = inputs.Relation((0, 1), 3, coef)
    axes = [(2.0, 3.0, 1), (2.0, 3.0, 1)]
    vals = oracle.corner_values(rel, axes)
    assert np.isnan(vals[1, 1])
    P, _ = oracle.plot(rel, axes)
    f = vals.ravel()
    le = np.any(f[~np.isnan(f)] <= 0)
    ge = np.any(f[~np.isnan(f)] >= 0)
    assert P[0, 0] == (le and ge)
