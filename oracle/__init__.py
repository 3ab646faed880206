"""CPU oracle for the pixel array method -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The product library never does, and this
package never imports the product library.  Inputs are plain numbers (axes,
coefficient arrays, byte arrays); the seeded instance generator lives in its
own module and holds none of the method's arithmetic.

Contents (each function cites the paper passage it follows):
  axis, eval_poly, corner_values, plot   -- Sec. 3.2 plotting (C, pa_oracle.c)
  plot_ineq                              -- corner plot of f <= 0 / f < 0 (C)
  centers, plot_center                   -- Def. sample_in_center (C)
  plot_relation                          -- dispatch on rule and target
  contract                               -- Sec. 3.3 GAM of a two-pack cluster (C)
  contract_count, alg1_literal_count     -- the same in the semiring N (counts)
  solve_entries, solve                   -- eqn GAM for a whole diagram with
                                            short-circuit AND/OR (C)
  alg1_literal                           -- Alg. "Generalized array
                                            multiplication" verbatim in Python
                                            (tiny inputs only)
  solve_pairwise                         -- a clustering (Sec. 3.5) executed as
                                            a sequence of two-pack GAMs
"""
from __future__ import annotations

import ctypes
import itertools
import os
from typing import Dict, List, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

DEFAULT_THREADS = max(1, min(16, os.cpu_count() or 1))


def build_lib(force: bool = False) -> str:
    """Compile pa_oracle.c with gcc (no FMA contraction, IEEE semantics)."""
    from .build import build_oracle
    return build_oracle(force=force)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_lib()
        L = ctypes.CDLL(_LIB_PATH)
        dp, ip, ucp = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int), ctypes.c_void_p
        L.orc_axis.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, dp]
        L.orc_axis.restype = ctypes.c_int
        L.orc_eval.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
        L.orc_eval.restype = ctypes.c_double
        L.orc_n_monomials.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_n_monomials.restype = ctypes.c_long
        L.orc_corner_values.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, ip, dp, ctypes.c_int]
        L.orc_corner_values.restype = ctypes.c_int
        L.orc_plot.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, ip, ucp,
                               ctypes.POINTER(ctypes.c_longlong), ctypes.c_int]
        L.orc_plot.restype = ctypes.c_int
        L.orc_plot_ineq.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, ip, ctypes.c_int, ucp, ctypes.c_int]
        L.orc_plot_ineq.restype = ctypes.c_int
        L.orc_centers.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, dp]
        L.orc_centers.restype = ctypes.c_int
        L.orc_plot_center.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, ip, ctypes.c_double, ctypes.c_int,
                                      ucp, ctypes.c_int]
        L.orc_plot_center.restype = ctypes.c_int
        L.orc_contract_count.argtypes = [ucp, ctypes.c_int, ip, ucp, ctypes.c_int, ip, ctypes.c_int, ip, ip, ucp]
        L.orc_contract_count.restype = ctypes.c_int
        L.orc_contract.argtypes = [ucp, ctypes.c_int, ip, ucp, ctypes.c_int, ip,
                                   ctypes.c_int, ip, ip, ucp, ctypes.c_int]
        L.orc_contract.restype = ctypes.c_int
        L.orc_solve_entries.argtypes = [ctypes.c_int, ip, ctypes.c_int, ip, ip,
                                        ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ip,
                                        ctypes.c_long, ip, ucp, ctypes.c_int]
        L.orc_solve_entries.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _i32(seq):
    return np.ascontiguousarray(np.asarray(seq, dtype=np.int32))


# ------------------------------------------------------------------ plotting
def axis(lo: float, hi: float, r: int) -> np.ndarray:
    """Pixel boundaries x_k = lo + k * ((hi - lo) / r), k = 0..r (eqn Pixel_def)."""
    x = np.empty(r + 1, dtype=np.float64)
    if lib().orc_axis(float(lo), float(hi), int(r), _dp(x)):
        raise ValueError("bad axis")
    return x


def n_monomials(arity: int, degree: int) -> int:
    return int(lib().orc_n_monomials(arity, degree))


def eval_poly(arity: int, degree: int, coef: np.ndarray, pt: Sequence[float]) -> float:
    """Canonical FP64 value (nested fma Horner in declared variable order)."""
    c = np.ascontiguousarray(coef, dtype=np.float64)
    x = np.ascontiguousarray(pt, dtype=np.float64)
    return float(lib().orc_eval(arity, degree, _dp(c), _dp(x)))


def _rel_axes(rel, axes):
    lo = np.array([axes[v][0] for v in rel.vars], dtype=np.float64)
    hi = np.array([axes[v][1] for v in rel.vars], dtype=np.float64)
    res = _i32([axes[v][2] for v in rel.vars])
    return lo, hi, res


def corner_values(rel, axes, nthreads: int = DEFAULT_THREADS) -> np.ndarray:
    """FP64 value at every corner, shape (r_0+1, ..., r_{n-1}+1), declared order."""
    lo, hi, res = _rel_axes(rel, axes)
    vals = np.empty(tuple(int(r) + 1 for r in res), dtype=np.float64)
    c = np.ascontiguousarray(rel.coef, dtype=np.float64)
    if lib().orc_corner_values(len(rel.vars), rel.degree, _dp(c), _dp(lo), _dp(hi), _ip(res),
                               _dp(vals), nthreads):
        raise ValueError("bad relation")
    return vals


def plot(rel, axes, nthreads: int = DEFAULT_THREADS) -> Tuple[np.ndarray, int]:
    """Corner sign-change plot of f = 0 (Sec. 3.2, corner rule): one byte per
    cell, shape (r_0, ..., r_{n-1}) in the relation's declared order.  Returns
    (array, number of corners with f == 0 exactly)."""
    lo, hi, res = _rel_axes(rel, axes)
    out = np.empty(tuple(int(r) for r in res), dtype=np.uint8)
    nz = ctypes.c_longlong(0)
    c = np.ascontiguousarray(rel.coef, dtype=np.float64)
    rc = lib().orc_plot(len(rel.vars), rel.degree, _dp(c), _dp(lo), _dp(hi), _ip(res),
                        out.ctypes.data, ctypes.byref(nz), nthreads)
    if rc:
        raise ValueError(f"orc_plot failed ({rc})")
    return out, int(nz.value)


def plot_ineq(rel, axes, target: int, nthreads: int = DEFAULT_THREADS) -> np.ndarray:
    """Corner plot of f <= 0 (target 1) or f < 0 (target 2) (Sec. 3.2): a cell is
    set iff one of its corners satisfies the inequality."""
    lo, hi, res = _rel_axes(rel, axes)
    out = np.empty(tuple(int(r) for r in res), dtype=np.uint8)
    c = np.ascontiguousarray(rel.coef, dtype=np.float64)
    if lib().orc_plot_ineq(len(rel.vars), rel.degree, _dp(c), _dp(lo), _dp(hi), _ip(res), int(target),
                           out.ctypes.data, nthreads):
        raise ValueError("orc_plot_ineq failed")
    return out


def centers(lo: float, hi: float, r: int) -> np.ndarray:
    """Pixel centres lo + (k + 1/2) * ((hi - lo) / r), k = 0..r-1 (eqn Pixel_def)."""
    x = np.empty(r, dtype=np.float64)
    if lib().orc_centers(float(lo), float(hi), int(r), _dp(x)):
        raise ValueError("bad axis")
    return x


def plot_center(rel, axes, eps: float, target: int = 0, nthreads: int = DEFAULT_THREADS) -> np.ndarray:
    """epsilon-tolerance sample-in-center plot (Def. sample_in_center): a cell
    is set iff the distance of f(centre) to the target set is at most eps
    (target 0: |f| <= eps; 1: f <= eps; 2: f < eps)."""
    lo, hi, res = _rel_axes(rel, axes)
    out = np.empty(tuple(int(r) for r in res), dtype=np.uint8)
    c = np.ascontiguousarray(rel.coef, dtype=np.float64)
    if lib().orc_plot_center(len(rel.vars), rel.degree, _dp(c), _dp(lo), _dp(hi), _ip(res), float(eps),
                             int(target), out.ctypes.data, nthreads):
        raise ValueError("orc_plot_center failed")
    return out


def plot_relation(rel, axes, rule: str = "corner", eps: float = 0.0, nthreads: int = DEFAULT_THREADS) -> np.ndarray:
    """The plot of a relation under a plotting rule: "corner" (sign change at
    the cell corners for f = 0, a satisfying corner for f <= 0 / f < 0) or
    "center" (the epsilon-tolerance sample-in-center plot).  The relation's
    `target` (0: f = 0, 1: f <= 0, 2: f < 0; 0 if absent) selects the target
    subset."""
    target = int(getattr(rel, "target", 0))
    if rule == "center":
        return plot_center(rel, axes, eps, target, nthreads)
    if target == 0:
        return plot(rel, axes, nthreads)[0]
    return plot_ineq(rel, axes, target, nthreads)


# ------------------------------------------------------------ multiplication
def contract(A: np.ndarray, a_vars: Sequence[int], B: np.ndarray, b_vars: Sequence[int],
             out_vars: Sequence[int], var_res: Dict[int, int], nthreads: int = DEFAULT_THREADS) -> np.ndarray:
    """C(out_vars) = OR over entries of vars(A) u vars(B) of A AND B (eqn GAM,
    two inner packs).  The entries of A are split over `nthreads` threads; the
    result does not depend on the split (OR is idempotent)."""
    nv = max(list(a_vars) + list(b_vars) + list(out_vars) + [0]) + 1
    res = _i32([var_res.get(v, 1) for v in range(nv)])
    A = np.asarray(A, dtype=np.uint8, order="C")
    B = np.asarray(B, dtype=np.uint8, order="C")
    assert A.shape == tuple(var_res[v] for v in a_vars)
    assert B.shape == tuple(var_res[v] for v in b_vars)
    C = np.empty(tuple(var_res[v] for v in out_vars), dtype=np.uint8)
    av, bv, cv = _i32(a_vars), _i32(b_vars), _i32(out_vars)
    rc = lib().orc_contract(A.ctypes.data, len(a_vars), _ip(av), B.ctypes.data, len(b_vars), _ip(bv),
                            len(out_vars), _ip(cv), _ip(res), C.ctypes.data, int(nthreads))
    if rc:
        raise ValueError(f"orc_contract failed ({rc})")
    return C


def contract_count(A: np.ndarray, a_vars: Sequence[int], B: np.ndarray, b_vars: Sequence[int],
                   out_vars: Sequence[int], var_res: Dict[int, int]) -> np.ndarray:
    """C(out_vars) = sum over entries of vars(A) u vars(B) of A * B in the
    semiring N (uint64, saturating): the count-semiring GAM of two packs."""
    nv = max(list(a_vars) + list(b_vars) + list(out_vars) + [0]) + 1
    res = _i32([var_res.get(v, 1) for v in range(nv)])
    A = np.asarray(A, dtype=np.uint64, order="C")      # keeps a 0-dim array 0-dim
    B = np.asarray(B, dtype=np.uint64, order="C")
    assert A.shape == tuple(var_res[v] for v in a_vars)
    assert B.shape == tuple(var_res[v] for v in b_vars)
    C = np.empty(tuple(var_res[v] for v in out_vars), dtype=np.uint64)
    av, bv, cv = _i32(a_vars), _i32(b_vars), _i32(out_vars)
    rc = lib().orc_contract_count(A.ctypes.data, len(a_vars), _ip(av), B.ctypes.data, len(b_vars), _ip(bv),
                                  len(out_vars), _ip(cv), _ip(res), C.ctypes.data)
    if rc:
        raise ValueError(f"orc_contract_count failed ({rc})")
    return C


def alg1_literal_count(var_res: Sequence[int], rel_vars: Sequence[Sequence[int]],
                       arrays: Sequence[np.ndarray], exposed: Sequence[int]) -> np.ndarray:
    """Alg. "Generalized array multiplication" as printed, in the semiring N:
    A'(Entr'(e)) += prod_i A_i(Entr^i(e)) over every link entry e.  Python
    integers; tiny inputs."""
    out = np.zeros(tuple(int(var_res[v]) for v in exposed), dtype=object)
    for e in itertools.product(*[range(int(r)) for r in var_res]):
        a_e = 1
        for A, vs in zip(arrays, rel_vars):
            a_e = a_e * int(A[tuple(e[v] for v in vs)])
        ep = tuple(e[v] for v in exposed)
        out[ep] = out[ep] + a_e
    return out


def solve_entries(var_res: Sequence[int], rel_vars: Sequence[Sequence[int]],
                  arrays: Sequence[np.ndarray], exposed: Sequence[int],
                  entries: np.ndarray, nthreads: int = DEFAULT_THREADS) -> np.ndarray:
    """A'(e') of eqn GAM for each listed output entry (rows of exposed indices)."""
    res = _i32(var_res)
    nd = _i32([len(v) for v in rel_vars])
    flat = _i32([v for vs in rel_vars for v in vs])
    arrs = [np.asarray(a, dtype=np.uint8, order="C") for a in arrays]
    for a, vs in zip(arrs, rel_vars):
        assert a.shape == tuple(int(var_res[v]) for v in vs)
    ptrs = (ctypes.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
    ent = _i32(entries).reshape(-1, max(1, len(exposed)))
    n = ent.shape[0] if len(exposed) else 1
    out = np.zeros(n, dtype=np.uint8)
    ex = _i32(exposed)
    rc = lib().orc_solve_entries(len(res), _ip(res), len(arrs), _ip(nd), _ip(flat), ptrs,
                                 len(exposed), _ip(ex), n, _ip(ent), out.ctypes.data, nthreads)
    if rc:
        raise ValueError(f"orc_solve_entries failed ({rc})")
    return out


def solve(var_res, rel_vars, arrays, exposed, nthreads: int = DEFAULT_THREADS) -> np.ndarray:
    """The whole output array A' over the exposed variables (eqn GAM)."""
    shape = tuple(int(var_res[v]) for v in exposed)
    if len(exposed) == 0:
        return solve_entries(var_res, rel_vars, arrays, exposed, np.zeros((1, 1)), nthreads).reshape(())
    grids = np.indices(shape).reshape(len(shape), -1).T
    return solve_entries(var_res, rel_vars, arrays, exposed, grids, nthreads).reshape(shape)


def alg1_literal(var_res: Sequence[int], rel_vars: Sequence[Sequence[int]],
                 arrays: Sequence[np.ndarray], exposed: Sequence[int]) -> np.ndarray:
    """Alg. "Generalized array multiplication" as printed: loop over every link
    entry e in Entr(Lambda), a_e = product over packs of A_i(Entr^i(e)), then
    A'(Entr'(e)) += a_e, in the Boolean semiring.  Pure Python; tiny inputs."""
    n = len(var_res)
    out = np.zeros(tuple(int(var_res[v]) for v in exposed), dtype=np.uint8)
    for e in itertools.product(*[range(int(r)) for r in var_res]):
        a_e = 1
        for A, vs in zip(arrays, rel_vars):
            a_e = a_e & int(A[tuple(e[v] for v in vs)])
        ep = tuple(e[v] for v in exposed)
        out[ep] = out[ep] | a_e
    assert n == len(var_res)
    return out


def solve_pairwise(var_res: Dict[int, int], rel_vars: Sequence[Sequence[int]],
                   arrays: Sequence[np.ndarray], exposed: Sequence[int],
                   merges: Sequence[Tuple[int, int]], nthreads: int = DEFAULT_THREADS, log=None) -> np.ndarray:
    """Execute a binary clustering (Sec. 3.5): factors are numbered 0..n-1 for
    the relations, and each merge (i, j) creates factor n, n+1, ... as the GAM of
    factors i and j whose output keeps every variable that is exposed or occurs
    in a factor not yet merged (the intermediate pack Q_C).  Variables private
    to a single relation are projected out first.  The last factor is permuted
    to the exposed order.  Each merge's operands are released once it is done;
    `log`, if given, is called with a line per merge."""
    factors: Dict[int, Tuple[np.ndarray, Tuple[int, ...]]] = {}
    alive = set()
    for i, (A, vs) in enumerate(zip(arrays, rel_vars)):
        factors[i] = (np.asarray(A, dtype=np.uint8), tuple(vs))
        alive.add(i)
    nxt = len(arrays)
    for (i, j) in merges:
        Ai, vi = factors[i]
        Aj, vj = factors[j]
        alive.discard(i)
        alive.discard(j)
        others = set(exposed)
        for k in alive:
            others |= set(factors[k][1])
        keep = tuple(v for v in dict.fromkeys(vi + vj) if v in others)
        C = contract(Ai, vi, Aj, vj, keep, var_res, nthreads)
        del factors[i], factors[j], Ai, Aj
        if log is not None:
            log(f"oracle merge ({i}, {j}) -> factor {nxt} over {keep}")
        factors[nxt] = (C, keep)
        alive.add(nxt)
        nxt += 1
    assert len(alive) == 1, "merges must combine all factors"
    (last,) = alive
    C, vs = factors[last]
    if set(vs) != set(exposed):
        # project out anything left that is not exposed
        C2 = np.ones(tuple(var_res[v] for v in ()), dtype=np.uint8)
        C = contract(C, vs, C2, (), tuple(v for v in vs if v in exposed), var_res, nthreads)
        vs = tuple(v for v in vs if v in exposed)
    perm = [vs.index(v) for v in exposed]
    return np.ascontiguousarray(np.transpose(C, perm)) if len(perm) else C
