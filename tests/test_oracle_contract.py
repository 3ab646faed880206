"""Pins for the oracle's generalized array multiplication (Sec. 3.3): the
printed algorithm run literally, library special cases (matmul, Kronecker,
trace), and the theorems (associativity, monotonicity)."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import planner
from paper_1609_00061_amd import inputs


def _rand(shape, density, seed):
    return inputs.random_bool_array(shape, density, seed)


CASES = [
    # (a_vars, b_vars, out_vars)
    ((0, 1), (1, 2), (0, 2)),            # matmul
    ((0, 1), (1, 2), (2, 0)),            # matmul, transposed output
    ((0, 1, 2), (2, 3), (0, 1, 3)),      # contraction of one index
    ((0, 1, 2), (1, 2, 3), (0, 3)),      # two shared latent indices
    ((0, 1, 2), (0, 2, 3), (0, 1, 3)),   # batch index 0
    ((0, 1), (2, 3), (0, 1, 2, 3)),      # Kronecker
    ((0, 1), (1, 2), ()),                # everything latent: 0-dim output
    ((0, 1, 2), (1,), (0,)),             # pre-reduce of 2, vector
    ((0,), (0,), (0,)),                  # elementwise AND
    ((0, 1), (1, 2), (1,)),              # kept shared index, both others latent
    ((0, 1), (2, 1), (0, 2)),            # B's shared index after its own one
    ((0, 1, 2), (3, 2, 1), (3, 0)),      # two shared indices in reverse order in B
    ((2, 0), (3, 1, 0), (1, 3, 2)),      # B's own indices around the shared one
]


@pytest.mark.parametrize("case", CASES)
def test_pairwise_contract_matches_printed_algorithm(case):
    a_vars, b_vars, out_vars = case
    res = {0: 3, 1: 4, 2: 2, 3: 3}
    for seed in range(4):
        A = _rand([res[v] for v in a_vars], 0.4, 100 + seed)
        B = _rand([res[v] for v in b_vars], 0.4, 200 + seed)
        C = oracle.contract(A, a_vars, B, b_vars, out_vars, res)
        nv = 1 + max(a_vars + b_vars)
        var_res = [res[v] for v in range(nv)]
        # The printed algorithm needs every link in some pack; links outside
        # both packs do not occur here.
        ref = oracle.alg1_literal(var_res, [a_vars, b_vars], [A, B], out_vars)
        assert np.array_equal(C, ref)


@pytest.mark.parametrize("case", CASES)
def test_pairwise_contract_independent_of_threads(case):
    """The contraction's entries of A are split over threads; the output does
    not depend on the split."""
    a_vars, b_vars, out_vars = case
    res = {0: 7, 1: 5, 2: 6, 3: 4}
    A = _rand([res[v] for v in a_vars], 0.3, 300)
    B = _rand([res[v] for v in b_vars], 0.3, 301)
    ref = oracle.contract(A, a_vars, B, b_vars, out_vars, res, nthreads=1)
    for t in (2, 3, 7, 64):
        assert np.array_equal(oracle.contract(A, a_vars, B, b_vars, out_vars, res, nthreads=t), ref), t


def test_matmul_special_case():
    """Thm after eqn GAM: the diagram M, N -> MN is matrix multiplication; in
    the Boolean semiring the product is (integer product > 0)."""
    res = {0: 37, 1: 29, 2: 41}
    for seed in range(3):
        M = _rand((37, 29), 0.08, seed)
        N = _rand((29, 41), 0.08, 50 + seed)
        C = oracle.contract(M, (0, 1), N, (1, 2), (0, 2), res)
        ref = (M.astype(np.int64) @ N.astype(np.int64)) > 0
        assert np.array_equal(C.astype(bool), ref)


def test_kronecker_special_case():
    """Diagram M1, M2 -> M1 (x) M2 with no shared link: AND outer product."""
    res = {0: 5, 1: 6, 2: 3, 3: 4}
    M1 = _rand((5, 6), 0.5, 7)
    M2 = _rand((3, 4), 0.5, 8)
    C = oracle.contract(M1, (0, 1), M2, (2, 3), (0, 1, 2, 3), res)
    ref = np.multiply.outer(M1, M2)
    assert np.array_equal(C, ref)


def test_trace_special_case():
    """Diagram P -> Tr(P): both ports of P wired to one link; the printed
    algorithm gives OR of the diagonal (numpy trace of the 0/1 matrix > 0)."""
    for seed in range(5):
        P = _rand((6, 6), 0.15, 300 + seed)
        out = oracle.alg1_literal([6], [(0, 0)], [P], ())
        assert int(out) == int(np.trace(P.astype(np.int64)) > 0)


def _random_system(seed, n_vars=5, n_rel=4, r=3, density=0.45):
    rng = inputs.SplitMix64(seed)
    rel_vars = []
    for _ in range(n_rel):
        a = rng.randint(1, 3)
        vs = []
        while len(vs) < a:
            v = rng.randint(0, n_vars - 1)
            if v not in vs:
                vs.append(v)
        rel_vars.append(tuple(vs))
    covered = sorted(set(v for vs in rel_vars for v in vs))
    n_exp = rng.randint(0, min(2, len(covered)))
    exposed = []
    while len(exposed) < n_exp:
        v = covered[rng.randint(0, len(covered) - 1)]
        if v not in exposed:
            exposed.append(v)
    var_res = [r + (v % 2) for v in range(n_vars)]
    # variables not in any relation get resolution 1 so Entr(Lambda) is unchanged
    for v in range(n_vars):
        if v not in covered:
            var_res[v] = 1
    arrays = [_rand([var_res[v] for v in vs], density, seed * 31 + i) for i, vs in enumerate(rel_vars)]
    return var_res, rel_vars, arrays, tuple(exposed)


@pytest.mark.parametrize("seed", range(12))
def test_whole_diagram_formula_matches_printed_algorithm(seed):
    var_res, rel_vars, arrays, exposed = _random_system(seed)
    ref = oracle.alg1_literal(var_res, rel_vars, arrays, exposed)
    out = oracle.solve(var_res, rel_vars, arrays, exposed, nthreads=2)
    assert np.array_equal(out, ref)


@pytest.mark.parametrize("seed", range(6))
def test_associativity_every_binary_clustering(seed):
    """Thm 'associative': every cluster tree gives the same array."""
    var_res, rel_vars, arrays, exposed = _random_system(100 + seed)
    ref = oracle.solve(var_res, rel_vars, arrays, exposed, nthreads=2)
    res = {v: var_res[v] for v in range(len(var_res))}
    n = len(rel_vars)
    seen = 0
    for tree in planner.all_binary_trees(list(range(n))):
        merges = []
        nxt = [n]

        def emit(t):
            if isinstance(t, int):
                return t
            a, b = emit(t[0]), emit(t[1])
            merges.append((a, b))
            nxt[0] += 1
            return nxt[0] - 1
        emit(tree)
        out = oracle.solve_pairwise(res, rel_vars, arrays, exposed, merges)
        assert np.array_equal(out, ref), tree
        seen += 1
    assert seen >= 1


@pytest.mark.parametrize("seed", range(6))
def test_monotonicity(seed):
    """Thm 'associative': A <= B entrywise implies Arr(Phi)(A) <= Arr(Phi)(B)."""
    var_res, rel_vars, arrays, exposed = _random_system(200 + seed, density=0.3)
    base = oracle.solve(var_res, rel_vars, arrays, exposed, nthreads=2)
    more = [a | _rand(a.shape, 0.2, 999 + i + seed) for i, a in enumerate(arrays)]
    grown = oracle.solve(var_res, rel_vars, more, exposed, nthreads=2)
    assert np.all(grown >= base)


def test_solve_entries_sampled_equals_full():
    var_res, rel_vars, arrays, exposed = _random_system(7, n_vars=6, n_rel=5, r=4)
    if len(exposed) == 0:
        exposed = (rel_vars[0][0],)
    full = oracle.solve(var_res, rel_vars, arrays, exposed)
    ent = np.indices(full.shape).reshape(len(exposed), -1).T[::3]
    part = oracle.solve_entries(var_res, rel_vars, arrays, exposed, ent)
    assert np.array_equal(part, full[tuple(ent.T)])


# ------------------------------------------------------------ count semiring
@pytest.mark.parametrize("case", CASES)
def test_count_contract_matches_printed_algorithm(case):
    """The printed algorithm run in the semiring N (sum of products over every
    link entry) equals the oracle's count contraction, on 0/1 inputs (plots)
    and on small integer inputs (intermediate counts)."""
    a_vars, b_vars, out_vars = case
    res = {0: 3, 1: 4, 2: 2, 3: 3}
    for seed in range(3):
        A = _rand([res[v] for v in a_vars], 0.5, 400 + seed).astype(np.uint64)
        B = _rand([res[v] for v in b_vars], 0.5, 500 + seed).astype(np.uint64)
        if seed == 2:
            A = A * np.uint64(3) + _rand(A.shape, 0.5, 600).astype(np.uint64)
            B = B * np.uint64(5)
        C = oracle.contract_count(A, a_vars, B, b_vars, out_vars, res)
        nv = 1 + max(a_vars + b_vars)
        ref = oracle.alg1_literal_count([res[v] for v in range(nv)], [a_vars, b_vars], [A, B], out_vars)
        assert np.array_equal(C.astype(object), ref)


def test_count_matmul_special_case():
    """Thm after eqn GAM in N: M, N -> MN is integer matrix multiplication;
    the Boolean result is its support (counts > 0)."""
    res = {0: 37, 1: 29, 2: 41}
    for seed in range(3):
        M = _rand((37, 29), 0.2, 700 + seed)
        N = _rand((29, 41), 0.2, 750 + seed)
        C = oracle.contract_count(M, (0, 1), N, (1, 2), (0, 2), res)
        ref = M.astype(np.int64) @ N.astype(np.int64)
        assert np.array_equal(C.astype(np.int64), ref)
        assert np.array_equal(C > 0, oracle.contract(M, (0, 1), N, (1, 2), (0, 2), res).astype(bool))


def test_count_associativity_and_saturation():
    """Associativity in N (Thm 'associative' holds in any semiring): both
    bracketings of a chain of three give the same counts; sums and products
    saturate at 2^64 - 1 instead of wrapping."""
    res = {0: 6, 1: 7, 2: 5, 3: 8}
    A = _rand((6, 7), 0.4, 800).astype(np.uint64) * np.uint64(2)
    B = _rand((7, 5), 0.4, 801).astype(np.uint64) * np.uint64(3)
    C = _rand((5, 8), 0.4, 802).astype(np.uint64)
    left = oracle.contract_count(oracle.contract_count(A, (0, 1), B, (1, 2), (0, 2), res), (0, 2), C, (2, 3), (0, 3), res)
    right = oracle.contract_count(A, (0, 1), oracle.contract_count(B, (1, 2), C, (2, 3), (1, 3), res), (1, 3), (0, 3), res)
    assert np.array_equal(left, right)
    assert np.array_equal(left.astype(np.int64),
                          A.astype(np.int64) @ B.astype(np.int64) @ C.astype(np.int64))
    big = np.full((1, 2), 2 ** 63, dtype=np.uint64)
    one = np.ones((2, 1), dtype=np.uint64)
    s = oracle.contract_count(big, (0, 1), one, (1, 2), (0, 2), {0: 1, 1: 2, 2: 1})
    assert s[0, 0] == np.uint64(2 ** 64 - 1)
    m = oracle.contract_count(np.full((1, 1), 2 ** 40, dtype=np.uint64), (0, 1), np.full((1, 1), 2 ** 40, dtype=np.uint64),
                              (1, 2), (0, 2), {0: 1, 1: 1, 2: 1})
    assert m[0, 0] == np.uint64(2 ** 64 - 1)
