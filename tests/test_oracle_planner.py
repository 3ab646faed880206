"""Pins for the planner reference (Sec. 3.5): the paper's worked examples and
the speed-up proposition, and the DP against brute force."""
import itertools
import json
import os

import pytest

from oracle import planner as P
from paper_1609_00061_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_cluster_tree_example_costs():
    """Sec. 3.5.1 example: Cost_T = 2r^5 + 2r^4 + r^3 and PCost_T = 2r^5."""
    g = _load("cluster_tree_example.json")
    packs = [tuple(p) for p in g["packs"]]
    tree = json.loads(json.dumps(g["tree"]), object_hook=None)

    def tup(t):
        return t if isinstance(t, int) else tuple(tup(x) for x in t)
    tree = tup(tree)
    cost, pcost = P.tree_cost(tree, packs, g["exposed"])
    assert cost == P.poly({int(k): v for k, v in g["cost"].items()})
    assert pcost == P.poly({int(k): v for k, v in g["pcost"].items()})
    # node costs r^5 (ABC), r^4 (EF), r^3 (EF,G), r^4 (EFG,D), r^5 (root)
    for r in (3, 10):  # at r = 2 the integer max differs from the N[r] order
        c_int, p_int = P.tree_cost(tree, packs, g["exposed"], res={v: r for v in range(10)})
        assert c_int == 2 * r ** 5 + 2 * r ** 4 + r ** 3
        assert p_int == 2 * r ** 5


def test_cluster_tree_example_minimum_reading():
    """The paper states the example tree is minimal; under our reading of its
    figure the exhaustive search finds {A, B, {{C,D},{{E,F},G}}} at 3r^4 + 2r^3,
    which is strictly smaller.  Pin what the search finds (the printed tree's
    cost is pinned above)."""
    g = _load("cluster_tree_example.json")
    packs = [tuple(p) for p in g["packs"]]
    best, tree = P.optimal_cost(packs, g["exposed"])
    assert best == P.poly({4: 3, 3: 2})
    assert P.tree_cost(tree, packs, g["exposed"])[0] == best
    printed = P.poly({5: 2, 4: 2, 3: 1})
    assert P.poly_key(best) < P.poly_key(printed)


def test_mnp_example():
    """Sec. 3.5: three n x n matrices, unclustered n^4, clustered 2n^3."""
    M, N, Pk = (0, 1), (1, 2), (2, 3)
    packs = [M, N, Pk]
    exposed = (0, 3)
    assert P.tree_cost((0, 1, 2), packs, exposed)[0] == P.poly({4: 1})
    assert P.tree_cost(((0, 1), 2), packs, exposed)[0] == P.poly({3: 2})
    assert P.optimal_cost(packs, exposed)[0] == P.poly({3: 2})


def test_speedup_proposition():
    """Prop 'speedup' (eqn difference): for a nontrivial cluster C the flat
    cost minus the clustered cost is r^Q (r^(L'+L'') - r^L' - r^L'') >= 0."""
    rng = inputs.SplitMix64(5)
    checked = 0
    for _ in range(300):
        n = rng.randint(2, 5)
        nv = rng.randint(3, 7)
        packs = [tuple(sorted(set(rng.randint(0, nv - 1) for _ in range(rng.randint(1, 3))))) for _ in range(n)]
        covered = sorted(set(v for p in packs for v in p))
        # Def. 'wd': every link (exposed ones included) is hit by an inner port
        exposed = tuple(sorted(set(covered[rng.randint(0, len(covered) - 1)] for _ in range(rng.randint(0, 2)))))
        m = rng.randint(1, n - 1)
        C = list(range(m))
        inner = set(v for i in C for v in packs[i])
        outer = set(exposed) | set(v for i in range(m, n) for v in packs[i])
        Q = inner & outer
        L1, L2 = inner - Q, outer - Q
        if not L1 or not L2:
            continue
        r = 3
        flat = P.tree_cost(tuple(range(n)), packs, exposed, res={v: r for v in range(nv)})[0]
        if m > 1:
            clustered = P.tree_cost((tuple(C),) + tuple(range(m, n)), packs, exposed,
                                    res={v: r for v in range(nv)})[0]
        else:
            # a one-pack cluster: interior diagram P_1 -> Q_C costs r^Lambda',
            # exterior diagram Q_C, P_2.. -> P' costs r^Lambda''
            outside = set(v for i in range(1, n) for v in packs[i])
            clustered = r ** len(inner) + r ** len(Q | outside)
        diff = r ** len(Q) * (r ** (len(L1) + len(L2)) - r ** len(L1) - r ** len(L2))
        assert flat - clustered == diff >= 0
        checked += 1
    assert checked > 50


@pytest.mark.parametrize("seed", range(8))
def test_binary_dp_matches_brute_force(seed):
    rng = inputs.SplitMix64(77 + seed)
    n = rng.randint(2, 6)
    nv = rng.randint(3, 8)
    packs = [tuple(sorted(set(rng.randint(0, nv - 1) for _ in range(rng.randint(1, 3))))) for _ in range(n)]
    exposed = tuple(sorted(set(rng.randint(0, nv - 1) for _ in range(rng.randint(0, 3)))))
    res = {v: rng.randint(2, 9) for v in range(nv)}
    best, tree = P.optimal_cost(packs, exposed, res=res, binary=True)
    brute = min(P.tree_cost(t, packs, exposed, res=res)[0] for t in P.all_binary_trees(range(n)))
    assert best == brute
    assert P.tree_cost(tree, packs, exposed, res=res)[0] == best


def _admissible(tree, packs, exposed, max_out, max_scope):
    """Every merge of a binary tree joins two connected clusters sharing a
    link, keeps at most max_out links and ranges over at most max_scope."""
    def links(block):
        return set(v for i in block for v in packs[i])

    def connected(block):
        block = list(block)
        seen, todo = {block[0]}, [block[0]]
        while todo:
            i = todo.pop()
            for j in block:
                if j not in seen and set(packs[i]) & set(packs[j]):
                    seen.add(j)
                    todo.append(j)
        return len(seen) == len(block)

    def rec(t):
        if isinstance(t, int):
            return True
        L, R = P.leaves(t[0]), P.leaves(t[1])
        if not (connected(L) and connected(R) and links(L) & links(R)):
            return False
        if len(P.q_pack(L + R, packs, exposed)) > max_out:
            return False
        if len(P.q_pack(L, packs, exposed) | P.q_pack(R, packs, exposed)) > max_scope:
            return False
        return rec(t[0]) and rec(t[1])
    return rec(tree)


def _tree_of(merges, n):
    f = {i: i for i in range(n)}
    for t, (a, b) in enumerate(merges):
        f[n + t] = (f[a], f[b])
    return f[n + len(merges) - 1] if merges else 0


def _bounded_cost(tree, packs, exposed, res):
    if isinstance(tree, int):
        return 0
    L, R = P.leaves(tree[0]), P.leaves(tree[1])
    node = 1
    for v in P.q_pack(L, packs, exposed) | P.q_pack(R, packs, exposed):
        node *= res[v]
    return node + _bounded_cost(tree[0], packs, exposed, res) + _bounded_cost(tree[1], packs, exposed, res)


@pytest.mark.parametrize("seed", range(10))
def test_bounded_merges_brute_force(seed):
    """The oracle's bounded tree is the cheapest admissible binary tree, found
    by brute force over every binary tree; None iff there is none."""
    rng = inputs.SplitMix64(900 + seed)
    nv = rng.randint(4, 8)
    n = rng.randint(2, 6)
    packs = [tuple(rng.randint(0, nv - 1) for _ in range(rng.randint(2, 3))) for _ in range(n)]
    packs = [tuple(dict.fromkeys(p)) for p in packs]
    exposed = tuple(sorted(set(rng.randint(0, nv - 1) for _ in range(rng.randint(1, 3)))))
    res = {v: rng.randint(2, 9) for v in range(nv)}
    max_out, max_scope = rng.randint(2, 4), rng.randint(3, 5)
    got = P.bounded_merges(packs, exposed, res, max_out=max_out, max_scope=max_scope)
    trees = [t for t in P.all_binary_trees(range(n)) if _admissible(t, packs, exposed, max_out, max_scope)]
    if not trees:
        assert got is None
        return
    best = min(_bounded_cost(t, packs, exposed, res) for t in trees)
    tree = _tree_of(got, n)
    assert _admissible(tree, packs, exposed, max_out, max_scope)
    assert _bounded_cost(tree, packs, exposed, res) == best


def test_generator_scope_filter_agrees_with_oracle():
    """The hypergraph generator's structural filter and the oracle's bounded
    tree search (two separate implementations) agree on which diagrams admit
    a tree within the caps."""
    rng = inputs.SplitMix64(950)
    checked = {True: 0, False: 0}
    for _ in range(60):
        nv = rng.randint(5, 9)
        n = rng.randint(nv - 1, nv + 1)
        packs = [tuple(dict.fromkeys(rng.randint(0, nv - 1) for _ in range(rng.randint(2, 3)))) for _ in range(n)]
        if len(set(v for p in packs for v in p)) != nv:
            continue
        exposed = tuple(sorted(set(rng.randint(0, nv - 1) for _ in range(rng.randint(2, 4)))))
        res = {v: 4 for v in range(nv)}
        for max_out, max_scope in ((2, 3), (3, 4), (4, 6)):
            a = inputs._fits_scope_caps(packs, exposed, max_out, max_scope)
            b = P.bounded_merges(packs, exposed, res, max_out=max_out, max_scope=max_scope) is not None
            assert a == b, (packs, exposed, max_out, max_scope)
            checked[a] += 1
    assert checked[True] > 10 and checked[False] > 10, checked
