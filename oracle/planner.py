"""Planner reference: cluster trees and their cost polynomials (Sec. 3.5) --
TEST INFRASTRUCTURE ONLY.

A wiring diagram is given as a list of inner packs (each a tuple of link ids,
i.e. variable ids) plus the outer pack (the exposed links).  A cluster tree is
a nested tuple whose leaves are pack indices.

  * intermediate pack Q_C of a cluster C: links of C's packs that also occur in
    a pack outside C or in the outer pack (Def. "efficient_factorization");
  * the cost of one node is the naive cost r^L of its generalized array
    multiplication (eqn naive_cost), L = union of the children's packs (a leaf's
    pack is the relation's own links, an inner node's is its Q);
  * Cost_T sums node costs; the parallel cost adds a node's cost to the max of
    its children's parallel costs (Sec. 3.5.1).

Costs are kept two ways: as exact integers for concrete resolutions, and as
polynomials in a constant resolution r (dict exponent -> coefficient) compared
in the well-order of N[r] (footnote of Sec. 3.5.1): higher degree first.
"""
from __future__ import annotations

import itertools
from functools import lru_cache
from typing import Dict, FrozenSet, Iterable, List, Sequence, Tuple

Poly = Tuple[Tuple[int, int], ...]   # sorted ((exponent, coeff), ...) descending exponent


# ------------------------------------------------------------ polynomials in r
def poly(d: Dict[int, int]) -> Poly:
    return tuple(sorted(((e, c) for e, c in d.items() if c), reverse=True))


def poly_add(a: Poly, b: Poly) -> Poly:
    d: Dict[int, int] = {}
    for e, c in a + b:
        d[e] = d.get(e, 0) + c
    return poly(d)


def poly_key(a: Poly):
    """Sort key realising the order of N[r]: compare coefficient vectors from
    the highest degree down."""
    return tuple(a)


def poly_max(a: Poly, b: Poly) -> Poly:
    return a if poly_key(a) >= poly_key(b) else b


def poly_eval(a: Poly, r: int) -> int:
    return sum(c * r ** e for e, c in a)


# -------------------------------------------------------------- diagram pieces
def q_pack(cluster: Iterable[int], packs: Sequence[Tuple[int, ...]], exposed: Iterable[int]) -> FrozenSet[int]:
    """Intermediate pack Q_C = Lambda'_C intersect Lambda''_C."""
    cl = set(cluster)
    inner = set(v for i in cl for v in packs[i])
    outer = set(exposed)
    for i in range(len(packs)):
        if i not in cl:
            outer |= set(packs[i])
    return frozenset(inner & outer)


def leaves(tree) -> List[int]:
    if isinstance(tree, int):
        return [tree]
    out: List[int] = []
    for t in tree:
        out += leaves(t)
    return out


def _node_links(tree, packs, exposed) -> FrozenSet[int]:
    links = set()
    for child in tree:
        if isinstance(child, int):
            links |= set(packs[child])
        else:
            links |= q_pack(leaves(child), packs, exposed)
    return frozenset(links)


def tree_cost(tree, packs, exposed, res: Dict[int, int] = None):
    """(Cost_T, PCost_T) of a cluster tree.  With res=None the costs are
    polynomials in a constant r; otherwise exact integers for the given
    resolutions."""
    def node_cost(links):
        if res is None:
            return poly({len(links): 1})
        out = 1
        for v in links:
            out *= res[v]
        return out

    def rec(t):
        if isinstance(t, int):
            zero = poly({}) if res is None else 0
            return zero, zero
        c = node_cost(_node_links(t, packs, exposed))
        total, par = c, None
        for child in t:
            ct, cp = rec(child)
            total = poly_add(total, ct) if res is None else total + ct
            if par is None:
                par = cp
            else:
                par = poly_max(par, cp) if res is None else max(par, cp)
        par = poly_add(c, par) if res is None else c + par
        return total, par
    if isinstance(tree, int):
        tree = (tree,)
    return rec(tree)


# ----------------------------------------------------------------- exhaustive
def _set_partitions(items: List[int]):
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for part in _set_partitions(rest):
        for i in range(len(part)):
            yield part[:i] + [[first] + part[i]] + part[i + 1:]
        yield [[first]] + part


def optimal_cost(packs: Sequence[Tuple[int, ...]], exposed: Sequence[int], res: Dict[int, int] = None,
                 binary: bool = False, parallel: bool = False):
    """Minimum of Cost_T (or PCost_T) over all cluster trees of the diagram, by
    dynamic programming over subsets of inner packs (Q_C depends only on C).
    binary=True restricts nodes to two children.  Returns (cost, tree)."""
    n = len(packs)

    def node_cost(links):
        if res is None:
            return poly({len(links): 1})
        out = 1
        for v in links:
            out *= res[v]
        return out

    def add(a, b):
        return poly_add(a, b) if res is None else a + b

    def better(a, b):
        if res is None:
            return poly_key(a) < poly_key(b)
        return a < b

    def mx(a, b):
        return (poly_max(a, b) if res is None else max(a, b))

    zero = poly({}) if res is None else 0

    @lru_cache(maxsize=None)
    def best(S: FrozenSet[int]):
        items = sorted(S)
        if len(items) == 1:
            return zero, items[0]
        best_c, best_t = None, None
        for part in _set_partitions(items):
            if len(part) < 2 or (binary and len(part) != 2):
                continue
            links = set()
            sub = []
            for block in part:
                if len(block) == 1:
                    links |= set(packs[block[0]])
                else:
                    links |= q_pack(block, packs, exposed)
                sub.append(best(frozenset(block)))
            c = node_cost(links)
            if parallel:
                m = sub[0][0]
                for s in sub[1:]:
                    m = mx(m, s[0])
                tot = add(c, m)
            else:
                tot = c
                for s in sub:
                    tot = add(tot, s[0])
            if best_c is None or better(tot, best_c):
                best_c, best_t = tot, tuple(s[1] for s in sub)
        return best_c, best_t

    full = frozenset(range(n))
    if n == 1:
        links = frozenset(packs[0])
        return node_cost(links), (0,)
    return best(full)


def all_binary_trees(items: Sequence[int]):
    """Every binary cluster tree over the given leaves (brute force, tiny n)."""
    items = list(items)
    if len(items) == 1:
        yield items[0]
        return
    first = items[0]
    rest = items[1:]
    # split into two non-empty blocks, the block with `first` on the left
    for k in range(0, len(rest)):
        for comb in itertools.combinations(rest, k):
            left = [first] + list(comb)
            right = [x for x in rest if x not in comb]
            if not right:
                continue
            for lt in all_binary_trees(left):
                for rt in all_binary_trees(right):
                    yield (lt, rt)


# ------------------------------------------------- bounded tree for the oracle
def bounded_merges(packs: Sequence[Tuple[int, ...]], exposed: Sequence[int], res: Dict[int, int],
                   max_out: int = 4, max_scope: int = 6):
    """A binary cluster tree (Sec. 3.5) for executing a diagram on the oracle
    with byte arrays: among trees whose every merge joins two clusters that
    share a link (the whole diagram being connected), whose intermediate packs
    Q_C (Def. "efficient_factorization") have at most max_out links and whose
    merges range over at most max_scope links, the one of least naive cost
    (eqn naive_cost, the product of the resolutions of the links a merge ranges
    over; a leaf enters a merge with its own Q).  Returns the merges in the
    format of oracle.solve_pairwise, or None when no such tree exists."""
    n = len(packs)
    ex = set(exposed)

    def q_of(block):
        return frozenset(q_pack(block, packs, ex))

    def links_of(block):
        return set(v for i in block for v in packs[i])

    def shares(b1, b2):
        return bool(links_of(b1) & links_of(b2))

    def connected(block):
        block = sorted(block)
        seen = {block[0]}
        frontier = [block[0]]
        while frontier:
            i = frontier.pop()
            for j in block:
                if j not in seen and set(packs[i]) & set(packs[j]):
                    seen.add(j)
                    frontier.append(j)
        return len(seen) == len(block)

    @lru_cache(maxsize=None)
    def best(S: FrozenSet[int]):
        """(cost, tree) of the cheapest admissible tree over S, or None."""
        if len(S) == 1:
            return 0, next(iter(S))
        if len(q_of(S)) > max_out:
            return None
        items = sorted(S)
        first, rest = items[0], items[1:]
        out = None
        for k in range(0, len(rest)):
            for comb in itertools.combinations(rest, k):
                L = frozenset((first,) + comb)
                R = S - L
                if not connected(L) or not connected(R) or not shares(L, R):
                    continue
                span = q_of(L) | q_of(R)
                if len(span) > max_scope:
                    continue
                bl, br = best(L), best(R)
                if bl is None or br is None:
                    continue
                c = bl[0] + br[0]
                node = 1
                for v in span:
                    node *= res[v]
                c += node
                if out is None or c < out[0]:
                    out = (c, (bl[1], br[1]))
        return out

    full = frozenset(range(n))
    got = best(full)
    if got is None:
        return None
    merges: List[Tuple[int, int]] = []
    counter = [n]

    def emit(t):
        if isinstance(t, int):
            return t
        a, b = emit(t[0]), emit(t[1])
        merges.append((a, b))
        counter[0] += 1
        return counter[0] - 1

    emit(got[1])
    return merges
