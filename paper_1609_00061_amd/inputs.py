"""Seeded synthetic inputs for the pixel-array hot path.

This module only *draws inputs*: variable boxes, relation structure and
polynomial coefficients.  It contains none of the method's arithmetic (no
plotting, no contraction, no planning), so that both the CPU oracle and the
GPU library can consume exactly the same instances without sharing code.

Workloads follow the paper's input format (Ch. 2, "Input to the pixel array
method"): a set of relations, a range and resolution per variable, and a list
of exposed variables.  Every relation here is a polynomial equation
f(vars) = 0 whose coefficients are listed in graded-lex order of the
monomials in the relation's declared variable order (total degree ascending,
then lexicographically descending exponent tuples, e.g. for (x, y) and
degree 3: 1, x, y, x^2, xy, y^2, x^3, x^2y, xy^2, y^3).

Random numbers come from SplitMix64 (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) and standard normals from the
Box-Muller transform; all draws are FP64.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

MASTER_SEED = 160900061
MASK64 = (1 << 64) - 1


# ---------------------------------------------------------------- generator
class SplitMix64:
    """SplitMix64 stream (64-bit state, golden-gamma increment)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """Uniform double in [0, 1) with 53 random bits."""
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)

    def randint(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] (inclusive)."""
        return lo + int(self.uniform() * (hi - lo + 1))

    def normals(self, n: int) -> np.ndarray:
        out = np.empty(n, dtype=np.float64)
        i = 0
        while i < n:
            u1 = 1.0 - self.uniform()          # (0, 1]
            u2 = self.uniform()
            rad = math.sqrt(-2.0 * math.log(u1))
            out[i] = rad * math.cos(2.0 * math.pi * u2)
            if i + 1 < n:
                out[i + 1] = rad * math.sin(2.0 * math.pi * u2)
            i += 2
        return out


def instance_seed(config: int, index: int, master: int = MASTER_SEED) -> int:
    """Per-instance seed: one SplitMix64 output of master ^ config<<32 ^ index."""
    return SplitMix64(master ^ (config << 32) ^ index).next_u64()


# ---------------------------------------------------------------- structures
def n_monomials(arity: int, degree: int) -> int:
    """Number of monomials of total degree <= degree in `arity` variables."""
    return math.comb(arity + degree, degree)


TARGET_EQ, TARGET_LE, TARGET_LT = 0, 1, 2     # f = 0, f <= 0, f < 0


@dataclass
class Relation:
    vars: Tuple[int, ...]          # distinct variable ids, declared order
    degree: int
    coef: np.ndarray               # float64, graded-lex order
    target: int = TARGET_EQ        # target subset of f: {0}, (-inf, 0] or (-inf, 0)

    def __post_init__(self):
        self.vars = tuple(int(v) for v in self.vars)
        self.coef = np.ascontiguousarray(self.coef, dtype=np.float64)
        assert self.coef.shape == (n_monomials(len(self.vars), self.degree),)


@dataclass
class System:
    axes: List[Tuple[float, float, int]]    # (lo, hi, resolution) per variable
    relations: List[Relation]
    exposed: Tuple[int, ...]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_vars(self) -> int:
        return len(self.axes)

    def digest(self) -> str:
        """SHA-256 over the instance's numbers (axes, structure, coefficients)."""
        h = hashlib.sha256()
        for lo, hi, r in self.axes:
            h.update(np.array([lo, hi], dtype="<f8").tobytes())
            h.update(np.array([r], dtype="<i8").tobytes())
        for rel in self.relations:
            h.update(np.array(rel.vars + (rel.degree,), dtype="<i8").tobytes())
            h.update(rel.coef.astype("<f8").tobytes())
            if rel.target:
                h.update(np.array([rel.target], dtype="<i8").tobytes())
        h.update(np.array(self.exposed, dtype="<i8").tobytes())
        return h.hexdigest()


def random_relation(rng: SplitMix64, vars: Sequence[int], degree: int = 3) -> Relation:
    return Relation(tuple(vars), degree, rng.normals(n_monomials(len(vars), degree)))


# ---------------------------------------------------------------- workloads
def config1() -> System:
    """Tiny plain case: x^2+y^2-1 on (x,y) and y-z^3+z/2 on (y,z), box [-2,2]^3
    at 64 cells per axis; y latent, (x, z) exposed.  Variables: x=0, y=1, z=2."""
    circle = Relation((0, 1), 2, np.array([-1.0, 0, 0, 1.0, 0, 1.0]))
    # monomials of (y, z), degree 3: 1, y, z, y^2, yz, z^2, y^3, y^2z, yz^2, z^3
    cubic = Relation((1, 2), 3, np.array([0, 1.0, 0.5, 0, 0, 0, 0, 0, 0, -1.0]))
    return System([(-2.0, 2.0, 64)] * 3, [circle, cubic], (0, 2), name="c1_circle_cubic_r64")


def config2(index: int = 0, res: int = 1024, n_rel: int = 8) -> System:
    """Chain of 8 binary cubic relations f_i(x_i, x_{i+1}) on [-3,3]^9 at
    `res` cells per axis; x_1 and x_9 exposed (ids 0 and 8)."""
    rng = SplitMix64(instance_seed(2, index))
    rels = [random_relation(rng, (i, i + 1)) for i in range(n_rel)]
    return System([(-3.0, 3.0, res)] * (n_rel + 1), rels, (0, n_rel),
                  name=f"c2_chain{n_rel}_r{res}_i{index}")


def config3(index: int = 0, res: int = 256) -> System:
    """Four ternary cubic relations over six variables, every pair sharing one
    variable: R1(v1,v2,v3) R2(v3,v4,v5) R3(v5,v6,v1) R4(v2,v4,v6) with ids
    v_k = k-1; (v1, v4) exposed; box [-3,3]^6."""
    rng = SplitMix64(instance_seed(3, index))
    struct = [(0, 1, 2), (2, 3, 4), (4, 5, 0), (1, 3, 5)]
    rels = [random_relation(rng, s) for s in struct]
    return System([(-3.0, 3.0, res)] * 6, rels, (0, 3), name=f"c3_ternary4_r{res}_i{index}")


def chain_system(rng: SplitMix64, length: int, res: Sequence[int]) -> System:
    rels = [random_relation(rng, (i, i + 1)) for i in range(length)]
    return System([(-3.0, 3.0, int(r)) for r in res], rels, (0, length))


def config4(n_systems: int = 512, index: int = 0, rmin: int = 64, rmax: int = 2048) -> List[System]:
    """Batch of independent chains: length L uniform in {2..6}, L+1 variables,
    resolution per variable round(exp(U(ln rmin, ln rmax))), ends exposed."""
    rng = SplitMix64(instance_seed(4, index))
    out = []
    for s in range(n_systems):
        L = rng.randint(2, 6)
        res = [int(round(math.exp(math.log(rmin) + rng.uniform() * (math.log(rmax) - math.log(rmin)))))
               for _ in range(L + 1)]
        sysm = chain_system(rng, L, res)
        sysm.name = f"c4_chain{L}_s{s}"
        out.append(sysm)
    return out


def _fits_scope_caps(rel_vars: Sequence[Tuple[int, ...]], exposed: Sequence[int], max_out: int = 4,
                     max_scope: int = 6) -> bool:
    """Structural filter of the hypergraph workload (variable sets only; no
    plotting, contraction or cost arithmetic): is there a binary merge tree of
    the relations, each merge joining two connected clusters that share a
    variable, in which every merge ranges over at most `max_scope` variables
    and keeps at most `max_out`?  A cluster S keeps the variables of its
    relations that are exposed or occur in a relation outside S; a merge of S1
    and S2 ranges over the union of what they keep.  At 128 cells per axis
    the caps are 128^4 bits (32 MiB) per intermediate and 128^6 pairs per
    step."""
    m = len(rel_vars)
    rv = [sum(1 << v for v in vs) for vs in rel_vars]
    ex = sum(1 << v for v in exposed)
    full = (1 << m) - 1
    var_of = [0] * (1 << m)                 # union of the variables of a relation set
    for S in range(1, 1 << m):
        low = S & -S
        var_of[S] = var_of[S ^ low] | rv[low.bit_length() - 1]
    adj = [0] * m
    for i in range(m):
        for j in range(m):
            if i != j and rv[i] & rv[j]:
                adj[i] |= 1 << j

    def kept(S):
        return var_of[S] & (var_of[full ^ S] | ex)

    conn = {}

    def connected(S):
        c = conn.get(S)
        if c is None:
            seen = frontier = S & -S
            while frontier:
                nb, f = 0, frontier
                while f:
                    b = f & -f
                    f ^= b
                    nb |= adj[b.bit_length() - 1]
                frontier = nb & S & ~seen
                seen |= frontier
            c = conn[S] = seen == S
        return c

    memo = {}

    def ok(S):
        r = memo.get(S)
        if r is None:
            r = S & (S - 1) == 0
            if not r and bin(kept(S)).count("1") <= max_out:
                low = S & -S
                rest = S ^ low
                sub = rest
                while True:
                    L = sub | low
                    R = S ^ L
                    if (R and connected(L) and connected(R) and var_of[L] & var_of[R]
                            and bin(kept(L) | kept(R)).count("1") <= max_scope and ok(L) and ok(R)):
                        r = True
                        break
                    if sub == 0:
                        break
                    sub = (sub - 1) & rest
            memo[S] = r
        return r

    return ok(full)


def random_hypergraph(rng: SplitMix64, res: int = 128, max_tries: int = 1000) -> System:
    """Random relation hypergraph: n in {8..14} variables, m = n-1+U{0,1,2}
    relations of arity U{2,3}, connected, covering every variable; 2-4 exposed.
    Drawn again until some merge tree keeps at most 4 variables per
    intermediate and ranges over at most 6 per step (_fits_scope_caps)."""
    for _ in range(max_tries):
        n = rng.randint(8, 14)
        m = n - 1 + rng.randint(0, 2)
        rel_vars = []
        for _r in range(m):
            a = rng.randint(2, 3)
            vs = []
            while len(vs) < a:
                v = rng.randint(0, n - 1)
                if v not in vs:
                    vs.append(v)
            rel_vars.append(tuple(vs))
        covered = set(v for vs in rel_vars for v in vs)
        if len(covered) != n:
            continue
        # connectivity over variables
        parent = list(range(n))

        def find(a):
            while parent[a] != a:
                parent[a] = parent[parent[a]]
                a = parent[a]
            return a
        for vs in rel_vars:
            for v in vs[1:]:
                parent[find(v)] = find(vs[0])
        if len(set(find(v) for v in range(n))) != 1:
            continue
        n_exp = rng.randint(2, 4)
        exposed = []
        while len(exposed) < n_exp:
            v = rng.randint(0, n - 1)
            if v not in exposed:
                exposed.append(v)
        if not _fits_scope_caps(rel_vars, exposed):
            continue
        rels = [random_relation(rng, vs) for vs in rel_vars]
        return System([(-3.0, 3.0, res)] * n, rels, tuple(exposed))
    raise RuntimeError("no admissible hypergraph drawn")


def config5(n_graphs: int = 256, index: int = 0, res: int = 128) -> List[System]:
    """Random relation hypergraphs for the learned-order workload.  Training
    graphs use other `index` values (a disjoint seed range)."""
    rng = SplitMix64(instance_seed(5, index))
    out = []
    for g in range(n_graphs):
        s = random_hypergraph(rng, res)
        s.name = f"c5_g{g}_i{index}"
        out.append(s)
    return out


# ---------------------------------------------------------------- raw arrays
def random_bool_array(shape: Sequence[int], density: float, seed: int) -> np.ndarray:
    """Boolean array (one byte per entry) with i.i.d. entries set w.p. density."""
    rng = SplitMix64(seed)
    n = int(np.prod(shape)) if len(shape) else 1
    words = np.array([rng.next_u64() for _ in range((n + 3) // 4)], dtype=np.uint64)
    u16 = words.view(np.uint16)[:n].astype(np.float64) / 65536.0
    return (u16 < density).reshape(tuple(shape)).astype(np.uint8)


def random_normals(n: int, seed: int) -> np.ndarray:
    return SplitMix64(seed).normals(n)
