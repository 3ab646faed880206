"""GPU parity of the fused pass pair: two sparse passes alone and the
streamed contraction that reads their outputs (eqn GAM for each), computed
in one step from lists of the set bits of the pass operands, without
storing the pass outputs; bit-exact against the oracle's pairwise
multiplication (merge order (R1 R2) (R3 R4), then the two results)."""
import numpy as np
import pytest

import oracle
from paper_1609_00061_amd import inputs, pa
from gpu_util import note, to_host

pytestmark = pytest.mark.gpu

# the ternary workload's wiring: every pair of relations shares one variable
WIRING = [(0, 1, 2), (2, 3, 4), (4, 5, 0), (1, 3, 5)]


def _system(res, seed=1, c0=0.0, coefs=None, name="fused"):
    rng = inputs.SplitMix64(seed)
    rels = []
    for i, st in enumerate(WIRING):
        r = inputs.random_relation(rng, st)
        if coefs is not None and coefs[i] is not None:
            c = np.zeros(inputs.n_monomials(3, 3))
            for k, v in coefs[i].items():
                c[k] = v
            r = inputs.Relation(st, 3, c)
        else:
            r.coef[0] = r.coef[0] + c0
        rels.append(r)
    return inputs.System([(-3.0, 3.0, int(x)) for x in res], rels, (0, 3), name=f"{name}{list(res)}")


def _ref(s):
    plots = [oracle.plot(r, s.axes)[0] for r in s.relations]
    res = {v: s.axes[v][2] for v in range(len(s.axes))}
    return oracle.solve_pairwise(res, [r.vars for r in s.relations], plots, s.exposed, [(0, 1), (2, 3), (4, 5)])


def _fused_op(s):
    ops = pa.describe_plan(s, sparse_pass=3)["ops"]
    f = [o for o in ops if o["op"] == "fused_pass_pair"]
    assert len(f) == 1, [o["op"] for o in ops]
    return f[0]


def _check(s, ref, kws):
    for kw in kws:
        note("fused", s.name, kw)
        out, dims, rep = pa.solve_system(s, **kw)
        got = to_host(out, dims)
        assert np.array_equal(got, ref), (s.name, kw)
        assert rep["nnz_out"] == int(ref.sum())


KWS = (dict(sparse_pass=3), dict(sparse_pass=3, graph=True), dict(sparse_pass=3, per_op=True))

# resolutions of v0..v5: the packed latent variable t of 5 .. 256 bits (rows
# of 2 or 8 words, padded to the 8-word LDS slots), ragged 8-blocks of p and
# q, one to three 32-bit output words (the last partial), latent entries s
# not a multiple of the 16 waves, either pass in the X role; c0 shifts
# every relation's constant term (sparser plots)
CASES = [([31, 5, 255, 9, 17, 40], 1, 0.0), ([37, 29, 200, 45, 33, 51], 2, 0.0), ([24, 33, 33, 9, 5, 256], 1, 6.0),
         ([9, 8, 33, 31, 21, 200], 2, 3.0), ([129, 255, 256, 13, 24, 255], 1, 6.0), ([70, 40, 256, 66, 36, 48], 2, 0.0)]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_fused_matches_oracle(case):
    res, seed, c0 = CASES[case]
    s = _system(res, seed, c0)
    f = _fused_op(s)
    note("fused op", f)
    ref = _ref(s)
    note("oracle nnz", int(ref.sum()), "of", ref.size)
    _check(s, ref, KWS)


def test_fused_planted_bands():
    """Linear relations, each free in one of its variables: R1 = v0 - v2,
    R2 = v2 - v3, R3 = v5 - v0, R4 = v3 - v5 (coefficients in graded-lex
    order 1, x, y, z of the relation's own variables).  The solution is a
    band around v3 = v0, and the rows of A along a free variable are full
    (every bit set: the longest row lists, all tail batches)."""
    coefs = [{1: 1.0, 3: -1.0}, {1: 1.0, 2: -1.0}, {2: 1.0, 3: -1.0}, {2: 1.0, 3: -1.0}]
    for res in ([37, 29, 200, 45, 33, 51], [70, 40, 256, 66, 36, 48], [129, 255, 256, 13, 24, 255]):
        s = _system(res, coefs=coefs, name="bands")
        _fused_op(s)
        ref = _ref(s)
        note("bands oracle nnz", int(ref.sum()), "of", ref.size)
        assert 0 < ref.sum() < ref.size // 2
        _check(s, ref, KWS[:2])


def test_fused_empty_and_full_operands():
    """Degenerate plots: R4 and R3 never zero (constant 1: empty A rows, an
    all-zero output), then R4 identically zero (every cell plotted: every
    A row of its pass has all its bits set)."""
    for coefs, name in (([None, None, {0: 1.0}, {0: 1.0}], "empty"), ([None, None, None, {}], "full")):
        s = _system([37, 29, 200, 45, 33, 51], seed=3, coefs=coefs, name=name)
        _fused_op(s)
        ref = _ref(s)
        note(name, "oracle nnz", int(ref.sum()), "of", ref.size)
        if name == "empty":
            assert ref.sum() == 0
        _check(s, ref, KWS[:2])


def test_fused_batch():
    """Three systems in one batch: their fused steps share one launch (tiles
    of several steps), replayed as one graph; every output against the
    oracle."""
    import torch
    systems = [_system(r, seed, c0) for r, seed, c0 in (CASES[0], CASES[1], CASES[5])]
    refs = [_ref(s) for s in systems]
    for kw in (dict(sparse_pass=3), dict(sparse_pass=3, graph=True)):
        note("fused batch", kw)
        b = pa.Batch(systems, **kw)
        stream = torch.cuda.Stream()
        for _ in range(2):
            outs, rep, nnz = b.execute(stream=stream, report=True)
            for i, (o, d, ref) in enumerate(zip(outs, b.dims, refs)):
                assert np.array_equal(to_host(o, d), ref), (i, kw)
                assert nnz[i] == int(ref.sum())
