"""GPU parity of the count-semiring contraction (pa_contract_count: the
two-pack generalized array multiplication in N) against the oracle's count
contraction and integer matrix products: the int8-MFMA path on canonical
layouts (ragged tiles, batch and several m / n / k variables, K splits,
densities from sparse to full) and the general path on other layouts, on
random arrays and on plotted relations."""
import numpy as np
import pytest

import oracle
from paper_1609_00061_amd import inputs, pa
from gpu_util import note, to_device

pytestmark = pytest.mark.gpu


def _counts(case, res, density, seed, arrays=None):
    a_vars, b_vars, out_vars = case
    a_dims = [res[v] for v in a_vars]
    b_dims = [res[v] for v in b_vars] if b_vars is not None else None
    o_dims = [res[v] for v in out_vars]
    if arrays is None:
        A = inputs.random_bool_array(a_dims, density, seed)
        B = inputs.random_bool_array(b_dims, density, seed + 1) if b_vars is not None else None
    else:
        A, B = arrays
    note("contract_count", case, [res[v] for v in sorted(res)], density)
    C = pa.contract_count(to_device(A), a_dims, a_vars, to_device(B) if B is not None else None, b_dims,
                          b_vars if b_vars is not None else [], out_vars, o_dims)
    got = C.cpu().numpy().view(np.uint32)[: int(np.prod(o_dims))].reshape(o_dims).astype(np.uint64)
    if B is None:
        ones = np.ones((), dtype=np.uint8)
        ref = oracle.contract_count(A, a_vars, ones, (), out_vars, res)
    else:
        ref = oracle.contract_count(A, a_vars, B, b_vars, out_vars, res)
    return got, ref, A, B


CANONICAL = [
    # (a_vars, b_vars, out_vars): A = [batch][m][k], B = [batch][n][k], C = [batch][m][n]
    ((0, 1), (2, 1), (0, 2)),
    ((0, 3, 1), (2, 3, 1), (0, 2)),               # two latent variables (k = (3, 1))
    ((4, 0, 1), (4, 2, 1), (4, 0, 2)),            # batch variable 4
    ((0, 5, 1), (2, 6, 1), (0, 5, 2, 6)),         # two m and two n variables
]


@pytest.mark.parametrize("case", range(len(CANONICAL)))
@pytest.mark.parametrize("density", [0.02, 0.3, 1.0])
def test_count_mfma_canonical(case, density):
    res = {0: 130, 1: 97, 2: 300, 3: 5, 4: 3, 5: 7, 6: 6}
    got, ref, A, B = _counts(CANONICAL[case], res, density, 9300 + 7 * case)
    assert np.array_equal(got, ref)
    if case == 0:
        assert np.array_equal(got.astype(np.int64), A.astype(np.int64) @ B.astype(np.int64).T)
    if density == 1.0:
        k = int(np.prod([res[v] for v in CANONICAL[case][0] if v not in CANONICAL[case][2]]))
        assert np.all(got == k)


def test_count_mfma_long_k_and_split():
    """A long latent axis (50000 entries, split over parts added atomically)
    and a short one (one word)."""
    for res, dens in (({0: 40, 1: 50000, 2: 70}, 0.05), ({0: 200, 1: 20, 2: 260}, 0.5)):
        got, ref, A, B = _counts(CANONICAL[0], res, dens, 9400)
        assert np.array_equal(got, ref)
        assert np.array_equal(got.astype(np.int64), A.astype(np.int64) @ B.astype(np.int64).T)


GENERAL = [
    ((0, 1), (1, 2), (0, 2)),           # B as [k][n]
    ((0, 1), (1, 2), (2, 0)),           # transposed output
    ((0, 1, 2), (1, 2, 3), (0, 3)),
    ((0, 1), (2, 3), (0, 1, 2, 3)),     # Kronecker: counts are products of bits
    ((0, 1), (1, 2), ()),               # everything latent: one count
    ((0, 1, 2), (1,), (0,)),
    ((0, 1), None, (1,)),               # no B: set entries of A per output entry
]


@pytest.mark.parametrize("case", range(len(GENERAL)))
def test_count_general_layouts(case):
    res = {0: 13, 1: 37, 2: 9, 3: 21}
    got, ref, _, _ = _counts(GENERAL[case], res, 0.3, 9500 + case)
    assert np.array_equal(got, ref)


def test_count_plotted_chain_step():
    """Counts of one step of the chain workload at 1024 per axis: the two
    oracle plots f1(x1, x2) and f2(x2, x3), multiplied over x2 in N (the
    number of x2 pixels joining each (x1, x3)); their support is the Boolean
    product."""
    s = inputs.config2()
    P1 = oracle.plot(s.relations[0], s.axes)[0]                 # (x1, x2)
    P2 = np.ascontiguousarray(oracle.plot(s.relations[1], s.axes)[0].T)   # (x3, x2)
    res = {0: 1024, 1: 1024, 2: 1024}
    got, ref, _, _ = _counts(((0, 1), (2, 1), (0, 2)), res, None, 0, arrays=(P1, P2))
    assert np.array_equal(got, ref)
    assert np.array_equal(got.astype(np.int64), P1.astype(np.int64) @ P2.astype(np.int64).T)
    bool_ref = oracle.contract(P1, (0, 1), P2, (2, 1), (0, 2), res)
    assert np.array_equal(got > 0, bool_ref.astype(bool))
    note("chain step counts: max", int(got.max()), "nonzero", int((got > 0).sum()))
