"""pa_contract_noalloc (no device allocation; its scratch table in a static
device array) against pa_contract and the oracle, through the C ABI: two
calls in a row on every case, the second with a smaller input, on streamed
contractions (word-streaming over a shared latent variable, and over an
output word with a broadcast operand), a bit-level one and a dense MFMA one;
a table beyond the static array is refused."""
import numpy as np
import pytest

import oracle
from paper_1609_00061_amd import inputs, pa
from gpu_util import note, to_device, to_host

pytestmark = pytest.mark.gpu

# (a_vars, b_vars, out_vars): variable 1 is latent in every case
CASES = [
    ((0, 1, 2), (3, 1, 2), (3, 0)),     # shared packed latent variable: stream mode K, table over variable 1
    ((1, 0), (1, 2), (0, 2)),           # A packed along an output variable: stream mode W, table over 1
    ((0, 1, 2), (1, 2, 3), (0, 3)),     # B packed along an output variable A lacks: bit level
    ((0, 1), (2, 1), (0, 2)),           # canonical layout: MFMA
]


def _run(case, res, seed):
    a_vars, b_vars, out_vars = case
    a_dims = [res[v] for v in a_vars]
    b_dims = [res[v] for v in b_vars]
    o_dims = [res[v] for v in out_vars]
    A = inputs.random_bool_array(a_dims, 0.15, seed)
    B = inputs.random_bool_array(b_dims, 0.15, seed + 1)
    ref = oracle.contract(A, a_vars, B, b_vars, out_vars, res)
    dA, dB = to_device(A), to_device(B)
    c0 = pa.contract(dA, a_dims, a_vars, dB, b_dims, b_vars, out_vars, o_dims)
    c1 = pa.contract(dA, a_dims, a_vars, dB, b_dims, b_vars, out_vars, o_dims, noalloc=True)
    got0, got1 = to_host(c0, o_dims), to_host(c1, o_dims)
    assert np.array_equal(got1, got0), (case, res)
    assert np.array_equal(got1, ref), (case, res)
    return int(ref.sum())


@pytest.mark.parametrize("case", range(len(CASES)))
def test_noalloc_two_calls(case):
    big = {0: 70, 1: 300, 2: 97, 3: 130}
    small = {0: 9, 1: 40, 2: 33, 3: 21}
    for i, res in enumerate((big, small)):
        note("contract_noalloc", CASES[case], res)
        nnz = _run(CASES[case], res, 9100 + 10 * case + i)
        note("nnz", nnz)


def test_noalloc_table_limit():
    """A streamed contraction whose table has more latent entries than the
    static array holds is refused with PA_ENOMEM (pa_contract takes it)."""
    a_vars, b_vars, out_vars = (0, 1, 4, 2), (3, 1, 4, 2), (3, 0)
    res = {0: 3, 1: 300, 4: 300, 2: 40, 3: 5}      # 90000 latent entries outside the packed one
    a_dims = [res[v] for v in a_vars]
    b_dims = [res[v] for v in b_vars]
    A = inputs.random_bool_array(a_dims, 0.01, 9200)
    B = inputs.random_bool_array(b_dims, 0.01, 9201)
    dA, dB = to_device(A), to_device(B)
    with pytest.raises(pa.PaError) as e:
        pa.contract(dA, a_dims, a_vars, dB, b_dims, b_vars, out_vars, [5, 3], noalloc=True)
    assert e.value.code == pa.PA_ENOMEM
    c = pa.contract(dA, a_dims, a_vars, dB, b_dims, b_vars, out_vars, [5, 3])
    assert np.array_equal(to_host(c, [5, 3]), oracle.contract(A, a_vars, B, b_vars, out_vars, res))
