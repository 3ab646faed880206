"""GPU parity of pairwise generalized array multiplication (eqn GAM, two
packs) through pa_contract: every kernel (MFMA GEMM, word streaming along a
latent or kept packed axis, bit level) against the oracle, bit-exact."""
import numpy as np
import pytest

import oracle
from paper_1609_00061_amd import inputs, pa
from gpu_util import note, to_device, to_host

pytestmark = pytest.mark.gpu


def _run(a_vars, b_vars, out_vars, res, density, seed, b_none=False):
    A = inputs.random_bool_array([res[v] for v in a_vars], density, seed)
    B = inputs.random_bool_array([res[v] for v in b_vars], density, seed + 1)
    ad, bd, cd = [res[v] for v in a_vars], [res[v] for v in b_vars], [res[v] for v in out_vars]
    note("contract", a_vars, b_vars, "->", out_vars, "dims", ad, bd, cd)
    C = pa.contract(to_device(A), ad, a_vars, None if b_none else to_device(B), bd, b_vars, out_vars, cd)
    got = to_host(C, cd)
    if b_none:
        ref = oracle.contract(A, a_vars, np.ones(()), (), out_vars, res)
    else:
        ref = oracle.contract(A, a_vars, B, b_vars, out_vars, res)
    assert np.array_equal(got, ref), (a_vars, b_vars, out_vars)


PATTERNS = [
    ((0, 1), (2, 1), (0, 2)),            # canonical GEMM (k packed in both)
    ((0, 1), (1, 2), (0, 2)),            # matmul, B not k-packed
    ((0, 1, 2), (0, 3, 2), (0, 1, 3)),   # batched canonical GEMM
    ((0, 1, 2), (1, 2, 3), (0, 3)),      # two latent, packed one shared
    ((0, 2, 1), (3, 2, 1), (3, 0)),      # stream over shared packed latent
    ((0, 1, 2), (0, 3, 2), (3, 1, 0)),   # permuted output
    ((0, 1), (0, 1), (0, 1)),            # elementwise AND, shared packed kept
    ((0, 2, 1), (2, 1), (0, 1)),         # kept packed axis, latent 2
    ((0, 1), (2, 3), (0, 1, 2, 3)),      # Kronecker
    ((0, 1), (1, 2), ()),                # 0-dim output
    ((0, 1, 2), (1,), (0,)),             # private latent 2 in A
    ((0, 1), (0, 2), (0, 1, 2)),         # batched outer product: A broadcast over C's packed axis
    ((0, 2), (0, 1), (0, 1, 2)),         # the same with B broadcast
    ((1,), (0, 2), (0, 1, 2)),           # one-axis A broadcast
    ((0, 1, 3), (0, 2), (0, 2, 1)),      # A packed along a latent variable: bit-level fallback
    ((3, 1, 0, 2), (0, 1, 3, 2), (0, 3)),  # stream over a shared packed latent, A contiguous along the row
                                           # variable and B along the packed one: rows x bits wave tiles
    ((1, 3, 0, 2), (1, 0, 3, 2), (0, 3)),  # the same with the other latent outermost
]

SIZES = [
    {0: 5, 1: 70, 2: 33, 3: 9},
    {0: 64, 1: 64, 2: 64, 3: 3},
    {0: 37, 1: 129, 2: 100, 3: 2},
]


@pytest.mark.parametrize("sizes", range(len(SIZES)))
@pytest.mark.parametrize("pat", range(len(PATTERNS)))
def test_patterns(pat, sizes):
    a_vars, b_vars, out_vars = PATTERNS[pat]
    _run(a_vars, b_vars, out_vars, SIZES[sizes], 0.08, 1000 + 17 * pat + sizes)


def test_projection_without_b():
    res = {0: 40, 1: 70, 2: 65}
    _run((0, 1, 2), (), (2, 0), res, 0.02, 55, b_none=True)
    _run((0, 1, 2), (), (0,), res, 0.02, 56, b_none=True)


@pytest.mark.parametrize("path", [1, 2, 3, 4])
@pytest.mark.parametrize("M,N,K", [(64, 64, 64), (128, 128, 256), (100, 130, 70), (1024, 1024, 1024),
                                   (33, 1000, 5000), (300, 65, 129), (257, 7, 3000), (600, 300, 520),
                                   (700, 1500, 256), (513, 900, 200), (2000, 260, 33)])
def test_mfma_gemm_sizes(M, N, K, path):
    """Dense canonical layout A[m][k], B[n][k] -> C[m][n] on the fp4 MFMA,
    with K chunks staged in LDS (path 1: 128 x 128 tiles, path 3: 256 x 128),
    loaded by each wave (path 2), or with A operands kept in registers across
    the 256 x 128 tiles of a workgroup's range (path 4, K <= 256 bits: several
    row blocks and many column tiles per workgroup; longer K falls back to
    3): all tile residues, ragged K tails, split K; against integer
    matmul > 0."""
    A = inputs.random_bool_array((M, K), 2.0 / K, 91 + M)
    B = inputs.random_bool_array((N, K), 2.0 / K, 92 + N)
    note("gemm", M, N, K, "path", path)
    C = pa.contract(to_device(A), [M, K], (0, 1), to_device(B), [N, K], (2, 1), (0, 2), [M, N], gemm_path=path)
    got = to_host(C, [M, N])
    ref = (A.astype(np.int64) @ B.astype(np.int64).T) > 0
    assert np.array_equal(got.astype(bool), ref)


@pytest.mark.parametrize("path", [1, 2, 3, 4])
def test_mfma_gemm_dense_and_batched(path):
    """Dense inputs (every count large) and a batch index."""
    nb, M, N, K = 3, 200, 150, 600
    A = inputs.random_bool_array((nb, M, K), 0.5, 5)
    B = inputs.random_bool_array((nb, N, K), 0.01, 6)
    note("gemm batched", nb, M, N, K, "path", path)
    C = pa.contract(to_device(A), [nb, M, K], (0, 1, 2), to_device(B), [nb, N, K], (0, 3, 2), (0, 1, 3), [nb, M, N],
                    gemm_path=path)
    got = to_host(C, [nb, M, N])
    ref = np.einsum("bmk,bnk->bmn", A.astype(np.int64), B.astype(np.int64)) > 0
    assert np.array_equal(got.astype(bool), ref)


@pytest.mark.parametrize("kdim", [100, 200, 400, 1000])
@pytest.mark.parametrize("latent", [3, 8, 13])
def test_stream_over_shared_packed_latent(kdim, latent):
    """Word streaming over a packed latent axis of 4, 8, 16 and 32 words
    per row (the 4/8/16-word rows take the four-entries-at-a-time path),
    with latent-entry counts that are and are not multiples of four, and
    rows-by-bits wave tiles."""
    res = {0: 40, 1: latent, 2: kdim, 3: 70}
    # about one matching latent entry per output bit: half the outputs set
    _run((3, 1, 0, 2), (0, 1, 3, 2), (0, 3), res, 1.0 / np.sqrt(kdim * latent), 700 + kdim + latent)
