"""GPU parity of whole solves (plot + cluster tree of contractions) against
the oracle, bit-exact, for every order policy."""
import numpy as np
import pytest

import oracle
from paper_1609_00061_amd import inputs, pa
from gpu_util import note, to_host

pytestmark = pytest.mark.gpu


def _oracle_plots(s):
    return [oracle.plot(r, s.axes)[0] for r in s.relations]


def _solve(s, max_workspace=None, **kw):
    note("solve", s.name, kw)
    import os
    old = os.environ.get("PA_MAX_WORKSPACE_BYTES")
    if max_workspace is not None:
        os.environ["PA_MAX_WORKSPACE_BYTES"] = str(max_workspace)
    try:
        out, dims, rep = pa.solve_system(s, **kw)
    finally:
        if max_workspace is not None:
            if old is None:
                os.environ.pop("PA_MAX_WORKSPACE_BYTES")
            else:
                os.environ["PA_MAX_WORKSPACE_BYTES"] = old
    return to_host(out, dims), rep


@pytest.mark.parametrize("precision", [pa.PLOT_FP64, pa.PLOT_FP32_ESCALATE])
def test_c1_solve(precision):
    s = inputs.config1()
    got, rep = _solve(s, precision=precision)
    ref = oracle.solve([a[2] for a in s.axes], [r.vars for r in s.relations], _oracle_plots(s), s.exposed)
    assert ref.sum() == 180
    assert np.array_equal(got, ref)
    assert rep["nnz_out"] == 180


def _random_small_system(seed):
    rng = inputs.SplitMix64(seed)
    g = inputs.random_hypergraph(rng, res=rng.randint(5, 24))
    # uneven resolutions
    g.axes = [(-3.0, 3.0, rng.randint(3, 40)) for _ in g.axes]
    g.name = f"small{seed}"
    return g


@pytest.mark.parametrize("seed", range(8))
def test_random_hypergraphs_all_policies(seed):
    s = _random_small_system(4200 + seed)
    res = [a[2] for a in s.axes]
    ref = oracle.solve(res, [r.vars for r in s.relations], _oracle_plots(s), s.exposed)
    outs = []
    for order in (pa.ORDER_GREEDY, pa.ORDER_EXHAUSTIVE):
        got, rep = _solve(s, order=order)
        assert np.array_equal(got, ref), order
        outs.append(got)
    # a deliberately poor given order (left to right) gives the same bits,
    # or is refused: when planned if an intermediate has more rows than the
    # kernels index (PA_EUNSUPPORTED), with PA_ENOMEM when its intermediates
    # cannot fit
    n = len(s.relations)
    merges = [0, 1] + [x for t in range(1, n - 1) for x in (n + t - 1, t + 1)]
    d = pa.describe_plan(s, order=pa.ORDER_GIVEN, given=merges)
    if "error" in d:
        assert d["error"] == pa.PA_EUNSUPPORTED
        with pytest.raises(pa.PaError) as e:
            _solve(s, order=pa.ORDER_GIVEN, given=merges)
        assert e.value.code == pa.PA_EUNSUPPORTED
        return
    need = d["workspace_bytes"]
    if need < 2 ** 30:
        got, _ = _solve(s, order=pa.ORDER_GIVEN, given=merges)
        assert np.array_equal(got, ref)
    else:
        with pytest.raises(pa.PaError) as e:
            _solve(s, order=pa.ORDER_GIVEN, given=merges, max_workspace=2 ** 30)
        assert e.value.code == pa.PA_ENOMEM


@pytest.mark.parametrize("seed", range(6))
def test_sparse_pass_on_random_hypergraphs(seed):
    """Every MFMA contraction whose B is a plot gets a sparse pass (batch
    variables, several latent and output variables in any layout); with a
    density threshold of 1/1024 the MFMA kernel computes them instead, with
    1024/1024 the pass always does, and with sparse_pass = 2 the pass alone
    (no count, no MFMA kernel): always the oracle's bits."""
    s = _random_small_system(4300 + seed)
    res = [a[2] for a in s.axes]
    ref = oracle.solve(res, [r.vars for r in s.relations], _oracle_plots(s), s.exposed)
    n_pass = len([o for o in pa.describe_plan(s, sparse_pass=1)["ops"] if o["op"] == "sparse_pass"])
    note("sparse passes", n_pass)
    for kw in (dict(sparse_pass=1), dict(sparse_pass=1, sparse_max_density=1),
               dict(sparse_pass=1, sparse_max_density=1024), dict(sparse_pass=1, gemm_split=2048, sparse_max_density=1),
               dict(sparse_pass=1, order=pa.ORDER_GREEDY, gemm_path=3), dict(sparse_pass=1, per_op=True),
               dict(sparse_pass=1, per_op=True, sparse_max_density=1), dict(sparse_pass=2),
               dict(sparse_pass=2, per_op=True), dict(sparse_pass=2, graph=True, gemm_split=2048)):
        got, _ = _solve(s, **kw)
        assert np.array_equal(got, ref), kw


def test_sparse_pass_chain_and_ternary():
    """The chain (pass on the first level) and the ternary system at reduced
    resolution, with the pass or the MFMA kernel computing the contractions."""
    for s in (inputs.config2(res=128), inputs.config3(res=24)):
        res = [a[2] for a in s.axes]
        ref = oracle.solve(res, [r.vars for r in s.relations], _oracle_plots(s), s.exposed)
        for kw in (dict(sparse_pass=1), dict(sparse_pass=1, sparse_max_density=1024),
                   dict(sparse_pass=1, sparse_max_density=1), dict(sparse_pass=1, graph=True),
                   dict(sparse_pass=2), dict(sparse_pass=2, graph=True), dict()):
            got, _ = _solve(s, **kw)
            assert np.array_equal(got, ref), (s.name, kw)


def test_sparse_pass_long_output_rows():
    """Output rows of 41 x 94 words (more than one 2048-word wave-tile per
    row, a row length that is not a multiple of 4 words): R1(a, k) and
    R2(k, b, c) with b at 41 and c at 3000 cells, k latent."""
    rng = inputs.SplitMix64(4400)
    s = inputs.System([(-3.0, 3.0, 40), (-3.0, 3.0, 40), (-3.0, 3.0, 41), (-3.0, 3.0, 3000)],
                      [inputs.random_relation(rng, (0, 1)), inputs.random_relation(rng, (1, 2, 3))], (0, 2, 3),
                      name="long_rows")
    sp = [o for o in pa.describe_plan(s, sparse_pass=1)["ops"] if o["op"] == "sparse_pass"]
    assert sp and sp[0]["Nw"] > 2048 and sp[0]["Nw"] % 4 == 2
    res = [a[2] for a in s.axes]
    ref = oracle.solve(res, [r.vars for r in s.relations], _oracle_plots(s), s.exposed)
    for kw in (dict(sparse_pass=1), dict(sparse_pass=1, per_op=True), dict(sparse_pass=-1), dict(sparse_pass=2)):
        got, _ = _solve(s, **kw)
        assert np.array_equal(got, ref), kw


@pytest.mark.parametrize("case", ["short_rows", "long_rows"])
def test_sparse_pass_two_latent_variables(case):
    """A rows of more than 64 words (two latent variables packed into K: 128
    and 80 words), so the pass reads each A row in several batches of 64
    words; output rows of 2 words (one position per lane) and of 282 words
    (more than 256: eight words per lane)."""
    rng = inputs.SplitMix64(4500 if case == "short_rows" else 4501)
    res = (48, 64, 64, 40) if case == "short_rows" else (40, 40, 40, 9000)
    s = inputs.System([(-3.0, 3.0, r) for r in res],
                      [inputs.random_relation(rng, (0, 1, 2)), inputs.random_relation(rng, (1, 2, 3))], (0, 3),
                      name="two_latent_" + case)
    sp = [o for o in pa.describe_plan(s, sparse_pass=2)["ops"] if o["op"] == "sparse_pass"]
    assert len(sp) == 1 and sp[0]["Kw"] > 64 and (sp[0]["Nw"] <= 256) == (case == "short_rows")
    ref = oracle.solve(list(res), [r.vars for r in s.relations], _oracle_plots(s), s.exposed)
    note(case, "Kw", sp[0]["Kw"], "Nw", sp[0]["Nw"], "nnz", int(ref.sum()))
    for kw in (dict(sparse_pass=2), dict(sparse_pass=2, per_op=True), dict(sparse_pass=1, sparse_max_density=1024),
               dict(sparse_pass=1, sparse_max_density=1), dict(sparse_pass=-1)):
        got, _ = _solve(s, **kw)
        assert np.array_equal(got, ref), kw


def test_huge_intermediate_with_grid_stride():
    """A Kronecker-heavy order whose intermediate has more than 2^32 bits:
    every contraction kernel loops over its output (grid-stride), so the
    result stays exact."""
    s = _random_small_system(4200)
    n = len(s.relations)
    merges = [0, 1] + [x for t in range(1, n - 1) for x in (n + t - 1, t + 1)]
    need = pa.describe_plan(s, order=pa.ORDER_GIVEN, given=merges)["workspace_bytes"]
    assert 2 ** 32 / 8 < need < 16 * 2 ** 30
    res = [a[2] for a in s.axes]
    ref = oracle.solve(res, [r.vars for r in s.relations], _oracle_plots(s), s.exposed)
    got, _ = _solve(s, order=pa.ORDER_GIVEN, given=merges)
    assert np.array_equal(got, ref)


def test_c2_reduced_resolution_exact():
    s = inputs.config2(res=128)
    res = [a[2] for a in s.axes]
    ref = oracle.solve(res, [r.vars for r in s.relations], _oracle_plots(s), s.exposed)
    got, rep = _solve(s)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("res", [16, 40])
def test_c3_reduced_resolution_exact(res):
    """The ternary system where its word-streaming steps run with 2 x 32 and
    8 x 8 row-by-bit wave tiles."""
    s = inputs.config3(res=res)
    tqs = [o.get("tq") for o in pa.describe_plan(s)["ops"] if o["op"] == "stream_k"]
    assert max(tqs) == (2 if res == 16 else 8)
    ref = oracle.solve([a[2] for a in s.axes], [r.vars for r in s.relations], _oracle_plots(s), s.exposed)
    got, rep = _solve(s)
    assert np.array_equal(got, ref)


def test_c2_full_size_exact():
    """Chain of 8 at 1024 per axis: the oracle multiplies the chain pairwise
    (Sec. 3.5 clustering, left to right)."""
    s = inputs.config2()
    plots = _oracle_plots(s)
    res = {v: s.axes[v][2] for v in range(len(s.axes))}
    merges = [(0, 1)] + [(8 + t, t + 2) for t in range(6)]
    ref = oracle.solve_pairwise(res, [r.vars for r in s.relations], plots, s.exposed, merges)
    got, rep = _solve(s)
    assert np.array_equal(got, ref)
    got2, _ = _solve(s, plain=True, order=pa.ORDER_GREEDY)
    assert np.array_equal(got2, ref)
    for kw in (dict(gemm_path=2), dict(gemm_path=2, gemm_split=1), dict(gemm_split=128), dict(gemm_path=3)):
        got3, _ = _solve(s, **kw)
        assert np.array_equal(got3, ref), kw


def test_c3_full_size_exact():
    """Four ternary relations at 256^3, the whole 256 x 256 output compared
    entry by entry with the oracle (plots, then the cluster tree
    {{R1, R2}, {R3, R4}} multiplied pairwise), for the default plan (sparse
    pass with MFMA fallback), the MFMA kernel alone on both operand paths,
    the fallback taken (density threshold 1/1024), the pass alone, the two
    passes fused with the streamed contraction, and the plain path."""
    s = inputs.config3()
    note("c3 full: oracle plots and pairwise solve")
    plots = _oracle_plots(s)
    res = {v: s.axes[v][2] for v in range(len(s.axes))}
    ref = oracle.solve_pairwise(res, [r.vars for r in s.relations], plots, s.exposed, [(0, 1), (2, 3), (4, 5)],
                                log=note)
    del plots
    note("c3 full: oracle nnz", int(ref.sum()))
    assert [o["op"] for o in pa.describe_plan(s)["ops"]].count("sparse_pass") == 2
    for kw in (dict(), dict(sparse_pass=-1), dict(sparse_pass=-1, gemm_path=2), dict(sparse_max_density=1),
               dict(sparse_pass=2), dict(sparse_pass=3), dict(sparse_pass=3, per_op=True),
               dict(plain=True, order=pa.ORDER_GREEDY)):
        got, rep = _solve(s, **kw)
        note("c3 full", kw, "nnz", int(got.sum()), "flagged", rep["corners_flagged"])
        assert np.array_equal(got, ref), kw
        assert rep["nnz_out"] == int(ref.sum())
