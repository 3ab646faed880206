"""CPU tests of the C ABI library: it loads, exports every symbol include/pa.h
declares, validates inputs, and its host planner agrees with the planner
reference.  No kernel is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import planner as P
from paper_1609_00061_amd import inputs, pa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", fn)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names += re.findall(r"\b(pa_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = pa.load()
    names = _declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n


def test_row_words_and_sizes():
    assert pa.row_words(1) == 2 and pa.row_words(64) == 2 and pa.row_words(65) == 4
    assert pa.row_words(1024) == 32 and pa.row_words(2049) == 66
    assert pa.array_words([]) == 1
    assert pa.array_words([3, 5, 70]) == 3 * 5 * 4


@pytest.mark.parametrize("dims", [(), (1,), (5,), (3, 64), (2, 3, 65), (4, 129)])
def test_pack_unpack_roundtrip(dims):
    a = inputs.random_bool_array(dims, 0.5, 11)
    w = pa.pack_bits(a)
    assert w.size == pa.array_words(list(dims))
    assert np.array_equal(pa.unpack_bits(w, dims), a)


def _kernels(plan):
    return [o["op"] for o in plan["ops"] if o["op"] != "fill"]


def test_plans_put_dense_steps_on_mfma():
    c1 = pa.describe_plan(inputs.config1())
    assert _kernels(c1) == ["gemm_mfma"]
    c2 = pa.describe_plan(inputs.config2())
    assert _kernels(c2) == ["gemm_mfma"] * 7
    # the sparse pass alone: the circle pair, and the chain's four first-level steps
    assert _kernels(pa.describe_plan(inputs.config1(), sparse_pass=2)) == ["sparse_pass"]
    c2p = pa.describe_plan(inputs.config2(), sparse_pass=2)
    assert sorted(_kernels(c2p)) == ["gemm_mfma"] * 3 + ["sparse_pass"] * 4
    c3 = pa.describe_plan(inputs.config3())
    assert _kernels(c3) == ["sparse_count", "sparse_pass", "gemm_mfma"] * 2 + ["stream_k"]
    assert _kernels(pa.describe_plan(inputs.config3(), sparse_pass=-1)) == ["gemm_mfma", "gemm_mfma", "stream_k"]
    # both r^5 steps (65536 x 65536 x 256) on MFMA after a sparse pass each,
    # the r^4 step streamed
    g = [o for o in c3["ops"] if o["op"] == "gemm_mfma"]
    assert all(o["macs"] == 256 ** 5 and o["Kw"] == 8 for o in g)
    assert [o["macs"] for o in c3["ops"] if o["op"] == "stream_k"] == [256 ** 4]
    assert c3["cost"] == 2 * 256 ** 5 + 256 ** 4


def test_stream_tile_shape_prefers_longer_runs():
    """The ternary system's final streamed step: 4 x 16 and 8 x 8 row-by-bit
    wave tiles touch the same number of 128-byte lines with their first
    loads (32), and the 8 x 8 tile reads them as 256-byte runs (16 segments
    against 24), so it is chosen."""
    d = pa.describe_plan(inputs.config3())
    assert [o["tq"] for o in d["ops"] if o["op"] == "stream_k"] == [8]


def test_sparse_pass_plan():
    """The ternary system's r^5 contractions (2^40 MACs) get a sparse pass:
    B's relation is plotted a second time with the output variables packed
    (256 rows of k x 65536 output bits), a count step reads A (65536 rows of
    8 words), the pass writes output rows of 2048 words when A has at most
    64 set bits per 1024 (default), and each MFMA contraction reads the same
    counter; the chain's 2^30-MAC contractions get none unless asked; the
    plain path and a single persistent launch never use it."""
    d = pa.describe_plan(inputs.config3())
    cn = [o for o in d["ops"] if o["op"] == "sparse_count"]
    sp = [o for o in d["ops"] if o["op"] == "sparse_pass"]
    gm = [o for o in d["ops"] if o["op"] == "gemm_mfma"]
    assert len(sp) == 2 and len(cn) == 2 and len(d["plots"]) == 6
    for k, s, g in zip(cn, sp, gm):
        assert s["rows"] == 65536 and s["Kw"] == 8 and s["Nw"] == 2048
        assert s["max_total"] == 65536 * 256 * 64 // 1024
        assert k["words"] == 65536 * 8 and k["a"] == s["a"] == g["a"]
        assert k["flag"] == s["flag"] == g["flag"] >= 0 and s["c"] == g["c"]
        bt = [p for p in d["plots"] if p["buf"] == s["bt"]][0]
        assert bt["vars"] == s["bt_vars"] and len(bt["vars"]) == 3
    # the chain (2^30-MAC steps): no pass by default; with sparse_pass = 2 the
    # four first-level contractions (B a plot) get the pass alone, with no
    # count step and no decision, and the other levels no pass
    assert all(o["flag"] == -1 for o in pa.describe_plan(inputs.config2())["ops"] if o["op"] == "gemm_mfma")
    c2 = pa.describe_plan(inputs.config2(), sparse_pass=2)
    assert all(o["flag"] == -1 for o in c2["ops"] if o["op"] == "gemm_mfma")
    sp = [o for o in c2["ops"] if o["op"] == "sparse_pass"]
    assert len(sp) == 4 and all(o["flag"] == -1 and o["max_total"] == -1 for o in sp)
    assert not [o for o in c2["ops"] if o["op"] == "sparse_count"]
    # each of them reads the second plot of B only, so B's first plot is
    # dropped: eight plots, as without the pass (twelve with the fallback)
    assert len(c2["plots"]) == 8 and {p["buf"] for p in c2["plots"]} >= {o["bt"] for o in sp}
    assert len(pa.describe_plan(inputs.config2())["plots"]) == 8
    assert len(pa.describe_plan(inputs.config2(), sparse_pass=1)["plots"]) == 12
    c2 = pa.describe_plan(inputs.config2(), sparse_pass=1, sparse_max_density=5)
    sp2 = [o for o in c2["ops"] if o["op"] == "sparse_pass"]
    assert len(sp2) == 4                                    # level 1: B is a plot
    assert all(o["max_total"] == 1024 * 1024 * 5 // 1024 and o["flag"] >= 0 for o in sp2)
    assert len([o for o in c2["ops"] if o["op"] == "sparse_count"]) == 4
    # sparse_pass = 2 on the ternary system: the pass alone for both r^5 steps
    c3 = pa.describe_plan(inputs.config3(), sparse_pass=2)
    assert _kernels(c3) == ["sparse_pass"] * 2 + ["stream_k"]
    for kw in (dict(plain=True), dict(single_launch=True), dict(sparse_pass=-1)):
        for s in (inputs.config2(), inputs.config3()):
            assert not [o for o in pa.describe_plan(s, **kw)["ops"] if o["op"].startswith("sparse")], kw
    assert _bad(inputs.config1(), sparse_pass=4) == pa.PA_EINVAL
    assert _bad(inputs.config1(), sparse_pass=-2) == pa.PA_EINVAL
    assert _bad(inputs.config1(), sparse_max_density=-1) == pa.PA_EINVAL
    assert _bad(inputs.config1(), sparse_max_density=1025) == pa.PA_EINVAL


def _fused_system(res, seed=1, c0=0.0):
    """Four ternary relations wired as the ternary workload (every pair of
    relations shares one variable, (v0, v3) exposed) at the resolutions
    `res`; c0 is added to every constant coefficient."""
    rng = inputs.SplitMix64(seed)
    rels = [inputs.random_relation(rng, st) for st in [(0, 1, 2), (2, 3, 4), (4, 5, 0), (1, 3, 5)]]
    for r in rels:
        r.coef[0] = r.coef[0] + c0
    return inputs.System([(-3.0, 3.0, r) for r in res], rels, (0, 3), name=f"fused{res}")


def test_plot_tilings():
    """Plot tiles as planned (Sec. 3.2 plotting; host logic): trivariate
    corner plots walk the fixed axis (a thread per 32-cell word and strip of
    s rows, ta fixed-axis cells each, tw x tb = 256 threads), with s capped
    so that the tile's (tb s + 1)(ta + 1) corner lines fit the 648-line
    table; centre-rule and bivariate plots keep their one-line-per-thread
    tiles.  Tile counts cover every cell exactly once (ceil divisions)."""
    c3 = inputs.config3()
    for strip, s_exp in ((1, 1), (2, 2), (4, 4), (8, 4)):
        for p in pa.describe_plan(c3, plot_strip=strip)["plots"]:
            tw, tb, ta, s = p["tile"]
            assert p["walk_fixed"] == 1 and (tw, tb, ta, s) == (8, 32, 4, s_exp), (strip, p)
            assert (tb * s + 1) * (ta + 1) <= 648
            # 256 cells per axis: 1 word block x ceil(256 / (tb s)) x 256 / ta
            assert p["tiles"] == -(-256 // (tb * s)) * (256 // ta), p
    ragged = inputs.System([(-3.0, 3.0, r) for r in (30, 65, 31)],
                           [inputs.random_relation(inputs.SplitMix64(5), (0, 1, 2))], (0, 2), name="ragged")
    p = pa.describe_plan(ragged, plot_strip=4)["plots"][0]
    tw, tb, ta, s = p["tile"]
    assert p["walk_fixed"] == 1 and tw * tb <= 256 and (tb * s + 1) * (ta + 1) <= 648, p
    res = {v: ragged.axes[v][2] for v in range(3)}
    fixed, walk = res[p["vars"][0]], res[p["vars"][1]]
    words = -(-res[p["vars"][2]] // 32)
    assert p["tiles"] == -(-words // tw) * -(-walk // (tb * s)) * -(-fixed // ta), p
    centre = pa.describe_plan(c3, plot_rule=pa.RULE_CENTER, tolerance=0.01)["plots"][0]
    assert centre["walk_fixed"] == 0
    assert all(p["walk_fixed"] == 0 for p in pa.describe_plan(inputs.config2())["plots"])


def test_fused_pass_pair_plan():
    """sparse_pass = 3 fuses the ternary workload's two passes and their
    streamed contraction: two row-list steps (one per pass, 65536 list rows,
    LDS rows 0..255 and 256..511, zero row 512) and one fused step of
    1024 tiles of 8 x 8 outputs; the 2 x 512 MiB pass outputs are gone from
    the workspace (the lists take room for every set bit of every row: 2 x
    64 MiB), and the fused step counts the MACs of all three."""
    s = inputs.config3()
    d2, d3 = pa.describe_plan(s, sparse_pass=2), pa.describe_plan(s, sparse_pass=3)
    assert _kernels(d3) == ["row_list", "row_list", "fused_pass_pair"]
    lx, ly, f = d3["ops"]
    assert lx["rows"] == ly["rows"] == 65536 and lx["lbase"] == 0 and ly["lbase"] == 256
    assert lx["zrow"] == ly["zrow"] == 512 and lx["cap"] == ly["cap"] == 256
    assert (f["n_p"], f["n_q"], f["n_s"], f["rwt"], f["kx"], f["ky"], f["tiles"]) == (256, 256, 256, 8, 256, 256, 1024)
    assert f["lists"] == lx["c"] == ly["c"] and f["c"] == -2 and f["c_vars"] == [0, 3]
    assert f["macs"] == sum(o.get("dense_macs", 0) for o in d2["ops"] if o["op"] == "sparse_pass") + \
        [o for o in d2["ops"] if o["op"] == "stream_k"][0]["macs"]
    assert d2["workspace_bytes"] > 2 * 2 ** 29 and d3["workspace_bytes"] < 160 * 2 ** 20
    # uneven resolutions: the packed latent variable of 5 .. 256 bits, ragged
    # 8-blocks and 32-bit output words, either pass in the X role
    for res in ([31, 5, 255, 9, 17, 40], [37, 29, 200, 45, 33, 51], [24, 33, 33, 9, 5, 256],
                [129, 255, 256, 13, 24, 255]):
        d = pa.describe_plan(_fused_system(res), sparse_pass=3)
        assert _kernels(d) == ["row_list", "row_list", "fused_pass_pair"], res
        lx, ly, f = d["ops"]
        # 16-bit entries: a list row holds every latent bit, at least 8 entries
        # (one 16-byte load), 16-byte aligned; the LDS rows of both operands
        # and the zero row fit the tile's 513
        for l, k in ((lx, f["kx"]), (ly, f["ky"])):
            assert l["cap"] % 8 == 0 and l["cap"] >= max(8, k), (res, l)
        assert lx["lbase"] == 0 and ly["lbase"] == f["kx"] and lx["zrow"] == f["kx"] + f["ky"] <= 512, res
        assert f["tiles"] == -(-f["n_p"] // 8) * -(-f["n_q"] // 8), res
    # no pattern, no fusion: the chain's passes feed MFMA contractions
    assert _kernels(pa.describe_plan(inputs.config2(), sparse_pass=3)) == \
        _kernels(pa.describe_plan(inputs.config2(), sparse_pass=2))


def test_large_k_mfma_plan_is_valid():
    """A random hypergraph at 128 whose greedy tree has an MFMA contraction of
    65536 K words in one part: plans are checked against their buffers at
    planning time, and such a K range is valid (fp32 sums of non-negative
    products cannot round a positive sum to zero)."""
    rng = inputs.SplitMix64(9011)
    g = inputs.random_hypergraph(rng, res=128)
    d = pa.describe_plan(g, order=pa.ORDER_GREEDY)
    big = [o for o in d["ops"] if o["op"] == "gemm_mfma" and o["Kw"] > 16384]
    assert big and big[0]["ksplit"] == 1


def test_exhaustive_prefers_parallel_trees_on_ties():
    """All cluster trees of the chain cost 7 r^3; the balanced one has the
    lowest parallel cost (3 r^3, Sec. 3.5.1) and is chosen."""
    d = pa.describe_plan(inputs.config2())
    assert d["cost"] == 7 * 1024 ** 3
    assert d["merges"][:8] == [0, 1, 2, 3, 8, 9, 4, 5] or sorted(d["merges"][:4]) == [0, 1, 2, 3]
    # depth of the tree: no merge consumes the previous merge's output three times in a row
    n = 8
    depth = {i: 0 for i in range(n)}
    for t in range(n - 1):
        a, b = d["merges"][2 * t], d["merges"][2 * t + 1]
        depth[n + t] = 1 + max(depth[a], depth[b])
    assert depth[2 * n - 2] == 3


def _packs(s):
    return [tuple(r.vars) for r in s.relations]


@pytest.mark.parametrize("seed", range(6))
def test_exhaustive_planner_matches_reference_dp(seed):
    """The library's exhaustive order reaches the minimum binary cluster-tree
    cost of the planner reference (Sec. 3.5 cost model)."""
    g = inputs.config5(n_graphs=1, index=1000 + seed, res=128)[0]
    if len(g.relations) > 11:
        pytest.skip("reference DP in Python too slow for this size")
    d = pa.describe_plan(g, order=pa.ORDER_EXHAUSTIVE)
    res = {v: g.axes[v][2] for v in range(len(g.axes))}
    # Latent variables private to one relation are projected first by a
    # one-pack cluster node (cost r^vars); the rest is a binary tree on the
    # intermediate packs Q of the relations.
    packs = _packs(g)
    qpacks = [tuple(sorted(P.q_pack([i], packs, g.exposed))) for i in range(len(packs))]
    unary = sum(int(np.prod([res[v] for v in p])) for p, q in zip(packs, qpacks) if len(q) < len(p))
    best, _ = P.optimal_cost(qpacks, g.exposed, res=res, binary=True)
    best += unary
    assert d["cost"] == pytest.approx(best, rel=1e-12)
    dg = pa.describe_plan(g, order=pa.ORDER_GREEDY)
    assert dg["cost"] >= best * (1 - 1e-12)


def test_given_order_cost_matches_reference():
    s = inputs.config3()
    merges = [0, 1, 4, 2, 5, 3]
    d = pa.describe_plan(s, order=pa.ORDER_GIVEN, given=merges)
    tree = (((0, 1), 2), 3)
    res = {v: 256 for v in range(6)}
    assert d["cost"] == pytest.approx(P.tree_cost(tree, _packs(s), s.exposed, res=res)[0], rel=1e-12)
    assert d["merges"] == merges


def _bad(system, exposed=None, **kw):
    d = pa.describe_plan(system, exposed, **kw)
    return d.get("error")


def test_validation_errors():
    c1 = inputs.config1()
    assert _bad(c1) is None
    s = inputs.config1()
    s.axes = [(-2.0, 2.0, 1)] + s.axes[1:]
    assert _bad(s) == pa.PA_EINVAL                      # resolution < 2
    s = inputs.config1()
    s.axes = [(2.0, -2.0, 64)] + s.axes[1:]
    assert _bad(s) == pa.PA_EINVAL                      # lo > hi
    s = inputs.config1()
    s.axes = s.axes + [(-1.0, 1.0, 8)]
    assert _bad(s) == pa.PA_EINVAL                      # variable in no relation
    assert _bad(c1, exposed=[0, 0]) == pa.PA_EINVAL     # repeated exposed
    assert _bad(c1, exposed=[7]) == pa.PA_EINVAL        # out of range
    s = inputs.config1()
    s.relations[0].coef[1] = float("nan")
    assert _bad(s) == pa.PA_EINVAL                      # non-finite coefficient
    assert _bad(c1, order=pa.ORDER_GIVEN, given=[0, 0]) == pa.PA_EINVAL
    s = inputs.config1()
    s.relations[0] = inputs.Relation((0, 0), 2, s.relations[0].coef)
    assert _bad(s) == pa.PA_EINVAL                      # repeated variable in a relation
    for k in ("persist_wg", "plot_strip", "contract_units", "gemm_split"):
        assert _bad(c1, **{k: -1}) == pa.PA_EINVAL      # negative tuning parameter


def test_gemm_split_target_sets_the_k_split():
    """The chain's balanced tree runs 4, 2 and 1 contractions of 1024^3 (64
    output tiles each) per level.  The default target (512 work items per
    grouped launch) splits K in 2 on the first level (256 tiles), in 4 on
    the second (128) and in 4 on the third (64 tiles; 4 parts of 256 bits is
    the most a 1024-bit K allows); a target of 1 never splits; every split
    contraction gets one fill.  With the first level on the sparse pass
    alone the other two levels keep their splits."""
    s = inputs.config2(res=1024)
    ks = lambda d: [o["ksplit"] for o in d["ops"] if o["op"] == "gemm_mfma"]
    assert ks(pa.describe_plan(s)) == [2, 2, 4, 2, 2, 4, 4]
    assert ks(pa.describe_plan(s, gemm_split=1)) == [1] * 7
    assert ks(pa.describe_plan(s, gemm_split=128)) == [1, 1, 1, 1, 1, 1, 2]
    assert ks(pa.describe_plan(s, sparse_pass=2)) == [4, 4, 4]
    fills = lambda d: [o for o in d["ops"] if o["op"] == "fill"]
    assert len(fills(pa.describe_plan(s))) == 7
    assert len(fills(pa.describe_plan(s, gemm_split=128))) == 1
    assert len(fills(pa.describe_plan(s, gemm_split=1))) == 0
    assert len(fills(pa.describe_plan(s, sparse_pass=2))) == 3


def test_mfma_operand_path_choice():
    """Default operand path: 256 x 128 tiles with the A operands kept in
    registers (path 3 in the plan) for the ternary system's two
    65536^2 x 256 contractions (262144 tiles of 128 x 128 each, K = 256
    bits), 128 x 128 tiles (path 0) for the chain's 1024^3 ones; gemm_path
    1/2/3/4 force paths 0/1/2/3, 4 falling back to 2 when K is longer than
    256 bits; a single persistent launch never uses 256-row tiles;
    out-of-range values are refused."""
    paths = lambda d: [o["path"] for o in d["ops"] if o["op"] == "gemm_mfma"]
    c2, c3 = inputs.config2(res=1024), inputs.config3()
    assert set(paths(pa.describe_plan(c3))) == {3}
    assert set(paths(pa.describe_plan(c2))) == {0}
    for opt, path in ((1, 0), (2, 1), (3, 2), (4, 2)):
        assert set(paths(pa.describe_plan(c2, gemm_path=opt))) == {path}
    for opt, path in ((1, 0), (2, 1), (3, 2), (4, 3)):
        assert set(paths(pa.describe_plan(c3, gemm_path=opt, sparse_pass=-1))) == {path}
    assert set(paths(pa.describe_plan(c3, single_launch=True))) == {0}
    assert set(paths(pa.describe_plan(c3, single_launch=True, gemm_path=3))) == {0}
    assert set(paths(pa.describe_plan(c3, single_launch=True, gemm_path=4))) == {0}
    assert set(paths(pa.describe_plan(c3, single_launch=True, gemm_path=2))) == {1}
    assert _bad(inputs.config1(), gemm_path=5) == pa.PA_EINVAL


def test_plan_create_rejects_before_touching_the_device():
    s = inputs.config1()
    s.axes = [(-2.0, 2.0, 1)] + s.axes[1:]
    with pytest.raises(pa.PaError) as e:
        pa.Plan(s)
    assert e.value.code == pa.PA_EINVAL


def test_workspace_bytes_is_host_planning():
    """pa_workspace_bytes sizes a plan on the host (no device here): the
    figure equals the plan description's, and invalid systems give an error
    instead of a size."""
    for s in (inputs.config1(), inputs.config2(), inputs.config3()):
        for kw in (dict(), dict(order=pa.ORDER_GREEDY, plain=True), dict(sparse_pass=2)):
            assert pa.workspace_bytes(s, **kw) == max(256, pa.describe_plan(s, **kw)["workspace_bytes"])
    with pytest.raises(pa.PaError):
        pa.workspace_bytes(inputs.config1(), exposed=[0, 0])
    s = inputs.config1()
    s.axes = [(-2.0, 2.0, 1)] + s.axes[1:]
    with pytest.raises(pa.PaError):
        pa.workspace_bytes(s)


def test_count_contraction_rejects_inexact_counts():
    """pa_contract_count refuses latent variables with 2^31 or more entries
    (its int32 accumulators would not be exact), before touching the device."""
    import ctypes
    L = pa.load()
    a = pa.BitArray()
    a.data = ctypes.c_void_p(0x1000)
    a.ndim = 3
    for i, d in enumerate((4, 65536, 65536)):
        a.dims[i] = d
    a.row_words = pa.row_words(65536)
    av = (ctypes.c_int32 * 3)(0, 1, 2)
    ov = (ctypes.c_int32 * 1)(0)
    rc = L.pa_contract_count(ctypes.byref(a), av, None, None, ov, 1, ctypes.c_void_p(0x2000), None, None)
    assert rc == pa.PA_EUNSUPPORTED
