"""GPU parity of the executors: the plain path (one launch per relation plot
and per step), the per-op path, the persistent work-queue launch, and its
hipGraph replays; every tuning parameter must give the same bits."""
import numpy as np
import pytest

import oracle
from paper_1609_00061_amd import inputs, pa
from gpu_util import note, to_host

pytestmark = pytest.mark.gpu


def _oracle_solve(s):
    plots = [oracle.plot(r, s.axes)[0] for r in s.relations]
    return oracle.solve([a[2] for a in s.axes], [r.vars for r in s.relations], plots, s.exposed)


def _systems():
    out = [inputs.config1(), inputs.config2(res=128), inputs.config3(res=24)]
    rng = inputs.SplitMix64(31337)
    for i in range(3):
        g = inputs.random_hypergraph(rng, res=12)
        g.axes = [(-3.0, 3.0, rng.randint(4, 30)) for _ in g.axes]
        g.name = f"hg{i}"
        out.append(g)
    return out


SYSTEMS = _systems()
MODES = [dict(plain=True, order=pa.ORDER_GREEDY), dict(per_op=True), dict(), dict(graph=True),
         dict(single_launch=True), dict(single_launch=True, graph=True)]


@pytest.mark.parametrize("mode", range(len(MODES)))
@pytest.mark.parametrize("si", range(len(SYSTEMS)))
def test_executors_agree(si, mode):
    import torch
    s = SYSTEMS[si]
    ref = _oracle_solve(s)
    kw = MODES[mode]
    note("exec", s.name, kw)
    stream = torch.cuda.Stream()
    plan = pa.Plan(s, **kw)
    out = pa.empty_bits(plan.dims)
    _, rep, _ = plan.execute(out, stream=stream, report=True)
    assert np.array_equal(to_host(out, plan.dims), ref)
    assert rep["nnz_out"] == int(ref.sum())


@pytest.mark.parametrize("params", [dict(single_launch=True, persist_wg=1),
                                    dict(single_launch=True, persist_wg=7, plot_strip=1),
                                    dict(single_launch=True, persist_wg=64, plot_strip=3, contract_units=256),
                                    dict(plot_strip=8, contract_units=8192), dict(plot_strip=1, contract_units=256),
                                    dict(gemm_split=1), dict(gemm_split=2048, plot_strip=2),
                                    dict(single_launch=True, gemm_split=1024), dict(gemm_path=2),
                                    dict(gemm_path=2, gemm_split=1), dict(single_launch=True, gemm_path=2),
                                    dict(gemm_path=2, graph=True, gemm_split=64), dict(gemm_path=3),
                                    dict(gemm_path=3, gemm_split=1), dict(single_launch=True, gemm_path=3)])
def test_persistent_tuning_parameters(params):
    for s in SYSTEMS[:4]:
        ref = _oracle_solve(s)
        note("tuning", s.name, params)
        out, dims, rep = pa.solve_system(s, **params)
        assert np.array_equal(to_host(out, dims), ref)


@pytest.mark.parametrize("kw", [dict(gemm_path=3), dict(single_launch=True, gemm_path=3), dict(gemm_path=3, gemm_split=1)])
def test_256_row_tiles_cover_every_row(kw):
    """A chain at 200 per axis (200-row contractions: one partial 256-row
    tile, two 128-row tiles in the single persistent launch, which keeps
    128 x 128 tiles)."""
    s = inputs.config2(res=200)
    ref = _oracle_solve(s)
    note("wide tiles", s.name, kw)
    out, dims, rep = pa.solve_system(s, **kw)
    assert np.array_equal(to_host(out, dims), ref)


@pytest.mark.parametrize("single", [False, True])
def test_graph_replays_with_eager_work_between(single):
    """Each replay of the captured launch is checked against the oracle, with
    the program's own eager work (clearing the output, unrelated kernels) and
    synchronizations between replays."""
    import torch
    s = inputs.config2(res=256)
    ref = _oracle_solve(s)
    stream = torch.cuda.Stream()
    plan = pa.Plan(s, graph=True, single_launch=single)
    out = pa.empty_bits(plan.dims)
    junk = torch.zeros(1 << 20, dtype=torch.int32, device="cuda")
    for rep in range(5):
        note("graph replay", rep)
        with torch.cuda.stream(stream):
            out.zero_()
            junk.add_(rep)
        plan.execute(out, stream=stream)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(out, plan.dims), ref), rep
        junk.mul_(2)
        torch.cuda.synchronize()
    # a second output buffer recaptures and still matches
    out2 = pa.empty_bits(plan.dims)
    plan.execute(out2, stream=stream)
    assert np.array_equal(to_host(out2, plan.dims), ref)


@pytest.mark.parametrize("strip", [1, 2, 5, 16])
def test_plot_strip_lengths(strip):
    """Plot tiles walk `strip` cells per thread; every length is bit-exact."""
    s = inputs.config3(res=40)
    for rel in s.relations[:2]:
        note("plot strip", strip, rel.vars)
        plan = pa.Plan(inputs.System([s.axes[v] for v in rel.vars],
                                     [inputs.Relation(tuple(range(len(rel.vars))), rel.degree, rel.coef)],
                                     tuple(range(len(rel.vars)))), plot_strip=strip)
        out, _, _ = plan.execute(report=True)
        ref, _ = oracle.plot(rel, s.axes)
        assert np.array_equal(to_host(out, plan.dims), ref)


def test_time_groups_leaves_output_exact():
    """Repeated back-to-back launches of every group (the benchmark's kernel
    timing) keep the plan's output bit-exact."""
    import torch
    s = inputs.config2(res=200)
    ref = _oracle_solve(s)
    stream = torch.cuda.Stream()
    plan = pa.Plan(s)
    out = pa.empty_bits(plan.dims)
    plan.execute(out, stream=stream)
    times = plan.time_groups(reps=5, stream=stream)
    assert len(times) >= 3 and all(ms > 0 for _, ms, _ in times)
    assert {k for k, _, _ in times} >= {pa.OPKIND_PLOT, pa.OPKIND_GEMM}
    assert np.array_equal(to_host(out, plan.dims), ref)
    b = pa.Batch([s, inputs.config1()])
    outs, _, _ = b.execute(stream=stream)
    assert len(b.time_groups(reps=3, stream=stream)) >= 3
    assert np.array_equal(to_host(outs[0], b.dims[0]), ref)


@pytest.mark.parametrize("graph", [False, True])
def test_persistent_wait_gives_up_when_forced_from_the_host(graph):
    """The single persistent launch's bounded dependency wait, made to give
    up from the host (a negative bound: every wait gives up at its first
    poll, every workgroup leaves, the kernel ends normally): the execute call
    with a report returns PA_EHIP; with the default bound written back the
    same plan (and graph) solves the system again, bit-exact."""
    import torch
    s = inputs.config2(res=128)
    ref = _oracle_solve(s)
    stream = torch.cuda.Stream()
    plan = pa.Plan(s, single_launch=True, graph=graph)
    out = pa.empty_bits(plan.dims)
    note("forced wait give-up", s.name, "graph", graph)
    plan.set_wait_limit(-1)
    with pytest.raises(pa.PaError) as e:
        plan.execute(out, stream=stream, report=True)
    assert e.value.code == pa.PA_EHIP and "gave up a dependency wait" in str(e.value)
    plan.set_wait_limit(1 << 26)
    _, rep, _ = plan.execute(out, stream=stream, report=True)
    assert np.array_equal(to_host(out, plan.dims), ref)
    assert rep["nnz_out"] == int(ref.sum())


def test_batch_persistent_wait_gives_up_when_forced_from_the_host():
    """As above for a batch's single persistent launch (two chains)."""
    import torch
    systems = [inputs.config2(res=64), inputs.config2(res=96)]
    refs = [_oracle_solve(s) for s in systems]
    stream = torch.cuda.Stream()
    b = pa.Batch(systems, single_launch=True)
    outs = b.alloc_outputs()
    note("forced wait give-up, batch")
    b.set_wait_limit(-1)
    with pytest.raises(pa.PaError) as e:
        b.execute(outs, stream=stream, report=True)
    assert e.value.code == pa.PA_EHIP
    b.set_wait_limit(1 << 26)
    b.execute(outs, stream=stream, report=True)
    for o, d, ref in zip(outs, b.dims, refs):
        assert np.array_equal(to_host(o, d), ref)
