"""GPU parity of batched solving: many independent systems in one merged step
table (grouped launches or one persistent launch, optionally one hipGraph),
bit-exact per system against the oracle."""
import numpy as np
import pytest

import oracle
from paper_1609_00061_amd import inputs, pa
from gpu_util import note, to_host

pytestmark = pytest.mark.gpu


def _oracle_solve(s):
    plots = [oracle.plot(r, s.axes)[0] for r in s.relations]
    return oracle.solve([a[2] for a in s.axes], [r.vars for r in s.relations], plots, s.exposed)


def _small_chains(n=24):
    return inputs.config4(n_systems=n, index=7, rmin=8, rmax=96)


MODES = [dict(), dict(graph=True), dict(single_launch=True), dict(single_launch=True, graph=True),
         dict(order=pa.ORDER_GREEDY, plot_strip=2, contract_units=512), dict(graph=True, sparse_pass=1),
         dict(sparse_pass=1, sparse_max_density=1), dict(sparse_pass=2, graph=True), dict(sparse_pass=-1)]


@pytest.mark.parametrize("mode", range(len(MODES)))
def test_uneven_chains(mode):
    import torch
    systems = _small_chains()
    refs = [_oracle_solve(s) for s in systems]
    kw = MODES[mode]
    note("batch chains", len(systems), kw)
    b = pa.Batch(systems, **kw)
    stream = torch.cuda.Stream()
    for rep_i in range(2):                      # second run reuses (or replays) the same plan
        outs, rep, nnz = b.execute(stream=stream, report=True)
        for i, (o, d, ref) in enumerate(zip(outs, b.dims, refs)):
            assert np.array_equal(to_host(o, d), ref), (i, systems[i].name)
            assert nnz[i] == int(ref.sum())
        assert rep["nnz_out"] == sum(int(r.sum()) for r in refs)


def test_random_hypergraph_batch():
    systems = inputs.config5(n_graphs=12, index=77, res=10)
    refs = [_oracle_solve(s) for s in systems]
    note("batch hypergraphs", len(systems))
    b = pa.Batch(systems, graph=True)
    import torch
    outs, rep, nnz = b.execute(stream=torch.cuda.Stream(), report=True)
    for i, (o, d, ref) in enumerate(zip(outs, b.dims, refs)):
        assert np.array_equal(to_host(o, d), ref), i


def test_full_size_batch_exact():
    """The 512-chain workload (resolutions 64..2048) in one batch replayed as
    one graph: every system's output compared entry by entry with the
    oracle's pairwise chain, and its per-system report (set bits, corners,
    escalations summing to the batch total)."""
    import torch
    systems = inputs.config4()
    note("batch c4", len(systems))
    b = pa.Batch(systems, graph=True)
    outs, rep, nnz, reps = b.execute(stream=torch.cuda.Stream(), report=True, per_system=True)
    torch.cuda.synchronize()
    assert sum(r["corners_flagged"] for r in reps) == rep["corners_flagged"]
    for i, s in enumerate(systems):
        plots = [oracle.plot(r, s.axes)[0] for r in s.relations]
        res = {v: s.axes[v][2] for v in range(len(s.axes))}
        n = len(s.relations)
        merges = [(0, 1)] + [(n + t, t + 2) for t in range(n - 2)]
        ref = oracle.solve_pairwise(res, [r.vars for r in s.relations], plots, s.exposed, merges)
        assert np.array_equal(to_host(outs[i], b.dims[i]), ref), s.name
        assert nnz[i] == int(ref.sum()) == reps[i]["nnz_out"]
        assert reps[i]["corners"] == sum((s.axes[r.vars[0]][2] + 1) * (s.axes[r.vars[1]][2] + 1)
                                         for r in s.relations)
        if i % 64 == 0:
            note("batch c4: checked through system", i)
