"""The executor autotuner: candidates are timed and the chosen settings give
the oracle's bits, for a batch and for a single plan."""
import numpy as np
import pytest

import oracle
from paper_1609_00061_amd import inputs, pa
from gpu_util import note, to_host

pytestmark = pytest.mark.gpu


def _oracle_solve(s):
    plots = [oracle.plot(r, s.axes)[0] for r in s.relations]
    return oracle.solve([a[2] for a in s.axes], [r.vars for r in s.relations], plots, s.exposed)


def test_autotune_batch_candidates_and_result():
    import torch
    systems = inputs.config4(n_systems=10, index=21, rmin=8, rmax=96)
    note("autotune batch", len(systems))
    best, tried = pa.autotune(systems, reps=2, graph=True, stream=torch.cuda.Stream())
    assert len(tried) >= 8
    assert best["ms"] > 0 and best["ms"] == min(t["ms"] for t in tried)
    assert best["plot_strip"] in (1, 2, 4, 8) and best["contract_units"] in (512, 2048, 8192, 32768)
    assert best["gemm_split"] in (1, 64, 128, 256, 512, 1024, 2048)
    refs = [_oracle_solve(s) for s in systems]
    b = pa.Batch(systems, graph=True, autotune=True)       # served from the cache
    outs, _, nnz = b.execute(stream=torch.cuda.Stream(), report=True)
    for o, d, r, k in zip(outs, b.dims, refs, nnz):
        assert np.array_equal(to_host(o, d), r)
        assert k == int(r.sum())


def test_autotuned_plan():
    s = inputs.config3(res=20)
    note("autotune plan", s.name)
    ref = _oracle_solve(s)
    plan = pa.Plan(s, autotune=True)                         # tuned on a cache miss
    out, rep, _ = plan.execute(report=True)
    assert np.array_equal(to_host(out, plan.dims), ref)
    assert rep["nnz_out"] == int(ref.sum())
