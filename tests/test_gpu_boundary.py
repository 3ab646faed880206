"""GPU tests of the C ABI's whole-system entry points, called directly:
pa_solve_system and pa_solve_batch against the oracle with their reports,
pa_workspace_bytes against the plans it sizes (and a caller-owned workspace
of exactly that size), repeated executions of one plan into new outputs on a
non-blocking stream without synchronizing in between, and the LDS read-rate
reference."""
import numpy as np
import pytest

import oracle
from paper_1609_00061_amd import inputs, pa
from gpu_util import note, to_host

pytestmark = pytest.mark.gpu


def _oracle_solve(s):
    plots = [oracle.plot(r, s.axes)[0] for r in s.relations]
    return oracle.solve([a[2] for a in s.axes], [r.vars for r in s.relations], plots, s.exposed)


def _small_system(seed):
    rng = inputs.SplitMix64(seed)
    g = inputs.random_hypergraph(rng, res=rng.randint(6, 20))
    g.axes = [(-3.0, 3.0, rng.randint(3, 36)) for _ in g.axes]
    g.name = f"boundary{seed}"
    return g


def _corners(s):
    tot = 0
    for r in s.relations:
        c = 1
        for v in r.vars:
            c *= s.axes[v][2] + 1
        tot += c
    return tot


@pytest.mark.parametrize("seed", range(4))
def test_solve_system_direct(seed):
    s = inputs.config1() if seed == 0 else _small_system(5100 + seed)
    ref = _oracle_solve(s)
    for kw in (dict(), dict(order=pa.ORDER_GREEDY, plain=True), dict(precision=pa.PLOT_FP64)):
        note("pa_solve_system", s.name, kw)
        out, dims, rep = pa.solve_system(s, **kw)
        assert np.array_equal(to_host(out, dims), ref), kw
        assert rep["nnz_out"] == int(ref.sum())
        assert rep["corners"] == _corners(s)
        assert rep["n_steps"] >= 1


def test_solve_batch_direct():
    """pa_solve_batch over uneven chains and random hypergraphs: every output
    is the oracle's; per-system reports carry each system's set bits, corner
    count and escalations, the latter equal to solving it alone."""
    systems = inputs.config4(n_systems=10, index=11, rmin=8, rmax=80) + [_small_system(5200 + i) for i in range(6)]
    refs = [_oracle_solve(s) for s in systems]
    for kw in (dict(), dict(graph=True), dict(single_launch=True), dict(order=pa.ORDER_GREEDY, sparse_pass=2)):
        note("pa_solve_batch", len(systems), kw)
        outs, dims, reps = pa.solve_batch(systems, **kw)
        for i, (o, d, ref) in enumerate(zip(outs, dims, refs)):
            assert np.array_equal(to_host(o, d), ref), (i, kw)
            assert reps[i]["nnz_out"] == int(ref.sum())
            assert reps[i]["corners"] == _corners(systems[i])
    alone = [pa.solve_system(s)[2]["corners_flagged"] for s in systems]
    assert [r["corners_flagged"] for r in reps] == alone


@pytest.mark.parametrize("kw", [dict(), dict(order=pa.ORDER_GREEDY), dict(sparse_pass=2), dict(plain=True),
                                dict(single_launch=True)])
def test_workspace_bytes(kw):
    """pa_workspace_bytes (host planning, no allocation) equals the workspace
    of the plan it describes; a caller-owned workspace of exactly that size
    runs the solve, one 256 bytes smaller is refused with PA_ENOMEM."""
    import torch
    s = inputs.config2(res=96, n_rel=5)
    need = pa.workspace_bytes(s, **kw)
    assert need == pa.Plan(s, **kw).workspace_bytes()
    ref = _oracle_solve(s)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    note("workspace", need, kw)
    out, dims, _ = pa.solve_system(s, workspace=ws, **kw)
    assert np.array_equal(to_host(out, dims), ref)
    small = ws[: need - 256]
    with pytest.raises(pa.PaError) as e:
        pa.solve_system(s, workspace=small, **kw)
    assert e.value.code == pa.PA_ENOMEM


@pytest.mark.parametrize("graph", [False, True])
def test_new_outputs_without_sync(graph):
    """One plan executed into three different outputs back to back on a
    non-blocking stream, then again on a second stream, with no
    synchronization in between: the step table and graph rewrites wait for
    the earlier executions, and every output holds the oracle's bits."""
    import torch
    s = inputs.config2(res=160, n_rel=6)
    ref = _oracle_solve(s)
    p = pa.Plan(s, graph=graph)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = [pa.empty_bits(p.dims) for _ in range(4)]
    torch.cuda.synchronize()          # the zero fills above ran on the default stream
    for o in outs[:3]:
        p.execute(o, stream=s1)
    p.execute(outs[3], stream=s2)
    p.execute(outs[0], stream=s2)
    torch.cuda.synchronize()
    for o in outs:
        assert np.array_equal(to_host(o, p.dims), ref)


def test_lds_read_rate():
    """pa_lds_read_rate (the reference of the fused step's LDS roofline): a
    finite positive rate, at most the device's LDS read capacity of 256
    bytes per clock per CU at a 2.4 GHz clock (with headroom for a higher
    clock); a null output pointer is refused with PA_EINVAL."""
    import ctypes
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    r = pa.lds_read_rate()
    note("lds read rate", r, "bytes/s on", cus, "CUs")
    assert 0.0 < r < 256.0 * cus * 3.0e9
    L = pa.load()
    assert L.pa_lds_read_rate(None, None) == pa.PA_EINVAL
