"""GPU parity of the learned step-time model: forward, gradient and Adam step
of the library's kernels against the float64 reference MLP, determinism,
checkpoints, and the learned-order planner (with a model whose prediction is
the naive cost it must reproduce the cost-optimal tree; with any model the
solution bits are the oracle's)."""
import os

import numpy as np
import pytest

import oracle
from oracle import mlp as ref
from paper_1609_00061_amd import inputs, pa
from gpu_util import note, to_host

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _case(seed, n):
    rng = np.random.default_rng(seed)
    p = (rng.normal(0, 0.3, ref.N_PARAMS)).astype(np.float32)
    X = rng.normal(0, 1.0, (n, ref.F)).astype(np.float32)
    T = rng.normal(0, 2.0, n).astype(np.float32)
    return p, X, T


def _rel_err(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("n", [1, 63, 257, 4099])
def test_forward_and_gradient_match_reference(n):
    """float32 kernels vs the float64 reference on the same float32 inputs:
    normwise relative error <= 1e-4 for predictions, loss and gradient."""
    import torch
    p, X, T = _case(n, n)
    note("mlp grad", n)
    m = pa.Model(seed=1)
    m.set_params(p)
    assert np.array_equal(m.get_params(), p)
    y = m.forward(_dev(X)).cpu().numpy()
    y_ref, _ = ref.forward(p.astype(np.float64), X.astype(np.float64))
    assert _rel_err(y, y_ref) <= 1e-4
    G, loss = m.gradient(_dev(X), _dev(T))
    g_ref = ref.grad(p.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
    assert _rel_err(G.cpu().numpy(), g_ref) <= 1e-4
    assert abs(loss - ref.loss(p.astype(np.float64), X, T)) <= 1e-4 * max(1.0, abs(loss))
    # every block of the gradient, not only the norm
    o = 0
    for size in (ref.H * ref.F, ref.H, ref.H * ref.H, ref.H, ref.H, 1):
        gb, rb = G.cpu().numpy()[o:o + size], g_ref[o:o + size]
        assert np.linalg.norm(gb - rb) <= 1e-4 * max(np.linalg.norm(g_ref), 1e-30), o
        o += size
    torch.cuda.synchronize()


def test_gradient_is_deterministic():
    p, X, T = _case(7, 3000)
    m = pa.Model()
    m.set_params(p)
    g1, _ = m.gradient(_dev(X), _dev(T))
    g2, _ = m.gradient(_dev(X), _dev(T))
    assert np.array_equal(g1.cpu().numpy(), g2.cpu().numpy())


def test_adam_steps_match_reference():
    p, X, T = _case(11, 500)
    m = pa.Model()
    m.set_params(p)
    pr = p.astype(np.float64)
    mm = np.zeros_like(pr)
    vv = np.zeros_like(pr)
    Xd, Td = _dev(X), _dev(T)
    for step in range(1, 6):
        m.train_step(Xd, Td, lr=1e-3)
        pr, mm, vv = ref.adam(pr, ref.grad(pr, X.astype(np.float64), T.astype(np.float64)), mm, vv, step, lr=1e-3)
        got = m.get_params().astype(np.float64)
        # each step moves a parameter by at most ~lr; sign decisions of tiny
        # gradients may differ between float32 and float64
        assert np.max(np.abs(got - pr)) <= 2e-3 * step, step
        assert _rel_err(got - p, pr - p) <= 5e-2, step


def test_training_reduces_loss():
    rng = np.random.default_rng(3)
    X = rng.normal(0, 1, (2048, ref.F)).astype(np.float32)
    T = (0.5 * X[:, 0] - X[:, 3] + 0.25 * X[:, 4] * X[:, 5] + 3.0).astype(np.float32)
    m = pa.Model(seed=5)
    Xd, Td = _dev(X), _dev(T)
    l0 = m.train_step(Xd, Td, lr=3e-3, want_loss=True)
    for _ in range(400):
        m.train_step(Xd, Td, lr=3e-3)
    l1 = m.train_step(Xd, Td, lr=3e-3, want_loss=True)
    assert l1 < 0.02 * l0, (l0, l1)


def test_checkpoint_round_trip(tmp_path):
    p, _, _ = _case(13, 1)
    m = pa.Model()
    m.set_params(p)
    path = str(tmp_path / "order_model.bin")
    m.save(path)
    m2 = pa.Model(path=path)
    assert np.array_equal(m2.get_params(), p)
    with open(path, "rb") as f:
        head = f.readline()
    assert b'"format": "pa-order-mlp"' in head
    bad = str(tmp_path / "bad.bin")
    with open(bad, "wb") as f:
        f.write(head + b"\x00" * 12)
    with pytest.raises(pa.PaError):
        pa.Model(path=bad)


def _naive_cost_model():
    """Parameters whose prediction is log2 of the step's scope size (the
    naive cost r^L): one hidden path carrying feature 4 (log2 scope / 8)."""
    W1 = np.zeros((ref.H, ref.F)); W1[0, 4] = 1.0
    W2 = np.zeros((ref.H, ref.H)); W2[0, 0] = 1.0
    w3 = np.zeros(ref.H); w3[0] = 8.0
    m = pa.Model()
    m.set_params(ref.pack(W1, np.zeros(ref.H), W2, np.zeros(ref.H), w3, 0.0).astype(np.float32))
    m.set_level_cost(0.0)
    return m


def _systems():
    out = [inputs.config1(), inputs.config2(res=64), inputs.config3(res=16)]
    out += inputs.config4(n_systems=4, index=3, rmin=8, rmax=64)
    out += inputs.config5(n_graphs=6, index=901, res=6)
    return out


@pytest.mark.parametrize("si", range(13))
def test_learned_order_with_naive_model(si):
    s = _systems()[si]
    m = _naive_cost_model()
    note("learned naive", s.name)
    d_l = pa.describe_plan(s, order=pa.ORDER_LEARNED, model=m)
    d_e = pa.describe_plan(s, order=pa.ORDER_EXHAUSTIVE)
    # exhaustive ranges over every tree, learned over trees of connected
    # clusters; chains and the cyclic four-relation system have connected optima
    assert d_l["cost"] >= d_e["cost"] * (1 - 1e-12)
    if si < 7:
        assert d_l["cost"] <= d_e["cost"] * (1 + 1e-6)
    assert d_l["predicted_us"] > 0
    ref_bits = oracle.solve([a[2] for a in s.axes], [r.vars for r in s.relations],
                            [oracle.plot(r, s.axes)[0] for r in s.relations], s.exposed)
    out, dims, _ = pa.solve_system(s, order=pa.ORDER_LEARNED, model=m)
    assert np.array_equal(to_host(out, dims), ref_bits)


def test_step_samples_from_timed_plan():
    s = inputs.config3(res=24)
    plan = pa.Plan(s, per_op=True, timing=2)
    plan.execute()
    X, T = pa.plan_step_samples(plan)
    assert X.shape == (len(s.relations) - 1, pa.MODEL_FEATURES)
    assert np.all(np.isfinite(T))
    d = pa.describe_plan(s)
    merges = d["merges"]
    # the features of every sample are those of its tree node
    n = len(s.relations)
    leaves = [1 << i for i in range(n)]
    for t in range(n - 1):
        a, b = merges[2 * t], merges[2 * t + 1]
        assert np.array_equal(X[t], pa.step_features(s, leaves[a], leaves[b]))
        leaves.append(leaves[a] | leaves[b])
