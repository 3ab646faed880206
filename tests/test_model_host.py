"""Host-side pieces of the learned order: the step feature map (worked by hand
on the two-relation example), argument validation, and that planning with
PA_ORDER_LEARNED refuses to run without a model."""
import numpy as np
import pytest

from paper_1609_00061_amd import inputs, pa


def test_features_of_the_two_relation_example():
    """Circle on (x0, x1), cubic on (x1, x2), 64 cells per axis, x0 and x2
    exposed.  The one step multiplies the packs {x0, x1} and {x1, x2} into
    {x0, x2}: no batch group, M = N = K = 64 (log2 6 each), scope 64^3,
    MFMA-eligible.  Each relation alone: 1 equation in 2 unknowns gives a
    curve, codimension 1 in its 2-d pack, density 2^-(6-1); the pair: 2
    equations in 3 unknowns, a curve projected onto the 2-d output pack,
    codimension 1 again."""
    s = inputs.config1()
    f = pa.step_features(s, 0b01, 0b10)
    want = np.array([0, 6 / 8, 6 / 8, 6 / 8, 18 / 8, 12 / 8, 12 / 8, 12 / 8, 1, 0, 0, 3 / 4, 2 / 4,
                     -5 / 8, -5 / 8, -5 / 8], dtype=np.float32)
    assert np.array_equal(f, want), f


def test_features_of_a_streaming_and_a_kronecker_step():
    # chain x0-x1-x2-x3 with resolutions 8, 16, 1024, 4; exposed x0, x3
    rng = inputs.SplitMix64(5)
    rels = [inputs.random_relation(rng, (0, 1)), inputs.random_relation(rng, (1, 2)),
            inputs.random_relation(rng, (2, 3))]
    s = inputs.System([(-1.0, 1.0, 8), (-1.0, 1.0, 16), (-1.0, 1.0, 1024), (-1.0, 1.0, 4)], rels, (0, 3))
    # rel0 * rel1: packs {0,1} and {1,2} -> {0,2}; K = x1 (16), M = x0 (8 < 32): streaming
    f = pa.step_features(s, 0b001, 0b010)
    assert f[8] == 0 and f[9] == 1 and f[10] == 0
    assert np.isclose(f[3], 4 / 8) and np.isclose(f[1], 3 / 8) and np.isclose(f[2], 10 / 8)
    # rel0 * rel2 share nothing: a Kronecker product into {0,1,2,3}
    f = pa.step_features(s, 0b001, 0b100)
    assert f[10] == 1 and f[3] == 0 and f[0] == 0
    assert np.isclose(f[4], (3 + 4 + 10 + 2) / 8) and np.isclose(f[12], 1.0)


def test_feature_argument_validation():
    s = inputs.config1()
    for s1, s2 in [(0, 1), (1, 0), (1, 1), (0b100, 1), (3, 2)]:
        with pytest.raises(pa.PaError):
            pa.step_features(s, s1, s2)


def test_learned_order_needs_a_model():
    d = pa.describe_plan(inputs.config2(res=32), order=pa.ORDER_LEARNED)
    assert d.get("error") == pa.PA_EINVAL


def test_model_shape_constants():
    L = pa.load()
    assert L.pa_model_n_features() == pa.MODEL_FEATURES == 16
    from oracle import mlp
    assert L.pa_model_n_params() == mlp.N_PARAMS
