"""Densities on the GPU: the per-tile set-bit counts of bit arrays (their
density maps) against numpy on the unpacked arrays, and the plot densities
a plan measures for the learned order (opts->measure_density) against the
oracle's plots."""
import math

import numpy as np
import pytest

import oracle
from paper_1609_00061_amd import inputs, pa
from gpu_util import note, to_device

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,tile", [((37, 300), (8, 4)), ((5, 7, 1000), (3, 5)), ((64, 64), (64, 2)),
                                        ((1000,), (1, 3)), ((3, 4, 5), (100, 100))])
def test_tile_popcount(shape, tile):
    A = inputs.random_bool_array(shape, 0.2, 9600 + len(shape))
    rows = int(np.prod(shape[:-1]))
    rw = pa.row_words(shape[-1])
    note("tile_popcount", shape, tile)
    got = pa.tile_popcount(to_device(A), list(shape), *tile).cpu().numpy().view(np.uint32)
    # reference: pad each row to its words, count per block
    padded = np.zeros((rows, rw * 32), dtype=np.int64)
    padded[:, :shape[-1]] = A.reshape(rows, shape[-1])
    per_word = padded.reshape(rows, rw, 32).sum(axis=2)
    tr, tw = -(-rows // tile[0]), -(-rw // tile[1])
    ref = np.zeros((tr, tw), dtype=np.int64)
    for i in range(tr):
        for j in range(tw):
            ref[i, j] = per_word[i * tile[0]:(i + 1) * tile[0], j * tile[1]:(j + 1) * tile[1]].sum()
    assert np.array_equal(got.astype(np.int64), ref)
    assert int(got.astype(np.int64).sum()) == int(A.sum())


def test_measured_plot_densities():
    """A plan with measure_density records log2(set cells / cells) of every
    relation's plot, which is the oracle plot's exact density; a relation
    with no zero in the box (x^2 + y^2 + 1 = 0) has none (null)."""
    s = inputs.config5(n_graphs=1, index=300, res=40)[0]
    s.relations.append(inputs.Relation((0, 1), 2, np.array([1.0, 0, 0, 1.0, 0, 1.0])))
    d = pa.describe_plan(s, measure_density=True)
    got = d["leaf_log2_density"]
    assert len(got) == len(s.relations)
    for r, g in zip(s.relations, got):
        P = oracle.plot(r, s.axes)[0]
        if P.sum() == 0:
            assert g is None
        else:
            assert g == pytest.approx(math.log2(P.sum() / P.size), abs=1e-12)
    assert got[-1] is None
    assert pa.describe_plan(s)["leaf_log2_density"] == []
    # the solve is unchanged (densities only steer the learned order)
    ref = oracle.solve([a[2] for a in s.axes], [r.vars for r in s.relations],
                       [oracle.plot(r, s.axes)[0] for r in s.relations], s.exposed)
    out, dims, _ = pa.solve_system(s, measure_density=True)
    from gpu_util import to_host
    assert np.array_equal(to_host(out, dims), ref)
