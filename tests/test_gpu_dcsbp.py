"""Divide-and-conquer SBP (Alg. 3) on the GPU against the oracle's twin.

Every stage is integer or quantised: the subgraph partitions (bit-exact
whole-method runs), the combination choices (floor(dS_local 2^20) keys) and
the final run on the full graph.  The labels, the block counts of every
subgraph and of the result must match exactly; the DL within 1e-9.
Calls go through the C-ABI.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2305_18663_amd import gen, sbp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sbp.lib()
    yield


def _parity(g, s, **kw):
    got = sbp.sbp_dcsbp(sbp.DeviceGraph(g), s, **kw)
    ref = O.dcsbp(g, s, **kw)
    assert np.array_equal(got["sub_C"], ref["sub_C"]), (got["sub_C"], ref["sub_C"])
    assert got["C"] == ref["C"]
    assert np.array_equal(got["lab"], ref["lab"])
    assert abs(got["dl"] - ref["dl"]) <= 1e-9 * abs(ref["dl"])
    return got


@pytest.mark.parametrize("s", [1, 2, 3, 8])
def test_dcsbp_1k(s):
    _parity(gen.plain_1k(seed=61), s, seed=21)


@pytest.mark.parametrize("s", [2, 5, 9])
def test_dcsbp_planted(s):
    g = gen.dcsbm([120] * 6, 14000, 5.0, seed=62, kmin=8, kmax=100)
    res = _parity(g, s, seed=22)
    if s == 2:
        from paper_2305_18663_amd import ablation
        assert ablation.nmi(res["lab"], g.planted) > 0.9


def test_dcsbp_one_batch_per_sweep():
    _parity(gen.plain_1k(seed=63), 6, seed=23, n_batches=1)


def test_dcsbp_hybrid_hubs():
    _parity(gen.plain_1k(seed=64), 3, seed=24, n_hubs=5)


def test_dcsbp_degenerate():
    # every subgraph a single vertex; an edgeless graph; a multigraph with self-loops
    g = gen.random_multigraph(12, 60, seed=5)
    _parity(g, 12, seed=3)
    _parity(gen.from_edges(7, [], []), 3, seed=4)
    _parity(gen.random_multigraph(300, 2500, seed=6), 7, seed=5)


def test_dcsbp_refusals():
    dg = sbp.DeviceGraph(gen.random_multigraph(10, 30, seed=1))
    for s in (0, 11):
        with pytest.raises(sbp.SbpError) as ei:
            sbp.sbp_dcsbp(dg, s)
        assert ei.value.code == -1
