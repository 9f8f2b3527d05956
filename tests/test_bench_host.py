"""Host-side pieces of bench.py that need no GPU: the bounded oracle legs of
the 256-graph batch workload (one process on one core, then a pool)."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_2305_18663_amd import gen  # noqa: E402


@pytest.mark.timeout(300)
def test_batch_oracle_legs_partition_in_order_and_match_a_direct_call():
    specs = [(60, 3100 + i, 4100 + i) for i in range(5)]
    legs = bench._start_oracle_legs(specs, budget_s=60.0)
    seq = bench._run_oracle_leg(legs["sequential"], 60.0)
    pool = bench._run_oracle_leg(legs["pool"], 60.0)
    # every graph, once each; the one-core leg takes them in the batch's order
    assert [r[0] for r in seq] == list(range(len(specs)))
    assert sorted(r[0] for r in pool) == list(range(len(specs)))
    for i, t, done, C, dl, lab in seq + pool:
        n, gseed, pseed = specs[i]
        ref = O.partition(gen.batch_graph(n, seed=gseed), seed=pseed)
        assert C == ref["C"] and dl == ref["dl"] and np.array_equal(lab, ref["lab"])
        assert 0.0 <= t <= done


@pytest.mark.timeout(300)
def test_batch_oracle_leg_starts_nothing_after_its_budget():
    specs = [(60, 3200 + i, 4200 + i) for i in range(50)]
    legs = bench._start_oracle_legs(specs, budget_s=0.0)
    out = bench._run_oracle_leg(legs["sequential"], 0.0)
    # a zero budget: the process ends before its first graph
    assert out == []
    bench._run_oracle_leg(legs["pool"], 0.0)
