"""The launch-shape autotuner: every candidate shape gives the same chain of
sweeps (bit for bit), the cache round-trips through JSON, and a tuned run
equals a default run."""
import json

import numpy as np
import pytest
import torch

from paper_2305_18663_amd import autotune, gen, sbp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sbp.lib()
    yield
    autotune.set_knobs(autotune.DEFAULTS)


def test_tuner_picks_a_shape_and_results_do_not_depend_on_it(tmp_path):
    g = gen.dcsbm([3000] * 10, 200_000, 2.5, seed=41)
    C = 10
    dg = sbp.DeviceGraph(g)
    lab0 = gen.initial_labels(g.n, C, seed=5)
    cand = {"dense_eval_workgroups": [0, 128], "dense_delta_workgroups": [64, 512],
            "dense_update_moved_share": [128, -1]}
    knobs, table = autotune.tune_graph(dg, lab0, C, sweeps=4, repeats=1, candidates=cand)
    assert len(table) == 8 and knobs in [k for _, k in table]
    path = str(tmp_path / "tune.json")
    autotune.record(path, g.n, g.e, C, 1, knobs, table)
    cache = json.load(open(path))
    assert cache[autotune.size_bin(g.n, g.e, C, 1)]["knobs"] == knobs
    # a tuned chain equals a default chain
    got = autotune.apply(path, g.n, g.e, C, 1)
    assert got == {**autotune.DEFAULTS, **knobs}
    tuned, lab_t = autotune._time_chain(dg, lab0, C, 9, 3, 1, 1)
    autotune.set_knobs(autotune.DEFAULTS)
    plain, lab_p = autotune._time_chain(dg, lab0, C, 9, 3, 1, 1)
    assert np.array_equal(lab_t, lab_p)
