"""Replayed sweeps (sbp_sweep_graph_*) against eager sweeps (sbp_nodal_sweep).

One sweep is captured once; each launch must equal the next eager sweep of
the same chain (sweep index s, s+1, ...): labels, block matrix, degrees, DL
and statistics bit for bit (the same kernels run on the same inputs).
Between replays the test runs unrelated eager work on the same stream (an
eager sweep of another graph, torch kernels) and synchronises, and every
replay is checked, not only the last.  Calls are made through the C-ABI.
"""
import numpy as np
import pytest
import torch

from paper_2305_18663_amd import gen, sbp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sbp.lib()
    yield


def _state(dg, C, lab, bm):
    coo = sbp.sbp_blockmodel_coo(dg, C, bm)
    return lab.cpu().numpy(), coo, sbp.sbp_description_length(dg, C, bm)


def _same_state(a, b):
    la, ca, da = a
    lb, cb, db = b
    assert np.array_equal(la, lb)
    for key in ("rows", "cols", "vals", "dout", "din"):
        assert np.array_equal(ca[key], cb[key]), key
    assert da == db


@pytest.mark.parametrize("case", [
    dict(g="plain_1k", C=10, n_batches=1, n_hubs=0, sweeps=4),
    dict(g="plain_1k", C=7, n_batches=3, n_hubs=0, sweeps=3),
    dict(g="dcsbm", C=45, n_batches=1, n_hubs=0, sweeps=3),
    dict(g="dcsbm", C=12, n_batches=4, n_hubs=16, sweeps=3),
    dict(g="plain_1k", C=1, n_batches=1, n_hubs=0, sweeps=2),
])
def test_replayed_sweeps_equal_eager_sweeps(case):
    g = gen.plain_1k(seed=21) if case["g"] == "plain_1k" else gen.dcsbm([3000] * 12, 240_000, 2.5, seed=22)
    other = gen.plain_1k(seed=23)
    C, nb, nh, seed, s0 = case["C"], case["n_batches"], case["n_hubs"], 17, 5
    lab0 = gen.initial_labels(g.n, C, seed=seed)
    # eager chain
    dg = sbp.DeviceGraph(g)
    lab_e = sbp.labels(lab0)
    bm_e = sbp.sbp_build_blockmodel(dg, lab_e, C)
    eager = []
    for k in range(case["sweeps"]):
        tr = sbp.sbp_nodal_sweep(dg, lab_e, C, bm_e, seed, s0 + k, n_batches=nb, n_hubs=nh, trace=False)
        eager.append((tr, _state(dg, C, lab_e, bm_e)))
    # replayed chain on fresh copies
    dg2 = sbp.DeviceGraph(g)
    lab_r = sbp.labels(lab0)
    bm_r = sbp.sbp_build_blockmodel(dg2, lab_r, C)
    do = sbp.DeviceGraph(other)
    lab_o = sbp.labels(gen.initial_labels(other.n, 6, seed=3))
    bm_o = sbp.sbp_build_blockmodel(do, lab_o, 6)
    sg = sbp.SweepGraph(dg2, lab_r, C, bm_r, seed, s0, n_batches=nb, n_hubs=nh)
    try:
        assert np.array_equal(lab_r.cpu().numpy(), lab0)  # creation runs nothing
        for k, (tr, st) in enumerate(eager):
            sg.launch()
            torch.cuda.synchronize()
            got = sg.stats()
            for key in ("proposals", "self_proposals", "accepted", "sum_dS", "dl_after"):
                assert got[key] == tr[key], (k, key)
            _same_state(_state(dg2, C, lab_r, bm_r), st)
            assert sg.sweep_index() == s0 + k + 1
            # unrelated eager work between replays
            sbp.sbp_nodal_sweep(do, lab_o, 6, bm_o, 99, k, trace=False)
            x = torch.arange(1 << 20, device="cuda", dtype=torch.float32)
            assert float((x * 2).sum()) == float(x.sum()) * 2
            torch.cuda.synchronize()
    finally:
        sg.close()


def test_replay_restarts_from_a_reset_index():
    """Setting the device index back replays the same sweep from the same state."""
    g = gen.plain_1k(seed=31)
    C, seed = 9, 4
    lab0 = gen.initial_labels(g.n, C, seed=seed)
    dg = sbp.DeviceGraph(g)
    lab = sbp.labels(lab0)
    bm = sbp.sbp_build_blockmodel(dg, lab, C)
    sg = sbp.SweepGraph(dg, lab, C, bm, seed, 0)
    try:
        sg.launch()
        first = _state(dg, C, lab, bm)
        lab.copy_(sbp.labels(lab0))
        bm2 = sbp.sbp_build_blockmodel(dg, lab, C)
        bm.copy_(bm2)
        sg.index.fill_(0)
        sg.launch()
        _same_state(_state(dg, C, lab, bm), first)
    finally:
        sg.close()


def test_graph_create_refusals():
    g = gen.plain_1k()
    dg = sbp.DeviceGraph(g)
    lab = sbp.labels(gen.initial_labels(g.n, 80, seed=1))
    bm = sbp.sbp_build_blockmodel(dg, lab, 80)
    with pytest.raises(sbp.SbpError) as ei:  # sparse tier
        sbp.SweepGraph(dg, lab, 80, bm, 1, 0)
    assert ei.value.code == -1
    lab10 = sbp.labels(gen.initial_labels(g.n, 10, seed=1))
    small = torch.zeros(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(sbp.SbpError) as ei:  # blockmodel storage too small
        sbp.SweepGraph(dg, lab10, 10, small, 1, 0)
    assert ei.value.code == -4
