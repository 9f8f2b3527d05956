"""The allocation-free sweep (sbp_nodal_sweep_static) against sbp_nodal_sweep.

Two calls in a row on one GPU, the second with a smaller graph: the static
scratch keeps the first call's contents, and the second must not read them.
Every output is compared with the workspace entry point's on the same
inputs: labels, block matrix and degrees bit for bit, DL changes within
1e-9, decisions equal (no near-tie allowance is needed: both run the same
kernels).  Calls are made through the C-ABI.
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


def _run(g, C, seed, sweeps, static, n_batches=1):
    dg = sbp.DeviceGraph(g)
    lab = sbp.labels(gen.initial_labels(g.n, C, seed=seed))
    bm = sbp.sbp_build_blockmodel(dg, lab, C)
    out = []
    for k in range(sweeps):
        tr = sbp.sbp_nodal_sweep(dg, lab, C, bm, seed, k, n_batches=n_batches, static=static)
        coo = sbp.sbp_blockmodel_coo(dg, C, bm)
        out.append((tr, lab.cpu().numpy(), coo, sbp.sbp_description_length(dg, C, bm)))
    return out


def _same(a, b):
    for (ta, la, ca, da), (tb, lb, cb, db) in zip(a, b):
        assert np.array_equal(la, lb)
        for key in ("rows", "cols", "vals", "dout", "din"):
            assert np.array_equal(ca[key], cb[key]), key
        assert da == db
        assert np.array_equal(ta["prop"], tb["prop"]) and np.array_equal(ta["accept"], tb["accept"])
        assert np.all(np.abs(ta["dS"] - tb["dS"]) <= 1e-9 * np.maximum(np.abs(tb["dS"]), 1.0))
        for key in ("proposals", "self_proposals", "accepted"):
            assert ta[key] == tb[key]
        assert ta["dl_after"] == tb["dl_after"]


def test_static_sweep_matches_workspace_sweep_twice():
    big = gen.dcsbm([4000] * 12, 400_000, 2.5, seed=8)
    small = gen.plain_1k(seed=12)
    for g, C, seed, sweeps, nb in ((big, 45, 3, 3, 1), (small, 10, 4, 3, 1), (small, 7, 5, 2, 3)):
        ref = _run(g, C, seed, sweeps, static=False, n_batches=nb)
        got = _run(g, C, seed, sweeps, static=True, n_batches=nb)
        _same(got, ref)


def test_static_sweep_rejects_before_any_work():
    g = gen.plain_1k()
    dg = sbp.DeviceGraph(g)
    lab = sbp.labels(gen.initial_labels(g.n, 80, seed=1))
    bm = sbp.sbp_build_blockmodel(dg, lab, 80)
    before = lab.cpu().numpy().copy()
    with pytest.raises(sbp.SbpError) as ei:  # sparse tier
        sbp.sbp_nodal_sweep(dg, lab, 80, bm, 1, 0, static=True)
    assert ei.value.code == -1
    lab10 = sbp.labels(gen.initial_labels(g.n, 10, seed=1))
    bm10 = sbp.sbp_build_blockmodel(dg, lab10, 10)
    with pytest.raises(sbp.SbpError) as ei:  # hub pass
        sbp.sbp_nodal_sweep(dg, lab10, 10, bm10, 1, 0, n_hubs=3, static=True)
    assert ei.value.code == -1
    assert np.array_equal(lab.cpu().numpy(), before)
    # more vertices than the scratch holds: refused from the sizes alone
    n = (1 << 20) + 1
    huge = gen.from_edges(n, [0, 1], [1, 0])
    dh = sbp.DeviceGraph(huge)
    labh = sbp.labels(np.zeros(n, np.int32))
    bmh = sbp.sbp_build_blockmodel(dh, labh, 2)
    with pytest.raises(sbp.SbpError) as ei:
        sbp.sbp_nodal_sweep(dh, labh, 2, bmh, 1, 0, static=True)
    assert ei.value.code == -6
