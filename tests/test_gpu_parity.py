"""GPU (HIP, gfx950) against the CPU oracle, element by element.

Bar: integer state (block matrix, degrees, labels, proposals, block counts)
bit-exact; FP64 DL changes within 1e-9 relative (floor of 1 nat); accept
decisions equal except near ties |margin| < 1e-9, where the oracle adopts
the GPU's decision and the event is counted.
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2305_18663_amd import gen, sbp

pytestmark = pytest.mark.gpu

RTOL = 1e-9


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sbp.lib()
    yield


def close(a, b, rtol=RTOL):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.all(np.abs(a - b) <= rtol * np.maximum(np.abs(b), 1.0))


GRAPHS = {
    "plain_1k": lambda: gen.plain_1k(),
    "multi_selfloops": lambda: gen.random_multigraph(300, 2500, seed=5, self_loops=True),
    "dcsbm_2k": lambda: gen.dcsbm([400] * 5, 30000, 3.0, seed=9, kmax=300),
}


def check_coo(dg, g, lab, C, bm):
    got = sbp.sbp_blockmodel_coo(dg, C, bm)
    ref = O.build_blockmodel(g, lab, C)
    assert np.array_equal(got["rows"], ref["rows"])
    assert np.array_equal(got["cols"], ref["cols"])
    assert np.array_equal(got["vals"], ref["vals"])
    assert np.array_equal(got["dout"], ref["dout"]) and np.array_equal(got["din"], ref["din"])
    return ref


# ---------------------------------------------------------------- graph ingest
@pytest.mark.parametrize("case", ["multi_selfloops", "plain_1k", "edgeless", "single", "200k"])
def test_graph_from_edges(case):
    g = {"multi_selfloops": lambda: gen.random_multigraph(300, 2500, seed=5, self_loops=True),
         "plain_1k": gen.plain_1k, "edgeless": lambda: gen.from_edges(7, [], []),
         "single": lambda: gen.from_edges(1, [0, 0], [0, 0]), "200k": gen.sweep_200k}[case]()
    src, dst = g.edges()
    rng = np.random.default_rng(1)
    perm = rng.permutation(g.e)  # any edge order gives the same canonical arrays
    dg = sbp.sbp_graph_from_edges(g.n, src[perm], dst[perm])
    assert np.array_equal(dg.out_ptr.cpu().numpy(), g.out_ptr)
    assert np.array_equal(dg.in_ptr.cpu().numpy(), g.in_ptr)
    assert np.array_equal(dg.out_idx.cpu().numpy()[: g.e], g.out_idx)
    assert np.array_equal(dg.in_idx.cpu().numpy()[: g.e], g.in_idx)
    sbp.sbp_validate_graph(dg)


def test_graph_from_edges_rejects_bad_endpoint():
    with pytest.raises(sbp.SbpError) as ei:
        sbp.sbp_graph_from_edges(5, [0, 1, 5], [1, 2, 0])
    assert ei.value.code == -2


# ---------------------------------------------------------------- blockmodel + DL
@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("C", [1, 7, 45, 64, 65, 300])
def test_blockmodel_and_dl(name, C):
    g = GRAPHS[name]()
    if C > g.n:
        pytest.skip("C > n")
    lab0 = gen.initial_labels(g.n, C, seed=C)
    dg = sbp.DeviceGraph(g)
    lab = sbp.labels(lab0)
    bm = sbp.sbp_build_blockmodel(dg, lab, C)
    ref = check_coo(dg, g, lab0, C, bm)
    assert close(sbp.sbp_description_length(dg, C, bm), ref["dl"], 1e-12)


def test_blockmodel_all_singletons():
    g = GRAPHS["multi_selfloops"]()
    dg = sbp.DeviceGraph(g)
    lab0 = np.arange(g.n, dtype=np.int32)
    bm = sbp.sbp_build_blockmodel(dg, sbp.labels(lab0), g.n)
    ref = check_coo(dg, g, lab0, g.n, bm)
    assert close(sbp.sbp_description_length(dg, g.n, bm), ref["dl"], 1e-12)


def test_blockmodel_200k_full_size():
    g = gen.sweep_200k()
    lab0 = gen.initial_labels(g.n, 45, seed=2001)
    dg = sbp.DeviceGraph(g)
    bm = sbp.sbp_build_blockmodel(dg, sbp.labels(lab0), 45)
    ref = check_coo(dg, g, lab0, 45, bm)
    assert close(sbp.sbp_description_length(dg, 45, bm), ref["dl"], 1e-12)
    # sparse tier at the same size
    lab1 = gen.initial_labels(g.n, 5000, seed=7)
    bm1 = sbp.sbp_build_blockmodel(dg, sbp.labels(lab1), 5000)
    ref1 = check_coo(dg, g, lab1, 5000, bm1)
    assert close(sbp.sbp_description_length(dg, 5000, bm1), ref1["dl"], 1e-12)


# ---------------------------------------------------------------- sweeps
def sweep_parity(g, lab0, C, seed, sweep, n_batches=1, beta=3.0, eps=1, dg=None, n_hubs=0):
    dg = dg or sbp.DeviceGraph(g)
    lab = sbp.labels(lab0)
    bm = sbp.sbp_build_blockmodel(dg, lab, C)
    tr = sbp.sbp_nodal_sweep(dg, lab, C, bm, seed, sweep, beta=beta, eps=eps, n_batches=n_batches, n_hubs=n_hubs)
    near = np.abs(tr["margin"]) < 1e-9
    force = np.full(g.n, -1, np.int8)
    force[near] = tr["accept"][near]
    ref = O.nodal_sweep(g, lab0, C, seed, sweep, beta=beta, eps=eps, n_batches=n_batches, force=force,
                        n_hubs=n_hubs)
    assert np.array_equal(tr["prop"], ref["prop"]), "proposals differ"
    noop = tr["prop"] == lab0
    assert close(tr["dS"][~noop], ref["dS"][~noop]), "dS differs"
    assert close(tr["lnH"][~noop], ref["lnH"][~noop]), "lnH differs"
    assert np.array_equal(tr["accept"], ref["acc"]), "accept decisions differ"
    new = lab.cpu().numpy()
    assert np.array_equal(new, ref["lab"]), "labels differ"
    assert tr["proposals"] == g.n and tr["accepted"] == ref["accepted"]
    assert tr["self_proposals"] == ref["self_proposals"]
    assert close([tr["sum_dS"]], [ref["sum_dS"]])
    refbm = check_coo(dg, g, new, C, bm)
    assert close([tr["dl_after"]], [refbm["dl"]], 1e-12)
    return new, int(near.sum()), ref


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("C", [3, 45, 64, 65, 200])
def test_sweep_parity(name, C):
    g = GRAPHS[name]()
    lab0 = gen.initial_labels(g.n, C, seed=C + 1)
    sweep_parity(g, lab0, C, seed=123, sweep=C)


@pytest.mark.parametrize("C", [16, 17, 32, 33, 48, 49])
@pytest.mark.parametrize("n_batches", [1, 3])
def test_sweep_parity_at_capacity_edges(C, n_batches):
    # the dense evaluation is built for block capacities 16, 32, 48 and 64
    # (four-lane scoring groups up to 48, eight beyond): both sides of every
    # boundary, one batch (end bytes) and several (labels gathered)
    g = GRAPHS["dcsbm_2k"]()
    lab0 = gen.initial_labels(g.n, C, seed=C + 5)
    sweep_parity(g, lab0, C, seed=31, sweep=C, n_batches=n_batches)


@pytest.mark.parametrize("C", [10, 80])
@pytest.mark.parametrize("n_batches", [2, 7])
def test_sweep_batches(C, n_batches):
    g = GRAPHS["plain_1k"]()
    lab0 = gen.initial_labels(g.n, C, seed=4)
    sweep_parity(g, lab0, C, seed=9, sweep=3, n_batches=n_batches)


@pytest.mark.parametrize("C", [3, 70])
def test_sweep_sequential_tiny(C):
    g = gen.random_multigraph(90, 400, seed=3, self_loops=True)
    lab0 = gen.initial_labels(g.n, C, seed=2)
    sweep_parity(g, lab0, C, seed=5, sweep=0, n_batches=g.n, beta=1.0)


def test_sweep_eps_and_beta():
    g = GRAPHS["plain_1k"]()
    lab0 = gen.initial_labels(g.n, 12, seed=1)
    sweep_parity(g, lab0, 12, seed=8, sweep=1, beta=1.0, eps=0)
    sweep_parity(g, lab0, 12, seed=8, sweep=2, beta=10.0, eps=3)


def test_sweep_isolated_vertices():
    g = gen.from_edges(50, [0, 1, 2, 3], [1, 2, 3, 0])  # 46 isolated vertices
    for C in (4, 49):
        lab0 = gen.initial_labels(g.n, C, seed=C)
        sweep_parity(g, lab0, C, seed=2, sweep=0)


def test_sweeps_200k_full_size():
    # the measured workload: 200k vertices, 45 blocks, consecutive sweeps
    g = gen.sweep_200k()
    lab0 = gen.initial_labels(g.n, 45, seed=2001)
    dg = sbp.DeviceGraph(g)
    lab = lab0
    ties = 0
    for k in range(2):
        lab, near, _ = sweep_parity(g, lab, 45, seed=2001, sweep=k, dg=dg)
        ties += near
    print(f"near ties logged: {ties}")


def test_sweep_200k_sparse_tier():
    g = gen.sweep_200k()
    lab0 = gen.initial_labels(g.n, 500, seed=3)
    sweep_parity(g, lab0, 500, seed=17, sweep=0)


def chain_step(g, dg, lab, cur, C, bm, seed, k, n_hubs=0):
    """One sweep on the device blockmodel carried over from the previous sweep,
    checked against the oracle started from the current labels."""
    tr = sbp.sbp_nodal_sweep(dg, lab, C, bm, seed, k, n_hubs=n_hubs)
    near = np.abs(tr["margin"]) < 1e-9
    force = np.full(g.n, -1, np.int8)
    force[near] = tr["accept"][near]
    ref = O.nodal_sweep(g, cur, C, seed, k, force=force, n_hubs=n_hubs)
    assert np.array_equal(tr["prop"], ref["prop"]), f"proposals differ at sweep {k}"
    assert np.array_equal(tr["accept"], ref["acc"]), f"decisions differ at sweep {k}"
    new = lab.cpu().numpy()
    assert np.array_equal(new, ref["lab"]), f"labels differ at sweep {k}"
    check_coo(dg, g, new, C, bm)
    return new


@pytest.mark.parametrize("share", [1024, -1])
@pytest.mark.parametrize("name,C", [("plain_1k", 10), ("multi_selfloops", 12), ("dcsbm_2k", 40)])
def test_sweep_chain_update_modes(name, C, share):
    # consecutive one-batch dense sweeps on one blockmodel, the update forced to
    # the move-driven path (1024: the moved vertices' edges, mirror end bytes)
    # or to the pass over every edge end (-1); every sweep reads the end bytes
    # the previous update left
    g = GRAPHS[name]()
    dg = sbp.DeviceGraph(g)
    cur = gen.initial_labels(g.n, C, seed=C + 11)
    lab = sbp.labels(cur)
    bm = sbp.sbp_build_blockmodel(dg, lab, C)
    sbp.sbp_tune("dense_update_moved_share", share)
    try:
        for k in range(5):
            cur = chain_step(g, dg, lab, cur, C, bm, 77, k)
    finally:
        sbp.sbp_tune("dense_update_moved_share", 64)


def test_sweeps_200k_chain_default_update():
    # 60 sweeps of the measured workload with the default update choice (the
    # pass over every edge end while many vertices move, the move-driven path
    # once few do), then two sweeps checked against the oracle
    g = gen.sweep_200k()
    C, seed = 45, 2001
    dg = sbp.DeviceGraph(g)
    lab = sbp.labels(gen.initial_labels(g.n, C, seed=seed))
    bm = sbp.sbp_build_blockmodel(dg, lab, C)
    accepted = [sbp.sbp_nodal_sweep(dg, lab, C, bm, seed, k, trace=False, stats=True)["accepted"]
                for k in range(60)]
    # both update paths ran: the default threshold is 64/1024 of the vertices
    assert max(accepted) * 1024 > 64 * g.n and min(accepted) * 1024 <= 64 * g.n, accepted
    cur = lab.cpu().numpy()
    for k in range(60, 62):
        cur = chain_step(g, dg, lab, cur, C, bm, seed, k)


def _state(dg, lab, C, bm):
    coo = sbp.sbp_blockmodel_coo(dg, C, bm)
    dl = sbp.sbp_description_length(dg, C, bm)
    return lab.cpu().numpy(), coo, dl


@pytest.mark.parametrize("mode", ["default", "moved", "every_end", "hubs"])
def test_sweeps_200k_traced_equals_untraced(mode):
    # the benchmark runs the evaluation without the per-vertex record; the
    # oracle comparisons run it with the record.  From one start on two copies
    # the two must stay bit-identical (labels, M, block degrees, DL) for 24
    # sweeps, and the last sweep must still match the oracle.
    g = gen.sweep_200k()
    C, seed = 45, 2001
    n_hubs = 16 if mode == "hubs" else 0
    dg = sbp.DeviceGraph(g)
    lab0 = gen.initial_labels(g.n, C, seed=seed)
    la, lb = sbp.labels(lab0), sbp.labels(lab0)
    ba, bb = sbp.sbp_build_blockmodel(dg, la, C), sbp.sbp_build_blockmodel(dg, lb, C)
    share = {"default": 64, "moved": 1024, "every_end": -1, "hubs": 64}[mode]
    sbp.sbp_tune("dense_update_moved_share", share)
    try:
        for k in range(24):
            ta = sbp.sbp_nodal_sweep(dg, la, C, ba, seed, k, trace=True, stats=True, n_hubs=n_hubs)
            sbp.sbp_nodal_sweep(dg, lb, C, bb, seed, k, trace=False, stats=False, n_hubs=n_hubs)
            if k % 6 == 5 or k == 0:
                A, B = _state(dg, la, C, ba), _state(dg, lb, C, bb)
                assert np.array_equal(A[0], B[0]), f"labels differ after sweep {k}"
                for key in ("rows", "cols", "vals", "dout", "din"):
                    assert np.array_equal(A[1][key], B[1][key]), f"{key} differs after sweep {k}"
                assert A[2] == B[2], f"DL differs after sweep {k}"
                assert ta["dl_after"] == B[2]
        cur = lb.cpu().numpy()
        chain_step(g, dg, lb, cur, C, bb, seed, 24, n_hubs=n_hubs)
    finally:
        sbp.sbp_tune("dense_update_moved_share", 64)


def hub_tail_graph(n=120_000):
    """The 1M-vertex workload's shape at reduced size: mean out-degree 8,
    Dirichlet block sizes, ratio 1.5 and a power-law hub tail up to a few
    thousand edge ends."""
    return gen.sparse_1m(seed=1102, n=n, e=8 * n, nb=60, max_degree=4000)


@pytest.mark.parametrize("C", [60_000, 3000, 120])
def test_sweep_sparse_hub_tail(C):
    g = hub_tail_graph()
    deg = np.diff(g.out_ptr) + np.diff(g.in_ptr)
    assert deg.max() > 1000  # the tail reaches the per-workgroup hub path
    dg = sbp.DeviceGraph(g)
    lab = gen.initial_labels(g.n, C, seed=C + 5)
    for sweep in range(2):
        lab, _, _ = sweep_parity(g, lab, C, seed=61, sweep=sweep, dg=dg)


def hub_graph():
    """24k vertices with five hubs of 500 to 15000 edge ends over a sparse
    random background: against thousands of blocks their distinct neighbour
    blocks fill all four, some or only one of the joined lists, in LDS and in
    the global slot."""
    rng = np.random.default_rng(77)
    n = 24000
    src, dst = [], []
    for h, (ko, ki) in enumerate([(300, 200), (1500, 1400), (2600, 2000), (4200, 3000), (9000, 6000)]):
        src += [h] * ko + list(rng.integers(0, n, ki))
        dst += list(rng.integers(0, n, ko)) + [h] * ki
    src += list(rng.integers(0, n, 60000))
    dst += list(rng.integers(0, n, 60000))
    return gen.from_edges(n, src, dst)


@pytest.mark.parametrize("C", [20000, 9000, 600])
def test_sweep_hubs_many_blocks(C):
    g = hub_graph()
    dg = sbp.DeviceGraph(g)
    lab0 = gen.initial_labels(g.n, C, seed=C)
    for sweep in range(3):
        sweep_parity(g, lab0, C, seed=41, sweep=sweep, dg=dg)


# ------------------------------------------------ hybrid (hubs one at a time)
@pytest.mark.parametrize("n_batches", [1, 3])
@pytest.mark.parametrize("n_hubs", [1, 7, 60])
@pytest.mark.parametrize("name,C", [("plain_1k", 10), ("multi_selfloops", 12), ("dcsbm_2k", 40)])
def test_sweep_hybrid_hubs(name, C, n_hubs, n_batches):
    # the n_hubs highest-degree vertices move one at a time, each against the
    # moves of the ones before it, then the others in asynchronous batches
    g = GRAPHS[name]()
    lab0 = gen.initial_labels(g.n, C, seed=C + 3)
    _, _, ref = sweep_parity(g, lab0, C, seed=31, sweep=n_hubs, n_batches=n_batches, n_hubs=n_hubs)
    order = O.hub_order(g, n_hubs)
    assert ref["proposals"] == g.n and len(order) == n_hubs


def test_sweep_hybrid_all_hubs_is_sequential():
    # every vertex a hub: the sequential sweep (one vertex per batch, in
    # degree order), on multi-edges and self-loops, dense blocks up to 64
    g = gen.random_multigraph(90, 400, seed=3, self_loops=True)
    for C in (3, 64):
        lab0 = gen.initial_labels(g.n, C, seed=C)
        sweep_parity(g, lab0, C, seed=5, sweep=1, beta=1.0, n_hubs=g.n)


def test_sweep_hybrid_chain():
    # consecutive hybrid sweeps on one blockmodel, the update forced to the
    # move-driven path and to the pass over every edge end in turn: the hubs'
    # moves reach the next evaluation only through the end bytes
    g = GRAPHS["dcsbm_2k"]()
    C = 40
    dg = sbp.DeviceGraph(g)
    cur = gen.initial_labels(g.n, C, seed=5)
    lab = sbp.labels(cur)
    bm = sbp.sbp_build_blockmodel(dg, lab, C)
    try:
        for k in range(6):
            sbp.sbp_tune("dense_update_moved_share", 1024 if k % 2 else -1)
            cur = chain_step(g, dg, lab, cur, C, bm, 13, k, n_hubs=25)
    finally:
        sbp.sbp_tune("dense_update_moved_share", 64)


@pytest.mark.parametrize("n_batches", [1, 2])
def test_sweep_hybrid_large_hubs(n_batches):
    # five hubs of 505 to 15004 edge ends, three of them beyond the ends a
    # thread of the sequential pass holds ahead, then the next-largest vertices
    g = hub_graph()
    lab0 = gen.initial_labels(g.n, 40, seed=40)
    sweep_parity(g, lab0, 40, seed=43, sweep=2, n_batches=n_batches, n_hubs=12)


def test_sweep_hybrid_edge_cases():
    # hubs without edges (the uniform proposal), one block (every proposal is
    # the own block), every vertex a hub on a mostly isolated graph
    g = gen.from_edges(50, [0, 1, 2, 3, 3], [1, 2, 3, 0, 3])  # 46 isolated, a self-loop
    for C, n_hubs in ((1, 5), (2, 50), (7, 50), (49, 50)):
        lab0 = gen.initial_labels(g.n, C, seed=C)
        sweep_parity(g, lab0, C, seed=3, sweep=C, n_hubs=n_hubs)
        sweep_parity(g, lab0, C, seed=3, sweep=C, n_batches=4, n_hubs=n_hubs)


def test_sweep_hybrid_200k():
    g = gen.sweep_200k()
    lab0 = gen.initial_labels(g.n, 45, seed=2001)
    sweep_parity(g, lab0, 45, seed=2001, sweep=0, n_hubs=16)


@pytest.mark.parametrize("n_batches", [1, 3])
@pytest.mark.parametrize("n_hubs", [1, 7, 40])
@pytest.mark.parametrize("name,C", [("plain_1k", 70), ("multi_selfloops", 150)])
def test_sweep_hybrid_hubs_sparse_tier(name, C, n_hubs, n_batches):
    # the sparse tier: every hub a batch of its own against the rebuilt blockmodel
    g = GRAPHS[name]()
    lab0 = gen.initial_labels(g.n, C, seed=C + 5)
    _, _, ref = sweep_parity(g, lab0, C, seed=33, sweep=n_hubs, n_batches=n_batches, n_hubs=n_hubs)
    assert ref["proposals"] == g.n


def test_sweep_hybrid_large_hubs_sparse_tier():
    g = hub_graph()
    lab0 = gen.initial_labels(g.n, 300, seed=41)
    sweep_parity(g, lab0, 300, seed=44, sweep=3, n_batches=2, n_hubs=6)


def test_sweep_hybrid_rejects():
    g = GRAPHS["plain_1k"]()
    dg = sbp.DeviceGraph(g)
    lab = sbp.labels(gen.initial_labels(g.n, 70, seed=1))
    before = lab.cpu().numpy().copy()
    lab10 = sbp.labels(gen.initial_labels(g.n, 10, seed=1))
    bm10 = sbp.sbp_build_blockmodel(dg, lab10, 10)
    with pytest.raises(sbp.SbpError):  # more hubs than vertices
        sbp.sbp_nodal_sweep(dg, lab10, 10, bm10, 1, 0, n_hubs=g.n + 1)
    with pytest.raises(sbp.SbpError):
        sbp.sbp_nodal_sweep(dg, lab10, 10, bm10, 1, 0, n_hubs=-1)
    assert np.array_equal(lab.cpu().numpy(), before)


# ---------------------------------------------------------------- merges
def merge_parity(g, lab0, C, seed, phase, x=10, eps=1):
    dg = sbp.DeviceGraph(g)
    lab = sbp.labels(lab0)
    bm = sbp.sbp_build_blockmodel(dg, lab, C)
    partner, dS, dSl = sbp.sbp_merge_scores(dg, lab, C, bm, seed, phase, proposals=x, eps=eps)
    rp, rdS, rdSl = O.merge_scores(g, lab0, C, seed, phase, x=x, eps=eps)
    ties = 0
    for c in np.nonzero(partner != rp)[0]:
        # only a near tie of two candidates' scores (keys 2^-20 apart) may differ
        a = O.merge_delta(g, lab0, C, c, partner[c])[1]
        b = O.merge_delta(g, lab0, C, c, rp[c])[1]
        assert abs(math.floor(a * 2**20) - math.floor(b * 2**20)) <= 1, (c, partner[c], rp[c], a, b)
        ties += 1
    same = partner == rp
    assert close(dS[same & (rp >= 0)], rdS[same & (rp >= 0)])
    assert close(dSl[same & (rp >= 0)], rdSl[same & (rp >= 0)])
    assert np.all(np.isinf(dS[rp < 0]))
    return partner, dSl, ties


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("C", [2, 20, 64, 65, 400])
def test_merge_scores(name, C):
    g = GRAPHS[name]()
    if C > g.n:
        pytest.skip("C > n")
    lab0 = gen.initial_labels(g.n, C, seed=C + 7)
    merge_parity(g, lab0, C, seed=31, phase=C)


def test_merge_scores_singletons():
    g = GRAPHS["plain_1k"]()
    merge_parity(g, np.arange(g.n, dtype=np.int32), g.n, seed=2000, phase=0)


def test_merge_scores_with_empty_blocks():
    g = GRAPHS["plain_1k"]()
    lab0 = gen.initial_labels(g.n, 50, seed=1) * 2  # odd labels empty, C = 100
    merge_parity(g, lab0.astype(np.int32), 100, seed=5, phase=1)


@pytest.mark.parametrize("C", [24000, 4000])
def test_merge_scores_long_rows(C):
    # rows and columns of M longer than the staged length (256 entries): the
    # hubs of hub_graph() at C = n hold thousands of nonzeros each
    g = hub_graph()
    lab0 = np.arange(g.n, dtype=np.int32) if C == g.n else gen.initial_labels(g.n, C, seed=9)
    M = O.build_blockmodel(g, lab0, C)
    assert np.bincount(M["rows"], minlength=C).max() > 256
    _, _, ties = merge_parity(g, lab0, C, seed=71, phase=2)
    print(f"merge near ties: {ties}")


@pytest.mark.parametrize("seed", range(6))
def test_merge_apply_random(seed):
    rng = np.random.default_rng(seed)
    C = int(rng.integers(2, 3000))
    partner = rng.integers(-1, C, C).astype(np.int32)
    partner[partner == np.arange(C)] = -1
    dSl = np.round(rng.normal(size=C) * 4, 1)  # many exact ties
    dSl[partner < 0] = np.inf
    for m in (0, 1, C // 3, C // 2, C):
        got = sbp.sbp_merge_apply(partner, dSl, m)
        ref = O.merge_apply(partner, dSl, m)
        assert got[0] == ref[0]
        assert np.array_equal(got[1], ref[1])


def test_merge_apply_cycles_and_chains():
    C = 12
    partner = np.array([1, 2, 0, 4, 5, 3, 7, 6, -1, 8, 9, 10], np.int32)
    dSl = np.array([.3, .1, .2, .5, .4, .6, .7, .7, np.inf, .2, .2, .2])
    for m in range(C + 1):
        got = sbp.sbp_merge_apply(partner, dSl, m)
        ref = O.merge_apply(partner, dSl, m)
        assert got[0] == ref[0] and np.array_equal(got[1], ref[1]), m


def test_compact():
    rng = np.random.default_rng(3)
    for C in (1, 5, 300, 5000):
        lab0 = rng.integers(0, C, 4000).astype(np.int32)
        lab = sbp.labels(lab0)
        k = sbp.sbp_compact(lab, C)
        rk, rlab = O.compact(lab0, C)
        assert k == rk and np.array_equal(lab.cpu().numpy(), rlab)


# ---------------------------------------------------------------- whole method
def partition_parity(g, **kw):
    dg = sbp.DeviceGraph(g)
    res = sbp.sbp_partition(dg, **kw)
    ora = O.partition(g, **kw)
    assert np.array_equal(res["trace"], ora["trace"]), (res["trace"], ora["trace"])
    assert close(res["trace_dl"], ora["trace_dl"])
    assert res["C"] == ora["C"]
    assert np.array_equal(res["lab"], ora["lab"])
    assert close([res["dl"]], [ora["dl"]])
    return res


def test_partition_tiny_two_cliques():
    src, dst = [], []
    for blk in (range(0, 4), range(4, 8)):
        for u in blk:
            for w in blk:
                if u != w:
                    src += [u] * 3
                    dst += [w] * 3
    g = gen.from_edges(8, src + [0, 5], dst + [5, 0])
    res = partition_parity(g, seed=7)
    assert res["C"] == 2


def test_partition_single_vertex_and_edgeless():
    partition_parity(gen.from_edges(1, [], []), seed=1)
    partition_parity(gen.from_edges(6, [], []), seed=1)


def test_partition_1k():
    res = partition_parity(gen.plain_1k(), seed=2000)
    assert 5 <= res["C"] <= 20


def test_partition_easy_planted():
    g = gen.dcsbm([100] * 6, 12000, 5.0, seed=31, kmin=10, kmax=100)
    partition_parity(g, seed=12)


def test_partition_batches_per_sweep():
    partition_parity(gen.plain_1k(seed=55), seed=3, n_batches=1)
    partition_parity(gen.plain_1k(seed=56), seed=3, n_batches=7)


@pytest.mark.parametrize("n_hubs", [1, 6, 40])
def test_partition_hybrid_hubs(n_hubs):
    # Hybrid SBP in the whole method: every sweep moves the n_hubs
    # highest-degree vertices one at a time first, on both tiers as C falls
    partition_parity(gen.plain_1k(seed=57), seed=5, n_hubs=n_hubs)


def test_partition_hybrid_every_vertex_a_hub():
    g = gen.dcsbm([25] * 4, 600, 4.0, seed=58, kmax=20)
    partition_parity(g, seed=6, n_hubs=g.n + 5, n_batches=1)


def test_batch_hybrid_equals_alone():
    graphs = [gen.batch_graph(n, seed=3400 + i) for i, n in enumerate([600, 1300, 900])]
    dgs = [sbp.DeviceGraph(g) for g in graphs]
    kw = [dict(seed=70 + i, n_hubs=h) for i, h in enumerate([0, 8, 3])]
    batch = sbp.sbp_partition_batch(dgs, kw)
    for i, dg in enumerate(dgs):
        alone = sbp.sbp_partition(dg, **kw[i])
        assert batch[i]["C"] == alone["C"] and batch[i]["dl"] == alone["dl"]
        assert np.array_equal(batch[i]["lab"], alone["lab"])
    ora = O.partition(graphs[1], **kw[1])
    assert batch[1]["C"] == ora["C"] and np.array_equal(batch[1]["lab"], ora["lab"])


def test_partition_from_given_assignment():
    g = gen.plain_1k()
    lab0 = gen.initial_labels(g.n, 80, seed=1)
    dg = sbp.DeviceGraph(g)
    res = sbp.sbp_partition(dg, assign_in=sbp.labels(lab0), C_in=80, seed=4)
    ora = O.partition(g, lab_in=lab0, C_in=80, seed=4)
    assert res["C"] == ora["C"] and np.array_equal(res["lab"], ora["lab"])


def test_partition_mid_size():
    # the whole method on a 20k-vertex graph shaped like the batched workload
    g = gen.batch_graph(20000, seed=3999)
    res = partition_parity(g, seed=4111)
    assert res["C"] > 10


def test_partition_keeps_empty_labels_until_the_end():
    # results are stored at the count their merge phase produced; the stored
    # count column of the trace equals the merged count, and the returned
    # assignment is compact with its DL at the non-empty count
    g = gen.plain_1k(seed=77)
    res = partition_parity(g, seed=19)
    assert np.array_equal(res["trace"][:, 2], res["trace"][:, 4])
    assert set(res["lab"].tolist()) == set(range(res["C"]))


# ---------------------------------------------------------------- batched and continuous
def test_batch_equals_alone():
    graphs = [gen.batch_graph(n, seed=3000 + i) for i, n in enumerate([500, 1200, 800, 2500, 650])]
    dgs = [sbp.DeviceGraph(g) for g in graphs]
    kw = [dict(seed=4000 + i) for i in range(len(graphs))]
    batch = sbp.sbp_partition_batch(dgs, kw)
    for i, dg in enumerate(dgs):
        alone = sbp.sbp_partition(dg, **kw[i])
        assert batch[i]["C"] == alone["C"]
        assert np.array_equal(batch[i]["lab"], alone["lab"])
        assert batch[i]["dl"] == alone["dl"]  # same arithmetic in the same order
        assert np.array_equal(batch[i]["trace"], alone["trace"])


@pytest.mark.parametrize("n_batches", [1, 3])
def test_engine_dense_sweeps_equal_sparse_sweeps(n_batches):
    # sweeps at C <= 64 run on the multi-graph dense kernels inside the engine;
    # switching them off (every sweep on the sparse kernels) changes nothing
    sizes = [500, 3000, 900, 12000, 1500, 700]
    graphs = [gen.batch_graph(n, seed=3300 + i) for i, n in enumerate(sizes)]
    dgs = [sbp.DeviceGraph(g) for g in graphs]
    kw = [dict(seed=600 + i, n_batches=n_batches) for i in range(len(graphs))]
    try:
        dense = sbp.sbp_partition_batch(dgs, kw)
        sbp.sbp_tune("engine_dense_max_c", 0)
        sparse = sbp.sbp_partition_batch(dgs, kw)
    finally:
        sbp.sbp_tune("engine_dense_max_c", 64)
    for a, b in zip(dense, sparse):
        assert a["C"] == b["C"] and a["dl"] == b["dl"]
        assert np.array_equal(a["lab"], b["lab"])
        assert np.array_equal(a["trace"], b["trace"])


@pytest.mark.parametrize("kw", [dict(n_batches=3), dict(n_batches=2, n_hubs=6), dict(n_batches=1, n_hubs=3)])
def test_batches_in_step_change_nothing(kw):
    # the later hubs and batches of a sweep run inside the engine step that
    # began it (rebuilt blockmodel, no host round trip); one a step gives the
    # same partitions, bit for bit
    sizes = [400, 2500, 900, 6000]
    graphs = [gen.batch_graph(n, seed=3700 + i) for i, n in enumerate(sizes)]
    dgs = [sbp.DeviceGraph(g) for g in graphs]
    kws = [dict(seed=710 + i, **kw) for i in range(len(graphs))]
    out = []
    try:
        for mode in (1, 0):
            sbp.sbp_tune("batches_in_step", mode)
            out.append(sbp.sbp_partition_batch(dgs, kws))
    finally:
        sbp.sbp_tune("batches_in_step", 1)
    for a, b in zip(*out):
        assert a["C"] == b["C"] and a["dl"] == b["dl"]
        assert np.array_equal(a["lab"], b["lab"])
        assert np.array_equal(a["trace"], b["trace"])


@pytest.mark.parametrize("C,n_batches,n_hubs", [(7, 1, 0), (45, 1, 6), (45, 3, 0), (150, 1, 0), (150, 2, 4)])
def test_sweep_stats_near_ties_and_totals(C, n_batches, n_hubs):
    # the sweep totals agree with the sweep's own trace on both tiers: near
    # ties are the proposals (not no-ops) with |margin| < 1e-9, accepted and
    # no-op counts follow the per-vertex records
    g = GRAPHS["dcsbm_2k"]()
    dg = sbp.DeviceGraph(g)
    lab = sbp.labels(gen.initial_labels(g.n, C, seed=C))
    bm = sbp.sbp_build_blockmodel(dg, lab, C)
    for k in range(6):
        tr = sbp.sbp_nodal_sweep(dg, lab, C, bm, 33, k, n_batches=n_batches, n_hubs=n_hubs)
        act = tr["margin"] != 0.0  # no-ops record a zero margin
        assert tr["accepted"] == int(tr["accept"].sum())
        assert tr["near_ties"] == int((act & (np.abs(tr["margin"]) < 1e-9)).sum())
        assert tr["proposals"] == g.n


def test_lookup_tables_change_nothing():
    # sparse-tier sweeps read M from a C x C table when C <= 2048; with the
    # tables switched off (binary searches of the rows) every result is equal
    g = GRAPHS["multi_selfloops"]()
    dg = sbp.DeviceGraph(g)
    for C in (70, 150, 299):
        lab0 = gen.initial_labels(g.n, C, seed=C)
        out = []
        for tmax in (2048, 0):
            sbp.sbp_tune("table_max_c", tmax)
            lab = sbp.labels(lab0)
            bm = sbp.sbp_build_blockmodel(dg, lab, C)
            tr = sbp.sbp_nodal_sweep(dg, lab, C, bm, 7, C, n_batches=2)
            out.append((lab.cpu().numpy(), tr))
        sbp.sbp_tune("table_max_c", 2048)
        (la, ta), (lb, tb) = out
        assert np.array_equal(la, lb) and np.array_equal(ta["prop"], tb["prop"])
        assert np.array_equal(ta["accept"], tb["accept"]) and np.array_equal(ta["dS"], tb["dS"])
    graphs = [gen.batch_graph(n, seed=3500 + i) for i, n in enumerate([800, 4000, 1500])]
    dgs = [sbp.DeviceGraph(x) for x in graphs]
    kw = [dict(seed=90 + i) for i in range(len(graphs))]
    try:
        sbp.sbp_tune("table_build", 2)
        a = sbp.sbp_partition_batch(dgs, kw)  # M counted into the tables whenever every count fits
        sbp.sbp_tune("table_build", 0)
        b = sbp.sbp_partition_batch(dgs, kw)  # tables as lookups only, the sort-based build
        sbp.sbp_tune("table_max_c", 0)
        c = sbp.sbp_partition_batch(dgs, kw)  # no tables
    finally:
        sbp.sbp_tune("table_max_c", 2048)
        sbp.sbp_tune("table_build", 1)
    for x, y, z in zip(a, b, c):
        assert x["C"] == y["C"] == z["C"] and x["dl"] == y["dl"] == z["dl"]
        assert np.array_equal(x["lab"], y["lab"]) and np.array_equal(x["lab"], z["lab"])
        assert np.array_equal(x["trace_dl"], z["trace_dl"])


def test_batch_matches_oracle():
    graphs = [gen.batch_graph(n, seed=3100 + i) for i, n in enumerate([500, 700])]
    res = sbp.sbp_partition_batch([sbp.DeviceGraph(g) for g in graphs], [dict(seed=7), dict(seed=8)])
    for i, g in enumerate(graphs):
        ora = O.partition(g, seed=7 + i)
        assert res[i]["C"] == ora["C"] and np.array_equal(res[i]["lab"], ora["lab"])


def test_engine_continuous_admission():
    graphs = [gen.batch_graph(n, seed=3200 + i) for i, n in enumerate([600, 900, 500, 1500])]
    dgs = [sbp.DeviceGraph(g) for g in graphs]
    alone = [sbp.sbp_partition(dg, seed=50 + i) for i, dg in enumerate(dgs)]
    V = sum(g.n for g in graphs[:2]) + 100
    E = sum(g.e for g in graphs[:2]) + 100
    eng = sbp.Engine(V, E, 3)
    pending = list(range(len(graphs)))
    results = {}
    steps = 0
    while pending or len(results) < len(graphs):
        while pending and eng.admit(dgs[pending[0]], pending[0], seed=50 + pending[0]):
            pending.pop(0)
        eng.step()
        steps += 1
        for tag, C, dl, out, _ in eng.poll():
            results[tag] = (C, dl, out.cpu().numpy())
        assert steps < 100000
    eng.close()
    for i in range(len(graphs)):
        C, dl, lab = results[i]
        assert C == alone[i]["C"] and dl == alone[i]["dl"] and np.array_equal(lab, alone[i]["lab"])


def test_profile_sampling_stride():
    # events on every k-th evaluation launch from the enabling call on
    g = GRAPHS["plain_1k"]()
    dg = sbp.DeviceGraph(g)
    lab = sbp.labels(gen.initial_labels(g.n, 10, seed=1))
    bm = sbp.sbp_build_blockmodel(dg, lab, 10)
    sbp.sbp_profile_read("sweep_eval", reset=True)
    try:
        for stride, want in ((3, 4), (1, 10), (11, 1)):
            sbp.sbp_profile_enable(True, stride=stride)
            for k in range(10):
                sbp.sbp_nodal_sweep(dg, lab, 10, bm, 5, k, trace=False, stats=False)
            ms, n = sbp.sbp_profile_read("sweep_eval", reset=True)
            assert n == want and ms > 0.0
        sbp.sbp_profile_enable(False)
        sbp.sbp_nodal_sweep(dg, lab, 10, bm, 5, 10, trace=False, stats=False)
        assert sbp.sbp_profile_read("sweep_eval", reset=True) == (0.0, 0)
        with pytest.raises(sbp.SbpError):
            sbp.sbp_profile_enable(True, stride=-2)
    finally:
        sbp.sbp_profile_enable(False)


def test_server_staggered_arrivals_and_oversized_request():
    from paper_2305_18663_amd import serve
    graphs = [gen.batch_graph(n, seed=3300 + i) for i, n in enumerate([700, 1500, 500, 900, 1200])]
    big = gen.batch_graph(6000, seed=3399)  # more vertices than the engine holds
    alone = [sbp.sbp_partition(sbp.DeviceGraph(g), seed=60 + i) for i, g in enumerate(graphs)]
    V = 2600
    E = 8 * V
    srv = serve.PartitionServer(8 << 30, V, E, 3)
    reqs = [serve.Request(i, g, 0.02 * i, dict(seed=60 + i)) for i, g in enumerate(graphs)]
    reqs.insert(2, serve.Request(99, big, 0.01, dict(seed=1)))
    srv.run(reqs)
    srv.close()
    by = {r.tag: r for r in reqs}
    assert by[99].error is not None and by[99].labels is None
    for i in range(len(graphs)):
        r = by[i]
        assert r.error is None
        assert r.C == alone[i]["C"] and r.dl == alone[i]["dl"] and np.array_equal(r.labels, alone[i]["lab"])
        assert np.array_equal(r.trace, alone[i]["trace"])
    s = serve.latency_summary(reqs)
    assert s["rejected"] == 1 and s["graphs_per_s"] > 0
