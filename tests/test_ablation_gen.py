"""The paper's parameter-search graph families (Sec. IV-A) and the study's metrics.

Generator properties fixed by the family definitions: degree ranges, the
duplicated vs split degree sequences, edge counts, removal of vertices without
edges.  DL^null (Sec. V) is pinned to the oracle's description length of the
one-community assignment.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_18663_amd import ablation, gen


def test_sixteen_families_cover_every_combination():
    keys = {(t[0], t[1], t[2], t[3]) for t in gen.ABLATION.values()}
    assert len(gen.ABLATION) == 16 and len(keys) == 16
    for name, (tmin, tmax, dup, nb, _) in gen.ABLATION.items():
        assert name == "".join("T" if x else "F" for x in (tmin, tmax, dup)) + str(nb)
    assert set(ablation.PAPER_NMI_1NODE) == set(gen.ABLATION)


@pytest.mark.parametrize("tmin", [True, False])
@pytest.mark.parametrize("tmax", [True, False])
def test_degree_sequences(tmin, tmax):
    kmin, kmax = gen.ablation_bounds(tmin, tmax)
    assert (kmin, kmax) == ((10 if tmin else 1), (100 if tmax else gen.ABLATION_N // 20))
    kmin, kmax = gen.ablation_bounds(tmin, tmax, 50000)  # the max scales with n
    rng = np.random.default_rng(1)
    ko, ki = gen.ablation_degrees(rng, 50000, tmin, tmax, dup=True)
    assert np.array_equal(ko, ki)  # one sequence for both directions
    assert ko.min() >= kmin and ko.max() <= kmax and ko.min() == kmin
    rng = np.random.default_rng(1)
    ko2, ki2 = gen.ablation_degrees(rng, 50000, tmin, tmax, dup=False)
    tot = ko2 + ki2
    assert np.array_equal(tot, ko)  # the same total sequence, split
    assert np.all(ko2 >= 0) and np.all(ki2 >= 0) and np.all(ko2 == np.round(ko2))
    if not tmin:
        assert np.any(tot == 1)  # total degree 1 exists only without duplication
    # the split is fair: out share near one half
    assert abs(ko2.sum() / tot.sum() - 0.5) < 0.01


@pytest.mark.parametrize("name", ["TTT33", "TFF150", "FTF33", "FFT150"])
def test_family_graph(name):
    tmin, tmax, dup, nb, e = gen.ABLATION[name]
    g = gen.ablation_graph(name, seed=4000, scale=0.1)
    assert g.e == round(e * 0.1)
    kout, kin = g.degrees()
    assert np.all(kout + kin > 0)  # vertices without edges removed
    assert g.n <= round(gen.ABLATION_N * 0.1)
    if tmin:
        assert g.n == round(gen.ABLATION_N * 0.1)  # none lost
    assert g.n_planted == nb and g.planted.min() >= 0 and g.planted.max() < nb
    assert len(np.unique(g.planted)) > 0.9 * nb
    src, dst = g.edges()
    assert np.all(src != dst)  # the generator redraws self-loops
    # within:between ratio 2 (a third of the edges cross communities)
    cross = np.mean(g.planted[src] != g.planted[dst])
    assert abs(cross - 1 / 3) < 0.02
    # deterministic per seed
    g2 = gen.ablation_graph(name, seed=4000, scale=0.1)
    assert np.array_equal(g.out_idx, g2.out_idx) and np.array_equal(g.planted, g2.planted)


def test_full_size_edge_counts():
    for name in ("TTT33", "FFF150"):
        g = gen.ablation_graph(name)
        assert g.e == gen.ABLATION[name][4]


def test_dl_null_is_the_one_community_dl():
    for name in ("TTF33", "FFT33"):
        g = gen.ablation_graph(name, seed=7, scale=0.05)
        ref = O.description_length(g, np.zeros(g.n, np.int32), 1)
        assert ablation.dl_null(g.e) == pytest.approx(ref, rel=1e-12)
        # planted labels describe the graph better than one community
        assert O.description_length(g, g.planted, g.n_planted) < ref


def test_nmi_and_summary():
    a = np.array([0, 0, 1, 1, 2, 2])
    assert ablation.nmi(a, (a + 1) % 3) == pytest.approx(1.0)
    assert ablation.nmi(a, np.zeros(6, int)) == pytest.approx(0.0)
    # closed form: two blocks split evenly by the other labelling -> I = 0
    assert ablation.nmi([0, 0, 1, 1], [0, 1, 0, 1]) == pytest.approx(0.0, abs=1e-12)
    # by hand from the joint distribution of two labellings
    x = [0, 0, 0, 1, 1, 1]
    y = [0, 0, 1, 1, 1, 1]
    px = np.array([0.5, 0.5]); py = np.array([1 / 3, 2 / 3])
    pxy = np.array([[2 / 6, 1 / 6], [0, 3 / 6]])
    I = sum(pxy[i, j] * math.log(pxy[i, j] / (px[i] * py[j])) for i in range(2) for j in range(2) if pxy[i, j] > 0)
    H = lambda p: -sum(q * math.log(q) for q in p if q > 0)
    assert ablation.nmi(x, y) == pytest.approx(2 * I / (H(px) + H(py)), rel=1e-12)
    rows = [dict(family="A", seed=s, n=10, e=20, C=3, nmi=0.5 + 0.1 * s, dl_norm=0.9, paper_nmi_1node=0.4)
            for s in range(3)]
    s = ablation.summarize(rows)
    assert len(s) == 1 and s[0]["nmi"] == pytest.approx(0.6) and s[0]["nmi_min"] == pytest.approx(0.5)
    assert "| A |" in ablation.markdown(s)


def test_generator_blocks_with_one_or_no_in_weight():
    # block 0 = {0, 1}: only vertex 0 has in-weight, so a within-block edge
    # from 0 could only self-loop; block 2 = {5, 6} has no in-weight at all.
    # Such edges take another block; no edge enters a vertex without in-weight.
    rng = np.random.default_rng(3)
    sizes = np.array([2, 3, 2])
    th_out = np.ones(7)
    th_in = np.array([2.0, 0, 1, 1, 1, 0, 0])
    g = gen._dcsbm_draw(rng, sizes, th_out, th_in, 4000, 3.0)
    src, dst = g.edges()
    assert g.e == 4000 and np.all(src != dst)
    kout, kin = g.degrees()
    # the three vertices without in-weight (one in block 0, both of block 2)
    blk0 = np.flatnonzero(g.planted == 0)
    blk2 = np.flatnonzero(g.planted == 2)
    assert np.all(kin[blk2] == 0)
    assert sorted(kin[blk0].tolist())[0] == 0
    with pytest.raises(ValueError):
        gen._dcsbm_draw(np.random.default_rng(1), np.array([1]), np.ones(1), np.ones(1), 5, 1.0)
