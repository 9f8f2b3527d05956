"""The accuracy study's GPU path on two parameter-search families, one tenth size.

The batched partitions must equal the oracle's partitions of the same graphs
label for label (the whole method, Alg. 1 and Alg. 2 with the golden search),
and the study's metrics must follow: a truncated-degree family recovered,
the untruncated split-degree family far below it.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2305_18663_amd import ablation, gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def test_study_matches_oracle_partitions():
    names = ["TTT33", "FFF33"]
    rows, _ = ablation.run(names, seeds=(0,), scale=0.1, keep_labels=True)
    fam = list(gen.ABLATION)
    for r in rows:
        g = gen.ablation_graph(r["family"], seed=4000 + fam.index(r["family"]), scale=0.1)
        ref = O.partition(g, seed=2000)
        assert np.array_equal(r["lab"], ref["lab"]), f"{r['family']}: labels differ"
        assert r["C"] == ref["C"] and r["n"] == g.n and r["e"] == g.e
        assert r["dl"] == pytest.approx(ref["dl"], rel=1e-12)
        assert r["nmi"] == pytest.approx(ablation.nmi(ref["lab"], g.planted), abs=1e-12)
        assert r["dl_norm"] == pytest.approx(ref["dl"] / ablation.dl_null(g.e), rel=1e-12)
    by = {r["family"]: r for r in rows}
    assert by["TTT33"]["nmi"] > 0.9 and by["TTT33"]["dl_norm"] < 1.0
    assert by["FFF33"]["nmi"] < by["TTT33"]["nmi"] - 0.3
