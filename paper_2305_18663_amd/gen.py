"""Seeded synthetic inputs: directed degree-corrected SBM graphs and start labels.

This module holds no part of the partitioning method's arithmetic.  It only
draws graphs and label vectors, so that the HIP path and the CPU oracle can be
fed identical inputs.

Generator (degree-corrected SBM of Karrer and Newman, the model the paper's
Sec. II-A builds on; the paper's synthetic graphs are DCSBM draws with
within:between ratio near 2 and Dirichlet block sizes, Sec. IV-A):

1. Block sizes are given per workload.
2. Each vertex draws out- and in-weights theta_out, theta_in i.i.d. from a
   discrete power law P(k) ~ k^-gamma on [k_min, k_max].
3. The edge count E is fixed.  Each edge picks its source proportional to
   theta_out; its target block is the source's block with probability
   ratio/(1+ratio), otherwise another block proportional to that block's total
   theta_in; its target vertex is proportional to theta_in inside the block.
   Self-loops are redrawn; an edge whose target block holds no in-weight
   besides its source's takes another block, drawn as a between-block
   target.  Multi-edges are kept.
4. Vertex ids are randomly permuted so planted blocks are not contiguous.

Graphs are returned as int32 CSR (out-edges) and CSC (in-edges), neighbours
ascending, multiplicity kept.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Graph:
    n: int
    e: int
    out_ptr: np.ndarray  # int32 [n+1]
    out_idx: np.ndarray  # int32 [e], ascending within each row
    in_ptr: np.ndarray   # int32 [n+1]
    in_idx: np.ndarray   # int32 [e], ascending within each column
    planted: np.ndarray | None = None  # int32 [n] planted block of each vertex
    n_planted: int = 0

    def degrees(self):
        kout = np.diff(self.out_ptr).astype(np.int64)
        kin = np.diff(self.in_ptr).astype(np.int64)
        return kout, kin

    def edges(self):
        """(src, dst) int64 arrays in CSR order."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.out_ptr))
        return src, self.out_idx.astype(np.int64)

    def nbytes(self) -> int:
        return 4 * (2 * (self.n + 1) + 2 * self.e)


def from_edges(n: int, src, dst, planted=None, n_planted: int = 0) -> Graph:
    """Canonical CSR/CSC (neighbours ascending, multiplicity kept) from an edge list."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if src.shape != dst.shape:
        raise ValueError("src and dst differ in length")
    if src.size and (src.min() < 0 or dst.min() < 0 or src.max() >= n or dst.max() >= n):
        raise ValueError("edge endpoint out of range")
    e = int(src.size)
    if e >= 2**31:
        raise ValueError("edge count exceeds int32")
    order = np.argsort(src * n + dst, kind="stable")
    out_idx = dst[order].astype(np.int32)
    out_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=out_ptr[1:])
    order = np.argsort(dst * n + src, kind="stable")
    in_idx = src[order].astype(np.int32)
    in_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(dst, minlength=n), out=in_ptr[1:])
    return Graph(n, e, out_ptr.astype(np.int32), out_idx, in_ptr.astype(np.int32), in_idx,
                 None if planted is None else np.asarray(planted, dtype=np.int32), n_planted)


def _power_law(rng, size, gamma, kmin, kmax):
    ks = np.arange(kmin, kmax + 1, dtype=np.float64)
    p = ks ** (-gamma)
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    return ks[np.searchsorted(cdf, rng.random(size), side="right").clip(0, ks.size - 1)]


def _draw_prop(rng, cum, size):
    """Indices drawn proportional to weights whose cumulative sum is `cum`."""
    return np.searchsorted(cum, rng.random(size) * cum[-1], side="right").clip(0, cum.size - 1)


def dcsbm(sizes, e, ratio, seed, gamma=2.1, kmin=1, kmax=100) -> Graph:
    """Directed DCSBM draw with fixed edge count (see module docstring)."""
    rng = np.random.default_rng(seed)
    sizes = np.asarray(sizes, dtype=np.int64)
    n = int(sizes.sum())
    th_out = _power_law(rng, n, gamma, kmin, kmax)
    th_in = _power_law(rng, n, gamma, kmin, kmax)
    return _dcsbm_draw(rng, sizes, th_out, th_in, e, ratio)


def _dcsbm_draw(rng, sizes, th_out, th_in, e, ratio) -> Graph:
    """Steps 3 and 4 of the module docstring for given vertex weights."""
    n = int(sizes.sum())
    nb = sizes.size
    block = np.repeat(np.arange(nb, dtype=np.int64), sizes)  # contiguous before permutation
    p_in = ratio / (1.0 + ratio)

    src = _draw_prop(rng, np.cumsum(th_out), e)
    sb = block[src]
    tb = sb.copy()
    between = rng.random(e) >= p_in
    wblk = np.bincount(block, weights=th_in, minlength=nb)
    cumb = np.cumsum(wblk)
    pos_in = np.bincount(block[th_in > 0], minlength=nb)  # vertices with in-weight, per block
    if nb > 1:
        idx = np.nonzero(between)[0]
        while idx.size:
            draw = _draw_prop(rng, cumb, idx.size)
            ok = draw != sb[idx]
            tb[idx[ok]] = draw[ok]
            idx = idx[~ok]
    idx = np.nonzero(wblk[tb] <= 0)[0]  # a block without in-weight takes no edges
    if idx.size and nb == 1:
        raise ValueError("no vertex has in-weight")
    while idx.size:
        draw = _draw_prop(rng, cumb, idx.size)
        ok = draw != sb[idx]
        tb[idx[ok]] = draw[ok]
        idx = idx[~ok]
    # target vertex proportional to theta_in within the target block
    cum_in = np.cumsum(th_in)
    bstart = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    lo = np.where(bstart > 0, cum_in[np.maximum(bstart - 1, 0)], 0.0)
    hi = cum_in[bstart + sizes - 1]
    dst = np.empty(e, dtype=np.int64)
    pending = np.arange(e)
    while pending.size:
        b_ = tb[pending]
        u = lo[b_] + rng.random(pending.size) * (hi[b_] - lo[b_])
        d = np.searchsorted(cum_in, u, side="right").clip(bstart[b_], bstart[b_] + sizes[b_] - 1)
        dst[pending] = d
        pending = pending[d == src[pending]]  # redraw self-loops
        if pending.size:
            # a target block with no in-weight besides the source's can only
            # give a self-loop: such an edge takes another block instead
            sp = src[pending]
            stuck = pos_in[tb[pending]] - (th_in[sp] > 0) <= 0
            if stuck.any():
                if nb == 1:
                    raise ValueError("one block with one target: every edge would be a self-loop")
                idx = pending[stuck]
                while idx.size:
                    draw = _draw_prop(rng, cumb, idx.size)
                    ok = draw != sb[idx]
                    tb[idx[ok]] = draw[ok]
                    idx = idx[~ok]
    perm = rng.permutation(n)
    planted = np.empty(n, dtype=np.int32)
    planted[perm] = block
    return from_edges(n, perm[src], perm[dst], planted, nb)


# --------------------------------------------------------------------------
# Workload recipes (sizes and seeds of the paper-shaped synthetic inputs)
# --------------------------------------------------------------------------

# The paper's exhaustive parameter-search families (Sec. IV-A, table of
# synthetic graphs): truncated min degree, truncated max degree, duplicated
# degree sequence, communities, edges.  Every family starts from 22,599
# vertices; vertices left without edges are dropped, as the table's smaller
# vertex counts for the untruncated-min families show.
ABLATION = {
    "TTT33": (True, True, True, 33, 899283), "TTT150": (True, True, True, 150, 826861),
    "TTF33": (True, True, False, 33, 452232), "TTF150": (True, True, False, 150, 421317),
    "TFT33": (True, False, True, 33, 1059970), "TFT150": (True, False, True, 150, 912644),
    "TFF33": (True, False, False, 33, 540410), "TFF150": (True, False, False, 150, 471071),
    "FTT33": (False, True, True, 33, 79683), "FTT150": (False, True, True, 150, 78226),
    "FTF33": (False, True, False, 33, 39719), "FTF150": (False, True, False, 150, 38408),
    "FFT33": (False, False, True, 33, 83939), "FFT150": (False, False, True, 150, 81298),
    "FFF33": (False, False, False, 33, 41378), "FFF150": (False, False, False, 150, 40835),
}
ABLATION_N = 22599
ABLATION_RATIO = 2.0


def ablation_bounds(tmin: bool, tmax: bool, n: int = ABLATION_N):
    """Degree range of a family: [10, 100] truncated; min 1 and max n/20 when not."""
    return (10 if tmin else 1), (100 if tmax else max(100, n // 20))


def ablation_degrees(rng, n, tmin, tmax, dup, gamma=2.1):
    """Out- and in-degree sequences of one family.

    A total-degree sequence k is drawn from PL(gamma) on the family's range.
    Duplicated: k serves as both the out- and the in-degree sequence (so every
    vertex has in-degree = out-degree >= the minimum).  Split: each unit of k
    goes to the out- or the in-degree at random (Binomial(k, 1/2)), so a vertex
    may have total degree 1.
    """
    kmin, kmax = ablation_bounds(tmin, tmax, n)
    k = _power_law(rng, n, gamma, kmin, kmax)
    if dup:
        return k.copy(), k.copy()
    kout = rng.binomial(k.astype(np.int64), 0.5).astype(np.float64)
    return kout, k - kout


def ablation_graph(name: str, seed: int = 4000, scale: float = 1.0) -> Graph:
    """One draw of an ablation family, vertices and edges scaled by `scale`.

    Block sizes are Dirichlet(2) over the family's community count; vertex
    weights come from ablation_degrees; edges as in the module docstring with
    within:between ratio 2 and the family's edge count; vertices without
    edges are then removed (ids renumbered in order, planted labels kept).
    """
    tmin, tmax, dup, nb, e = ABLATION[name]
    rng = np.random.default_rng(seed)
    n = max(nb, int(round(ABLATION_N * scale)))
    w = rng.dirichlet(np.full(nb, 2.0))
    sizes = np.maximum(2, np.floor(w * n)).astype(np.int64)
    sizes[np.argmax(sizes)] += n - sizes.sum()
    th_out, th_in = ablation_degrees(rng, n, tmin, tmax, dup)
    g = _dcsbm_draw(rng, sizes, th_out, th_in, int(round(e * scale)), ABLATION_RATIO)
    kout, kin = g.degrees()
    keep = (kout + kin) > 0
    if keep.all():
        return g
    new_id = np.cumsum(keep) - 1
    src, dst = g.edges()
    return from_edges(int(keep.sum()), new_id[src], new_id[dst], g.planted[keep], nb)


def plain_1k(seed: int = 1000) -> Graph:
    """1,000 vertices, 10 equal planted blocks, 8,000 edges, ratio 2.5, PL(2.1,[1,100])."""
    return dcsbm([100] * 10, 8000, 2.5, seed)


def sweep_200k_sizes(n=200_000, nb=45, spread=5.0):
    w = spread ** (np.arange(nb) / (nb - 1))
    s = np.floor(w / w.sum() * n).astype(np.int64)
    s[np.argsort(-(w / w.sum() * n - s))[: n - s.sum()]] += 1
    return s


def sweep_200k(seed: int = 1001, n: int = 200_000, e: int = 4_000_000) -> Graph:
    """200,000 vertices, 45 blocks with sizes spread 5x, 4M edges, ratio 2.5."""
    return dcsbm(sweep_200k_sizes(n), e, 2.5, seed)


def sparse_1m(seed: int = 1002, n: int = 1_000_000, e: int = 8_000_000, nb: int = 180,
              max_degree: int = 10_000) -> Graph:
    """1M vertices, mean out-degree 8, 180 Dirichlet(2) blocks, ratio 1.5, hub tail."""
    rng = np.random.default_rng(seed + 7)
    w = rng.dirichlet(np.full(nb, 2.0))
    sizes = np.maximum(1, np.floor(w * n)).astype(np.int64)
    sizes[np.argmax(sizes)] += n - sizes.sum()
    # realised degree ~ theta * e / sum(theta); mean theta of PL(2.1) on [1,kmax] ~ 3.3
    kmax = int(max(100, max_degree / 2 / (e / n / 3.3)))
    return dcsbm(sizes, e, 1.5, seed, kmax=kmax)


def batch_sizes(count=256, seed=3000, median=5000, lo=500, hi=50_000):
    rng = np.random.default_rng(seed)
    sigma = math.log(hi / median) / 3.0
    return np.clip(np.round(rng.lognormal(math.log(median), sigma, count)), lo, hi).astype(np.int64)


def batch_graph(n: int, seed: int) -> Graph:
    """Uneven-batch member: ~sqrt(N) equal blocks, E = 8N, ratio 2.5."""
    nb = max(1, int(round(math.sqrt(n))))
    sizes = np.full(nb, n // nb, dtype=np.int64)
    sizes[: n - sizes.sum()] += 1
    return dcsbm(sizes, 8 * n, 2.5, seed)


def request_sizes(count=2000, seed=5001, median=14142, lo=1000, hi=200_000):
    return batch_sizes(count, seed, median, lo, hi)


def initial_labels(n: int, c: int, seed: int = 2001) -> np.ndarray:
    """Uniform random start labels in [0, c)."""
    return np.random.default_rng(seed).integers(0, c, n, dtype=np.int64).astype(np.int32)


def random_multigraph(n: int, e: int, seed: int, self_loops: bool = True) -> Graph:
    """Unstructured small multigraph (optionally with self-loops) for edge cases."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, e)
    dst = rng.integers(0, n, e)
    if not self_loops:
        bad = src == dst
        while bad.any():
            dst[bad] = rng.integers(0, n, bad.sum())
            bad = src == dst
    return from_edges(n, src, dst)
