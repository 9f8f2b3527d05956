"""Launch-shape autotuner for the dense sweep, cached per size bin in JSON.

The dense sweep's launch shapes (the evaluation grid, the update grid and
the share of moved vertices below which the block matrix is updated from the
moved vertices alone) change its speed, never its results.  For a graph the
tuner times one short chain of sweeps under each candidate shape, starting
every candidate from the same assignment, checks that every candidate ends
in the same assignment (bit for bit), and stores the fastest shape under the
graph's size bin: (log2 of the vertex count, log2 of the edge-end count,
block-count bin, batch count).  `apply()` looks a graph's bin up and sets
the knobs through `sbp_tune`; a bin without an entry keeps the defaults.

Usage:
    python -m paper_2305_18663_amd.autotune --out tune.json     # tune the standard workloads
and in code:
    autotune.apply("tune.json", n, e, C, n_batches)
"""
from __future__ import annotations

import argparse
import itertools
import json
import math
import os
import sys

import numpy as np

DEFAULTS = {"dense_eval_workgroups": 0, "dense_delta_workgroups": 512, "dense_update_moved_share": 64}
CANDIDATES = {
    "dense_eval_workgroups": [0, 256, 512, 768],
    "dense_delta_workgroups": [256, 512, 1024],
    "dense_update_moved_share": [64, 128, 256, -1],
}


def size_bin(n: int, e: int, C: int, n_batches: int = 1) -> str:
    """Key of the size bin a sweep falls in."""
    cb = 0 if C <= 8 else 1 if C <= 24 else 2 if C <= 48 else 3
    return f"n{max(0, int(math.log2(max(n, 1))))}_k{max(0, int(math.log2(max(2 * e, 1))))}_c{cb}_b{int(n_batches)}"


def set_knobs(knobs: dict):
    from . import sbp
    for k, v in knobs.items():
        sbp.sbp_tune(k, v)


def _time_chain(dg, lab0, C, seed, sweeps, n_batches, repeats):
    """Milliseconds per sweep (best of `repeats` chains) and the final labels."""
    import torch
    from . import sbp
    best = float("inf")
    final = None
    for _ in range(repeats):
        lab = sbp.labels(lab0, dg.device)
        bm = sbp.sbp_build_blockmodel(dg, lab, C)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for k in range(sweeps):
            sbp.sbp_nodal_sweep(dg, lab, C, bm, seed, k, n_batches=n_batches, trace=False, stats=False)
        t1.record()
        torch.cuda.synchronize()
        best = min(best, t0.elapsed_time(t1) / sweeps)
        out = lab.cpu().numpy()
        if final is not None and not np.array_equal(out, final):
            raise RuntimeError("the same chain gave two different assignments")
        final = out
    return best, final


def tune_graph(dg, lab0, C, seed=1, sweeps=8, n_batches=1, repeats=3, candidates=None, log=None):
    """Time every candidate shape on (dg, lab0, C); return (best knobs, table of times)."""
    if C > 64:
        raise ValueError("the autotuner covers the dense tier (C <= 64)")
    cand = candidates or CANDIDATES
    keys = sorted(cand)
    table = []
    ref = None
    try:
        for vals in itertools.product(*(cand[k] for k in keys)):
            knobs = dict(zip(keys, vals))
            set_knobs(knobs)
            ms, lab = _time_chain(dg, lab0, C, seed, sweeps, n_batches, repeats)
            if ref is None:
                ref = lab
            elif not np.array_equal(lab, ref):
                raise RuntimeError(f"launch shape {knobs} changed the result")
            table.append((ms, knobs))
            if log:
                log(f"{knobs}: {ms * 1000:.1f} us/sweep")
    finally:
        set_knobs(DEFAULTS)
    table.sort(key=lambda t: t[0])
    return table[0][1], table


def load(path: str) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def apply(path: str, n: int, e: int, C: int, n_batches: int = 1) -> dict:
    """Set the knobs of the graph's size bin from the cache (defaults if absent); returns them."""
    entry = load(path).get(size_bin(n, e, C, n_batches))
    knobs = dict(DEFAULTS)
    if entry:
        knobs.update({k: int(v) for k, v in entry["knobs"].items() if k in DEFAULTS})
    set_knobs(knobs)
    return knobs


def record(path: str, n: int, e: int, C: int, n_batches: int, knobs: dict, table):
    cache = load(path)
    cache[size_bin(n, e, C, n_batches)] = {
        "knobs": knobs, "us_per_sweep": round(table[0][0] * 1000, 2),
        "default_us_per_sweep": round(next(ms for ms, k in table if k == _default_like(k)) * 1000, 2)
        if any(k == _default_like(k) for _, k in table) else None,
        "graph": {"n": int(n), "e": int(e), "C": int(C), "n_batches": int(n_batches)}}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _default_like(knobs):
    return {k: DEFAULTS[k] for k in knobs}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default="tune.json")
    ap.add_argument("--sweeps", type=int, default=8)
    ap.add_argument("--repeats", type=int, default=3)
    args = ap.parse_args(argv)
    import torch
    from . import gen, sbp
    torch.cuda.set_device(0)
    work = [("200k sweep", gen.sweep_200k(), 45, 1),
            ("1k graph", gen.plain_1k(), 10, 1),
            ("50k graph", gen.batch_graph(50_000, seed=3001), 45, 1)]
    for name, g, C, nb in work:
        dg = sbp.DeviceGraph(g)
        lab0 = gen.initial_labels(g.n, C)
        knobs, table = tune_graph(dg, lab0, C, sweeps=args.sweeps, n_batches=nb, repeats=args.repeats,
                                  log=lambda m: print(f"[tune] {name}: {m}", file=sys.stderr, flush=True))
        record(args.out, g.n, g.e, C, nb, knobs, table)
        print(json.dumps({"workload": name, "bin": size_bin(g.n, g.e, C, nb), "knobs": knobs,
                          "us_per_sweep": table[0][0] * 1000}), flush=True)


if __name__ == "__main__":
    main()
