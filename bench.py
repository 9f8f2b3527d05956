"""Benchmark: asynchronous-Gibbs sweeps of stochastic block partitioning on one MI355X.

Workload: directed degree-corrected SBM, 200,000 vertices, 45 blocks with
sizes spread 5x, 4,000,000 edges, within:between ratio 2.5, power-law degrees
(exponent 2.1, [1, 100]), seeded; start assignment uniform over 45 blocks
(seed 2001).  One step = one sweep in which every vertex proposes a move
against the blockmodel at the start of the sweep (Alg. 2 in its
asynchronous-Gibbs form), followed by the exact update of M, the block
degrees, the proposal tables and the FP64 description length.

Prints one JSON line: vertex proposals per second over K timed sweeps (inputs
resident in HBM), the HBM roofline of the sweep-evaluation kernel (timed with
HIP events on its launch stream), and the CPU oracle on a bounded sample of
the same sweeps.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
TIMED_LAUNCHES = 5  # evaluation launches timed with HIP events in the timed loop (evenly spaced)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_eval_traffic.json")
EVAL_SOURCE = os.path.join(ROOT, "paper_2305_18663_amd", "csrc", "sbp_dense.hip")


def source_hash():
    """Hash of the evaluation kernel's source and its compile flags."""
    import hashlib
    from paper_2305_18663_amd import build
    h = hashlib.sha256(open(EVAL_SOURCE, "rb").read())
    h.update(" ".join(build.flags_of(os.path.basename(EVAL_SOURCE))).encode())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per evaluation launch from the committed counter runs, or None
    when the kernel source changed since they were taken."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256_16") != source_hash():
        return None
    return rec.get("bytes_per_launch")


def eval_bytes_per_sweep(g):
    """Algorithmic bytes of one sweep-evaluation launch over all vertices:
    per vertex 2 pointer pairs (8 B amortised), its label (4 B) and the
    new-label write (4 B); per edge end the neighbour id (4 B) and the
    neighbour's label (4 B)."""
    return 16 * g.n + 8 * (2 * g.e)


def host_cpu():
    """CPU model, logical CPUs and the cores this process may run on."""
    model = platform.processor() or platform.machine()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        allowed = sorted(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = list(range(os.cpu_count() or 1))
    return model, os.cpu_count() or 1, allowed


class pinned_to_one_core:
    """Runs the enclosed code with this process pinned to one allowed core."""

    def __enter__(self):
        self.core = None
        try:
            self.saved = os.sched_getaffinity(0)
            self.core = max(self.saved)
            os.sched_setaffinity(0, {self.core})
        except (AttributeError, OSError):
            self.saved = None
        return self

    def __exit__(self, *exc):
        if self.saved is not None:
            os.sched_setaffinity(0, self.saved)


def cpu_baseline(g, lab0, C, seed, budget_s=15.0, max_sweeps=4):
    """The oracle (single-threaded FP64 C, gcc -O2) on the first sweeps of the
    same workload, pinned to one core of the host."""
    from oracle import oracle as O
    O.build()
    model, nproc, allowed = host_cpu()
    lab = lab0.copy()
    with pinned_to_one_core() as pin:
        t0 = time.perf_counter()
        done = 0
        while done < max_sweeps:
            r = O.nodal_sweep(g, lab, C, seed, done)
            lab = r["lab"]
            done += 1
            if time.perf_counter() - t0 > budget_s:
                break
        dt = time.perf_counter() - t0
    return {"value": g.n * done / dt, "unit": "vertex proposals/s", "cores": 1, "kind": "oracle",
            "sample": f"first {done} sweeps of the same 200k-vertex workload, single-threaded FP64 C oracle "
                      f"(gcc -O2), {dt:.1f} s",
            "cpu_model": model, "nproc": nproc, "allowed_cores": len(allowed), "pinned_core": pin.core}


def _batch_member(args):
    from paper_2305_18663_amd import gen
    n, seed = args
    return gen.batch_graph(int(n), seed=int(seed))


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_graphs(specs, workers=16):
    """Seeded graphs generated in fresh (spawned) processes, before any GPU use."""
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(min(workers, len(specs))) as pool:
        return pool.map(_batch_member, specs, chunksize=4)


def _oracle_batch_worker(core, go, nxt, lock, q, specs, deadline_s):
    """One oracle process of the batch workload's CPU legs: waits for `go`,
    then partitions graphs in the batch's order (the next index from the
    shared counter) on its own core until `deadline_s` seconds have passed."""
    from oracle import oracle as O
    from paper_2305_18663_amd import gen
    try:
        os.sched_setaffinity(0, {core})
    except (AttributeError, OSError):
        pass
    O.lib()
    go.wait()
    t_start = time.perf_counter()
    while time.perf_counter() - t_start < deadline_s:
        with lock:
            i = nxt.value
            nxt.value += 1
        if i >= len(specs):
            break
        n, gseed, pseed = specs[i]
        g = gen.batch_graph(int(n), seed=int(gseed))
        t0 = time.perf_counter()
        r = O.partition(g, seed=int(pseed))
        q.put((i, time.perf_counter() - t0, time.perf_counter() - t_start, int(r["C"]), float(r["dl"]), r["lab"]))
    q.put(None)


def _start_oracle_legs(specs, budget_s):
    """The CPU legs of the batch workload, started before any GPU use: one
    process on one core (sequential), then a pool with a process per host core
    the benchmark may use (up to 16).  Each leg runs when its event is set."""
    import multiprocessing as mp

    from oracle import oracle as O
    O.build()  # once, before the workers load it
    ctx = mp.get_context("spawn")
    _, _, allowed = host_cpu()
    legs = {}
    for name, cores in (("sequential", allowed[-1:]), ("pool", allowed[-min(16, len(allowed)):])):
        go, q, nxt, lock = ctx.Event(), ctx.Queue(), ctx.Value("i", 0), ctx.Lock()
        procs = [ctx.Process(target=_oracle_batch_worker, args=(c, go, nxt, lock, q, specs, budget_s), daemon=True)
                 for c in cores]
        for p in procs:
            p.start()
        legs[name] = (go, q, procs, nxt, lock)  # the parent keeps every shared object alive
    return legs


def _run_oracle_leg(leg, budget_s, grace_s=10.0):
    """Sets the leg going and gathers (index, time, finish, C, DL, labels) per
    graph finished within the budget and a short grace; a graph still running
    then is dropped with its process."""
    go, q, procs = leg[:3]
    go.set()
    out, ended = [], 0
    t_end = time.perf_counter() + budget_s + grace_s
    while ended < len(procs) and time.perf_counter() < t_end:
        try:
            item = q.get(timeout=max(0.1, t_end - time.perf_counter()))
        except Exception:
            break
        if item is None:
            ended += 1
        else:
            out.append(item)
    for p in procs:
        if p.is_alive():
            p.terminate()
        p.join()
    return out


def bench_batch(args):
    """256 uneven DCSBM graphs: one batched partition vs 256 plain partitions,
    and the oracle's partitions of the same graphs on the host (a bounded leg
    on one core and one on a process pool)."""
    import numpy as np
    from paper_2305_18663_amd import gen
    sizes = gen.batch_sizes(args.graphs, seed=3000)
    specs = [(int(n), 3000 + i, 4000 + i) for i, n in enumerate(sizes)]
    legs = _start_oracle_legs(specs, args.batch_oracle_budget) if args.batch_oracle_budget > 0 else None
    graphs = make_graphs([(n, 3000 + i) for i, n in enumerate(sizes)])
    progress(f"generated {len(graphs)} graphs")
    import torch
    from paper_2305_18663_amd import sbp
    torch.cuda.set_device(0)
    dgs = [sbp.DeviceGraph(g, "cuda:0") for g in graphs]
    params = [dict(seed=4000 + i) for i in range(len(dgs))]
    sbp.sbp_partition(dgs[0], **params[0])  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batched = sbp.sbp_partition_batch(dgs, params)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    progress(f"batched partition of {len(dgs)} graphs: {t_b:.2f} s")
    t0 = time.perf_counter()
    plain = []
    for i, d in enumerate(dgs):
        plain.append(sbp.sbp_partition(d, **params[i]))
        if i % 32 == 31:
            progress(f"plain partitions: {i + 1}/{len(dgs)}")
    torch.cuda.synchronize()
    t_p = time.perf_counter() - t0
    same = all(b["C"] == p["C"] and b["dl"] == p["dl"] and np.array_equal(b["lab"], p["lab"])
               for b, p in zip(batched, plain))
    oracle = None
    if legs:
        model, nproc, allowed = host_cpu()
        e_all = float(sum(g.e for g in graphs))
        oracle = {"kind": "oracle", "budget_s": args.batch_oracle_budget, "cpu_model": model, "nproc": nproc}
        for name in ("sequential", "pool"):
            res = _run_oracle_leg(legs[name], args.batch_oracle_budget)
            progress(f"oracle {name}: {len(res)} graphs")
            if not res:
                oracle[name] = {"graphs": 0}
                continue
            wall = max(r[2] for r in res)
            busy = sum(r[1] for r in res)
            e_done = float(sum(graphs[r[0]].e for r in res))
            ident = all(r[3] == batched[r[0]]["C"] and np.array_equal(r[5], batched[r[0]]["lab"]) for r in res)
            oracle[name] = {"cores": len(legs[name][2]), "graphs": len(res), "wall_s": wall,
                            "graphs_per_s": len(res) / wall,
                            "edge_share": e_done / e_all,
                            # the whole batch at the sample's rate per edge end
                            "est_all_graphs_s": wall * e_all / e_done,
                            "identical_to_gpu": bool(ident),
                            "sample": f"graphs in the batch's order until {args.batch_oracle_budget:.0f} s had passed; "
                                      f"{busy:.1f} s of oracle time"}
    line = {"metric": "graphs/s, batched vs plain (256 uneven DCSBM graphs)", "value": len(dgs) / t_b,
            "unit": "graphs/s", "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": f"{len(dgs)} directed DCSBM graphs, N lognormal on [500, 50000] (median 5000), "
                                   f"~sqrt(N) planted blocks, E = 8N, ratio 2.5; whole method from C = N",
                       "total_vertices": int(sizes.sum()), "total_edges": int(sum(g.e for g in graphs))},
            "batched_s": t_b, "plain_s": t_p, "plain_graphs_per_s": len(dgs) / t_p, "speedup": t_p / t_b,
            "identical_results": bool(same),
            "mean_C": float(np.mean([b["C"] for b in batched]))}
    if oracle:
        line["cpu_baseline"] = oracle
    print(json.dumps(line), flush=True)


def bench_serve(args):
    """Poisson stream of partition requests at 70% of measured batched capacity."""
    import numpy as np
    from paper_2305_18663_amd import gen
    sizes = gen.request_sizes(args.requests, seed=5001)
    cal_sizes = gen.request_sizes(args.calibration, seed=5002)
    graphs = make_graphs([(n, 6000 + j) for j, n in enumerate(sizes)] +
                         [(n, 9000 + j) for j, n in enumerate(cal_sizes)])
    req_graphs, cal_graphs = graphs[:len(sizes)], graphs[len(sizes):]
    import torch
    from paper_2305_18663_amd import serve
    torch.cuda.set_device(0)
    V = 2_000_000
    E = 8 * V
    budget = 48 << 30
    # capacity: the calibration draw all at time 0
    srv = serve.PartitionServer(budget, V, E, 512)
    cal = [serve.Request(j, g, 0.0, dict(seed=7000 + j)) for j, g in enumerate(cal_graphs)]
    srv.run(cal)
    progress("calibration done")
    capacity = serve.latency_summary(cal)["graphs_per_s"]
    rate = 0.7 * capacity
    rng = np.random.default_rng(5000)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, len(req_graphs)))
    reqs = [serve.Request(j, g, float(a), dict(seed=8000 + j)) for j, (g, a) in enumerate(zip(req_graphs, arrivals))]
    srv.run(reqs)
    srv.close()
    progress("batched serving done")
    batched = serve.latency_summary(reqs)
    seq = [serve.Request(j, g, float(a), dict(seed=8000 + j)) for j, (g, a) in enumerate(zip(req_graphs, arrivals))]
    serve.serve_sequential(seq, progress=progress)
    plain = serve.latency_summary(seq)
    same = all(a.C == b.C and a.dl == b.dl and np.array_equal(a.labels, b.labels) for a, b in zip(reqs, seq))
    line = {"metric": "graphs/s and p50/p99 latency, continuous batching vs plain (Poisson requests)",
            "value": batched["graphs_per_s"], "unit": "graphs/s", "n_gpus": 1, "higher_is_better": True,
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"{len(reqs)} requests, N lognormal on [1000, 200000] (median 14142), "
                                   f"~sqrt(N) planted blocks, E = 8N; Poisson arrivals at 70% of the batched "
                                   f"capacity measured on {len(cal)} calibration requests",
                       "arrival_rate_per_s": rate, "capacity_graphs_per_s": capacity,
                       "hbm_budget_bytes": budget, "engine_vertices": V, "engine_edges": E},
            "batched": batched, "plain": plain, "identical_results": bool(same)}
    print(json.dumps(line), flush=True)


def _oracle_partition_child(q, which, seed):
    from oracle import oracle as O
    from paper_2305_18663_amd import gen
    with pinned_to_one_core():
        g = gen.plain_1k() if which == "partition1k" else gen.sweep_200k()
        t0 = time.perf_counter()
        r = O.partition(g, seed=seed)
        q.put((time.perf_counter() - t0, int(r["C"]), float(r["dl"]), r["lab"]))


def bench_partition(args):
    """The whole method (merges, MCMC, golden search) from C = N on one graph:
    the 1k-vertex, 10-block workload or the 200k-vertex sweep workload, beside
    the oracle run in a child process on one core (a bounded leg: reported as
    not finished when it exceeds its budget)."""
    import multiprocessing as mp

    import numpy as np
    import torch

    from paper_2305_18663_amd import gen, sbp
    which = args.workload
    seed = 2000 if which == "partition1k" else 2001
    budget = args.oracle_budget
    ctx = mp.get_context("spawn")
    q = ctx.Queue()
    child = ctx.Process(target=_oracle_partition_child, args=(q, which, seed), daemon=True)
    child.start()  # before any GPU use in this process
    g = gen.plain_1k() if which == "partition1k" else gen.sweep_200k()
    torch.cuda.set_device(0)
    dg = sbp.DeviceGraph(g, "cuda:0")
    sbp.sbp_partition(dg, seed=seed, max_iters=2)  # warm-up (library load, first launches)
    torch.cuda.synchronize()
    times, res = [], None
    for _ in range(args.repeats):
        t0 = time.perf_counter()
        res = sbp.sbp_partition(dg, seed=seed)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    progress(f"{which}: GPU partition {min(times):.3f} s, C={res['C']}")
    oracle = {"kind": "oracle", "cores": 1, "budget_s": budget}
    try:
        t_o, C_o, dl_o, lab_o = q.get(timeout=budget)
        oracle.update(time_s=t_o, C=C_o, dl=dl_o, identical=bool(C_o == res["C"] and np.array_equal(lab_o, res["lab"])))
    except Exception:
        oracle.update(time_s=None, finished=False)
    if child.is_alive():
        child.terminate()
    child.join()
    model, nproc, _ = host_cpu()
    oracle.update(cpu_model=model, nproc=nproc)
    sweeps = int(res["trace"][:, 3].sum()) if len(res["trace"]) else 0
    line = {"metric": "whole-method partition time (from C = N)", "value": min(times), "unit": "s",
            "n_gpus": 1, "steps": args.repeats, "higher_is_better": False, "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": ("directed DCSBM N=1000, 10 equal blocks, E=8000, ratio 2.5, PL(2.1,[1,100])"
                                    if which == "partition1k" else
                                    "directed DCSBM N=200000, 45 blocks (sizes spread 5x), E=4000000, ratio 2.5"),
                       "vertices": g.n, "edges": g.e, "seed": seed},
            "times_s": times, "C": res["C"], "dl": res["dl"], "iterations": len(res["trace"]), "sweeps": sweeps,
            "dl_norm": res["dl"] / ((g.e + 1) * np.log(g.e + 1)),
            "cpu_baseline": oracle}
    if which == "partition1k":
        from sklearn.metrics import normalized_mutual_info_score
        line["nmi"] = float(normalized_mutual_info_score(res["lab"], g.planted, average_method="arithmetic"))
    print(json.dumps(line), flush=True)


def bench_sparse1m(args):
    """The 1M-vertex, 180-block sparse workload: merge scoring at C = N (the
    first merge phase), sweeps on the sparse tier at C = 500000 from a seeded
    assignment (the scale of the first MCMC phase), and the whole method."""
    import ctypes as ct
    import numpy as np
    import torch
    from paper_2305_18663_amd import gen, sbp
    torch.cuda.set_device(0)
    g = gen.sparse_1m()
    progress(f"generated N={g.n} E={g.e}")
    dg = sbp.DeviceGraph(g)
    L = sbp.lib()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    # (1) merge scoring at C = N (identity assignment), device buffers only
    C = g.n
    lab = sbp.labels(np.arange(g.n, dtype=np.int32))
    bm = sbp.sbp_build_blockmodel(dg, lab, C)
    partner = torch.empty(C, dtype=torch.int32, device="cuda")
    dS = torch.empty(C, dtype=torch.float64, device="cuda")
    dSl = torch.empty(C, dtype=torch.float64, device="cuda")
    ws = dg.workspace()
    def merge_once(phase):
        p = sbp.MergeParams(6000, phase, 10, 1, 0)
        sbp._check(L.sbp_merge_scores(ct.byref(dg.struct), sbp._ptr(lab), C, sbp._ptr(bm), ct.byref(p),
                                      sbp._ptr(partner), sbp._ptr(dS), sbp._ptr(dSl), sbp._ptr(ws), ws.numel(),
                                      sbp._stream()))
    merge_once(0)
    a, b = ev(), ev()
    torch.cuda.synchronize(); a.record()
    for k in range(args.steps):
        merge_once(k + 1)
    b.record(); torch.cuda.synchronize()
    t_merge = a.elapsed_time(b) / 1e3 / args.steps
    progress(f"merge scoring at C={C}: {t_merge * 1e3:.2f} ms per phase")
    del bm
    # (2) sparse sweeps at C = 500000 from a seeded assignment
    C2 = 500_000
    lab2 = sbp.labels(gen.initial_labels(g.n, C2, seed=2002))
    bm2 = sbp.sbp_build_blockmodel(dg, lab2, C2)
    for k in range(args.warmup):
        sbp.sbp_nodal_sweep(dg, lab2, C2, bm2, 2002, k, trace=False, stats=False)
    a, b = ev(), ev()
    torch.cuda.synchronize(); a.record()
    for k in range(args.steps):
        sbp.sbp_nodal_sweep(dg, lab2, C2, bm2, 2002, args.warmup + k, trace=False, stats=False)
    b.record(); torch.cuda.synchronize()
    t_sweep = a.elapsed_time(b) / 1e3 / args.steps
    progress(f"sparse sweep at C={C2}: {t_sweep * 1e3:.2f} ms per sweep")
    del bm2
    # (3) the whole method from C = N
    res = {"C": None, "dl": None}
    t_part = None
    if not args.skip_partition:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = sbp.sbp_partition(dg, seed=6001)
        torch.cuda.synchronize()
        t_part = time.perf_counter() - t0
        progress(f"partition: {t_part:.2f} s, C={res['C']}")
    line = {"metric": "vertex proposals/s (1M-vertex sparse sweep)", "value": g.n / t_sweep,
            "unit": "vertex proposals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": t_sweep * 1e3, "higher_is_better": True, "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": "directed DCSBM N=1000000, 180 Dirichlet(2) blocks, E=8000000, ratio 1.5, "
                                   "power-law degrees 2.1 with a hub tail; sparse tier",
                       "sweep_blocks": C2, "merge_blocks": C},
            "merge_proposals_per_s": C * 10 / t_merge, "merge_phase_ms": t_merge * 1e3,
            "partition_s": t_part, "partition_C": res["C"], "partition_dl": res["dl"]}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["sweep", "batch", "serve", "sparse1m", "partition1k", "partition200k"],
                    default="sweep")
    ap.add_argument("--repeats", type=int, default=3, help="partition workloads: timed runs")
    ap.add_argument("--oracle-budget", type=float, default=120.0,
                    help="partition workloads: seconds the oracle leg may take before it is reported unfinished")
    ap.add_argument("--graphs", type=int, default=256)
    ap.add_argument("--batch-oracle-budget", type=float, default=30.0,
                    help="batch workload: seconds for each oracle leg (one core, then a process pool); 0 = none")
    ap.add_argument("--skip-partition", action="store_true", help="sparse1m: merges and sweeps only")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--calibration", type=int, default=100)
    ap.add_argument("--hubs", type=int, default=0,
                    help="sweep workload: the highest-degree vertices moved one at a time first (hybrid sweep)")
    ap.add_argument("--cold", type=int, default=0,
                    help="sweep workload: copy this many MiB device to device before every timed sweep "
                         "(512 is twice the Infinity Cache), so each sweep starts with the graph evicted; "
                         "the copies are outside the timed sweeps")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="MiB copied device-to-device first (reference size for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported in this build "
              f"(the multi-GPU sharding is a design note, not code)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "sparse1m":
        return bench_sparse1m(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload in ("partition1k", "partition200k"):
        return bench_partition(args)

    import numpy as np
    import torch

    from paper_2305_18663_amd import gen, sbp

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    g = gen.sweep_200k()
    C, seed = 45, 2001
    lab0 = gen.initial_labels(g.n, C, seed=seed)
    dg = sbp.DeviceGraph(g, "cuda:0")
    sbp.sbp_validate_graph(dg)

    # warmup on a scratch copy
    lab = sbp.labels(lab0)
    bm = sbp.sbp_build_blockmodel(dg, lab, C)
    for k in range(args.warmup):
        sbp.sbp_nodal_sweep(dg, lab, C, bm, seed, k, trace=False, stats=False, n_hubs=args.hubs)
    torch.cuda.synchronize()

    # timed region: K sweeps from the seeded assignment
    lab = sbp.labels(lab0)
    bm = sbp.sbp_build_blockmodel(dg, lab, C, bm)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    sbp.sbp_profile_read("sweep_eval", reset=True)
    # HIP events on TIMED_LAUNCHES evenly spaced evaluation launches of the
    # timed loop: attaching them to every launch would slow each sweep by a
    # few microseconds
    stride = max(1, args.steps // TIMED_LAUNCHES)
    sbp.sbp_profile_enable(True, stride=stride)
    if args.cold:
        # every sweep starts after a copy larger than the Infinity Cache; only
        # the sweeps are timed (an event pair each)
        scrub_src = torch.ones(args.cold << 18, dtype=torch.float32, device="cuda:0")
        scrub_dst = torch.empty_like(scrub_src)
        pairs = []
        for k in range(args.steps):
            scrub_dst.copy_(scrub_src)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            sbp.sbp_nodal_sweep(dg, lab, C, bm, seed, k, trace=False, stats=False, n_hubs=args.hubs)
            b.record(stream)
            pairs.append((a, b))
        torch.cuda.synchronize()
        sbp.sbp_profile_enable(False)
        ms = sum(a.elapsed_time(b) for a, b in pairs)
        del scrub_src, scrub_dst
    else:
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for k in range(args.steps):
            sbp.sbp_nodal_sweep(dg, lab, C, bm, seed, k, trace=False, stats=False, n_hubs=args.hubs)
        end.record(stream)
        torch.cuda.synchronize()
        sbp.sbp_profile_enable(False)
        ms = start.elapsed_time(end)
    eval_ms, launches = sbp.sbp_profile_read("sweep_eval", reset=True)
    dl = sbp.sbp_description_length(dg, C, bm)

    value = g.n * args.steps / (ms / 1e3)
    avg_eval_s = eval_ms / max(launches, 1) / 1e3
    bytes_launch = eval_bytes_per_sweep(g)
    achieved = bytes_launch / avg_eval_s / 1e9
    traffic = measured_traffic() if not args.cold else None  # the committed counters are the warm runs
    line = {
        "metric": "vertex proposals/s (200k-vertex sweep)",
        "value": value,
        "unit": "vertex proposals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "directed DCSBM N=200000, 45 blocks (sizes spread 5x), E=4000000, ratio 2.5, "
                               "power-law degrees 2.1 on [1,100]; async-Gibbs sweeps from a seeded assignment",
                   "vertices": g.n, "edges": g.e, "blocks": C, "batches_per_sweep": 1, "hubs_per_sweep": args.hubs, "beta": 3.0, "eps": 1,
                   "dl_after": dl,
                   "cache": f"cold: {args.cold} MiB copied before every sweep" if args.cold else "warm"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_dense_eval", "avg_launch_us": avg_eval_s * 1e6,
                     "timed_launches": launches, "timing_stride": stride,
                     "algorithmic_bytes_per_launch": bytes_launch,
                     # the counters' bytes over the same launch time: what the HBM actually moved
                     "traffic_gbs": traffic / avg_eval_s / 1e9 if traffic else None,
                     "traffic_frac": traffic / avg_eval_s / 1e9 / HBM_PEAK_GBS if traffic else None},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(g, lab0, C, seed)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
