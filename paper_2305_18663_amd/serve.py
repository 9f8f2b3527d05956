"""Continuous-batching partition server on one GPU.

Requests (directed graphs) arrive over time.  A request is admitted when its
HBM footprint fits: its CSR/CSC and output assignment (resident on the
device from upload to completion) plus its share of the engine (vertices,
edges, a slot).  Admitted graphs advance together: every engine step runs
one step of each graph's own partition (a merge phase, one sweep batch or a
compaction) in shared launches, and graphs that finish leave at once, freeing
room for the next arrivals.  Each result is bit-identical to running the
graph alone (the engine's launches never mix graphs' arithmetic).

The sequential baseline serves the same trace one request at a time with the
plain single-graph partition call.
"""
from __future__ import annotations

import dataclasses
import time
from collections import deque

import numpy as np
import torch

from . import sbp


@dataclasses.dataclass
class Request:
    tag: int
    graph: object          # gen.Graph (host arrays)
    arrival: float         # seconds after the start of the run
    params: dict
    admitted: float = -1.0
    done: float = -1.0
    C: int = 0
    dl: float = 0.0
    labels: np.ndarray | None = None
    error: str | None = None   # set when the request can never be served (it is not run)
    trace: np.ndarray | None = None


def graph_bytes(n: int, e: int) -> int:
    """Device bytes a request holds while resident (graph + output assignment)."""
    return 4 * (2 * (n + 1) + 2 * max(e, 1)) + 4 * n


class PartitionServer:
    """Admission by HBM footprint, continuous batching through sbp.Engine."""

    def __init__(self, hbm_budget: int, max_vertices: int, max_edges: int, max_graphs: int, device="cuda"):
        self.device = torch.device(device)
        self.engine = sbp.Engine(max_vertices, max_edges, max_graphs, device)
        self.engine_bytes = self.engine.ws.numel()
        self.budget = int(hbm_budget) - self.engine_bytes
        if self.budget <= 0:
            raise ValueError("HBM budget smaller than the engine workspace")
        self.max_vertices, self.max_edges, self.max_graphs = int(max_vertices), int(max_edges), int(max_graphs)
        self.in_use = 0
        self.used_v = self.used_e = 0
        self.resident = {}
        self.staged = {}  # tag -> DeviceGraph uploaded for an admission that has not succeeded yet

    def never_fits(self, req: Request) -> str | None:
        """Why the request cannot be served even by an empty engine, or None."""
        g = req.graph
        if g.n > self.max_vertices:
            return f"{g.n} vertices exceed the engine's {self.max_vertices}"
        if g.e > self.max_edges:
            return f"{g.e} edges exceed the engine's {self.max_edges}"
        if graph_bytes(g.n, g.e) > self.budget:
            return "graph larger than the HBM budget"
        return None

    def _try_admit(self, req: Request, now: float) -> bool:
        g = req.graph
        need = graph_bytes(g.n, g.e)
        # host-side checks first, so a request that does not fit now is not uploaded
        if (self.in_use + need > self.budget or self.used_v + g.n > self.max_vertices or
                self.used_e + g.e > self.max_edges or len(self.resident) >= self.max_graphs):
            return False
        dg = self.staged.pop(req.tag, None) or sbp.DeviceGraph(g, self.device)
        if not self.engine.admit(dg, req.tag, **req.params):
            self.staged[req.tag] = dg  # kept for the next attempt (engine pool fragmentation)
            return False
        self.in_use += need
        self.used_v += g.n
        self.used_e += g.e
        self.resident[req.tag] = (dg, need)
        req.admitted = now
        return True

    def run(self, requests: list[Request], clock=time.perf_counter):
        """Serve the requests at their arrival times; returns them completed.
        A request that can never fit is answered at once with `error` set."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        by_tag = {r.tag: r for r in requests}
        active = 0
        t0 = clock()
        while pending or active:
            now = clock() - t0
            # admit in arrival order while the head fits
            while pending and pending[0].arrival <= now:
                head = pending[0]
                why = self.never_fits(head)
                if why is not None:
                    head.error = why
                    head.admitted = head.done = now
                    pending.popleft()
                    continue
                if not self._try_admit(head, now):
                    break
                pending.popleft()
                active += 1
            if active == 0:
                if pending:
                    time.sleep(max(0.0, min(pending[0].arrival - now, 0.01)))
                continue
            self.engine.step()
            for tag, C, dl, out, trace in self.engine.poll():
                r = by_tag[tag]
                r.done = clock() - t0
                r.C, r.dl = C, dl
                r.labels = out.cpu().numpy()
                r.trace = trace
                dg, need = self.resident.pop(tag)
                self.in_use -= need
                self.used_v -= r.graph.n
                self.used_e -= r.graph.e
                active -= 1
        return requests

    def close(self):
        self.engine.close()


def serve_sequential(requests: list[Request], device="cuda", clock=time.perf_counter, progress=None):
    """The same arrival trace, one plain partition at a time (FIFO)."""
    t0 = clock()
    for i, r in enumerate(sorted(requests, key=lambda r: r.arrival)):
        if progress and i % 25 == 24:
            progress(f"sequential: {i + 1}/{len(requests)} served")
        now = clock() - t0
        if r.arrival > now:
            time.sleep(r.arrival - now)
        r.admitted = clock() - t0
        dg = sbp.DeviceGraph(r.graph, device)
        res = sbp.sbp_partition(dg, **r.params)
        r.done = clock() - t0
        r.C, r.dl, r.labels = res["C"], res["dl"], res["lab"]
    return requests


def latency_summary(requests: list[Request]) -> dict:
    served = [r for r in requests if r.error is None]
    lat = np.array([r.done - r.arrival for r in served])
    makespan = max(r.done for r in served) - min(r.arrival for r in served)
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "graphs_per_s": len(served) / makespan, "makespan_s": makespan,
            "rejected": len(requests) - len(served)}
