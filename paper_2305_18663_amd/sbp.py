"""Python binding of libsbp.so (argument marshalling only).

Every function forwards to the C-ABI entry point of the same name declared in
include/sbp.h; torch supplies device memory and the current HIP stream.  The
library must be built (paper_2305_18663_amd/build.py); nothing here falls
back to another implementation.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsbp.so")

SBP_DENSE_MAX_C = 64
SBP_MAX_DEGREE = 16384
SBP_E = {0: "OK", -1: "SBP_E_ARG", -2: "SBP_E_GRAPH", -3: "SBP_E_LABEL", -4: "SBP_E_SPACE", -5: "SBP_E_HIP",
         -6: "SBP_E_LIMIT"}


class SbpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{SBP_E.get(code, code)}: {msg}")
        self.code = code


class Graph(ct.Structure):
    _fields_ = [("n", ct.c_int32), ("e", ct.c_int32), ("out_ptr", ct.c_void_p), ("out_idx", ct.c_void_p),
                ("in_ptr", ct.c_void_p), ("in_idx", ct.c_void_p)]


class SweepParams(ct.Structure):
    _fields_ = [("seed", ct.c_uint64), ("sweep", ct.c_uint32), ("n_batches", ct.c_int32), ("beta", ct.c_double),
                ("eps", ct.c_int32), ("n_hubs", ct.c_int32)]


class SweepStats(ct.Structure):
    _fields_ = [("proposals", ct.c_int64), ("self_proposals", ct.c_int64), ("accepted", ct.c_int64),
                ("near_ties", ct.c_int64), ("sum_dS_accepted", ct.c_double), ("dl_after", ct.c_double)]


class SweepTrace(ct.Structure):
    _fields_ = [("prop", ct.c_void_p), ("dS", ct.c_void_p), ("lnH", ct.c_void_p), ("margin", ct.c_void_p),
                ("accept", ct.c_void_p)]


class MergeParams(ct.Structure):
    _fields_ = [("seed", ct.c_uint64), ("phase", ct.c_uint32), ("proposals", ct.c_int32), ("eps", ct.c_int32),
                ("reserved", ct.c_int32)]


class PartitionParams(ct.Structure):
    _fields_ = [("seed", ct.c_uint64), ("beta", ct.c_double), ("eps", ct.c_int32), ("merge_proposals", ct.c_int32),
                ("max_sweeps", ct.c_int32), ("n_batches", ct.c_int32), ("t_pre", ct.c_double),
                ("t_post", ct.c_double), ("merge_rate", ct.c_double), ("max_iters", ct.c_int32),
                ("n_hubs", ct.c_int32)]


# Two batches per sweep in the whole method: a fully asynchronous sweep (one
# batch, every vertex against the same snapshot) can stall the block-count
# search on dense graphs whose description length is flat at high block
# counts; the single-sweep entry point keeps one batch as its default.
PARTITION_DEFAULTS = dict(seed=2000, beta=3.0, eps=1, merge_proposals=10, max_sweeps=100, n_batches=2,
                          t_pre=5e-4, t_post=1e-4, merge_rate=0.5, max_iters=200, n_hubs=0)

_SIGS = {
    "sbp_last_error": (ct.c_char_p, []),
    "sbp_blockmodel_bytes": (ct.c_size_t, [ct.c_int32, ct.c_int32, ct.c_int32]),
    "sbp_workspace_bytes": (ct.c_size_t, [ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32]),
    "sbp_validate_graph": (ct.c_int, [ct.POINTER(Graph), ct.c_void_p, ct.c_size_t, ct.c_void_p]),
    "sbp_graph_workspace_bytes": (ct.c_size_t, [ct.c_int32, ct.c_int32]),
    "sbp_graph_from_edges": (ct.c_int, [ct.c_int32, ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                        ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p]),
    "sbp_check_labels": (ct.c_int, [ct.c_int32, ct.c_void_p, ct.c_int32, ct.c_void_p, ct.c_size_t, ct.c_void_p]),
    "sbp_build_blockmodel": (ct.c_int, [ct.POINTER(Graph), ct.c_void_p, ct.c_int32, ct.c_void_p, ct.c_size_t,
                                        ct.c_void_p, ct.c_size_t, ct.c_void_p]),
    "sbp_blockmodel_coo": (ct.c_int, [ct.POINTER(Graph), ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                      ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.POINTER(ct.c_int64), ct.c_void_p]),
    "sbp_description_length": (ct.c_int, [ct.POINTER(Graph), ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    "sbp_nodal_sweep": (ct.c_int, [ct.POINTER(Graph), ct.c_void_p, ct.c_int32, ct.c_void_p, ct.c_size_t,
                                   ct.POINTER(SweepParams), ct.c_void_p, ct.POINTER(SweepTrace), ct.c_void_p,
                                   ct.c_size_t, ct.c_void_p]),
    "sbp_nodal_sweep_static": (ct.c_int, [ct.POINTER(Graph), ct.c_void_p, ct.c_int32, ct.c_void_p, ct.c_size_t,
                                          ct.POINTER(SweepParams), ct.c_void_p, ct.POINTER(SweepTrace),
                                          ct.c_void_p]),
    "sbp_sweep_graph_create": (ct.c_int, [ct.POINTER(Graph), ct.c_void_p, ct.c_int32, ct.c_void_p, ct.c_size_t,
                                          ct.POINTER(SweepParams), ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                          ct.c_size_t, ct.POINTER(ct.c_void_p)]),
    "sbp_sweep_graph_launch": (ct.c_int, [ct.c_void_p, ct.c_void_p]),
    "sbp_sweep_graph_destroy": (ct.c_int, [ct.c_void_p]),
    "sbp_dcsbp_workspace_bytes": (ct.c_size_t, [ct.c_int32, ct.c_int32, ct.c_int32]),
    "sbp_dcsbp": (ct.c_int, [ct.POINTER(Graph), ct.c_int32, ct.POINTER(PartitionParams), ct.c_void_p,
                             ct.POINTER(ct.c_int32), ct.POINTER(ct.c_double), ct.c_void_p, ct.c_void_p, ct.c_size_t,
                             ct.c_void_p]),
    "sbp_merge_scores": (ct.c_int, [ct.POINTER(Graph), ct.c_void_p, ct.c_int32, ct.c_void_p, ct.POINTER(MergeParams),
                                    ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p]),
    "sbp_merge_apply": (ct.c_int, [ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_int32, ct.c_void_p,
                                   ct.POINTER(ct.c_int32), ct.c_void_p, ct.c_size_t, ct.c_void_p]),
    "sbp_relabel": (ct.c_int, [ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    "sbp_compact": (ct.c_int, [ct.c_int32, ct.c_void_p, ct.c_int32, ct.POINTER(ct.c_int32), ct.c_void_p,
                               ct.c_size_t, ct.c_void_p]),
    "sbp_partition_workspace_bytes": (ct.c_size_t, [ct.c_int32, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32)]),
    "sbp_partition": (ct.c_int, [ct.POINTER(Graph), ct.c_void_p, ct.c_int32, ct.POINTER(PartitionParams),
                                 ct.c_void_p, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_double), ct.c_void_p,
                                 ct.c_size_t, ct.c_void_p]),
    "sbp_partition_batch": (ct.c_int, [ct.c_int32, ct.POINTER(Graph), ct.POINTER(PartitionParams),
                                       ct.POINTER(ct.c_void_p), ct.POINTER(ct.c_int32), ct.POINTER(ct.c_double),
                                       ct.c_void_p, ct.c_size_t, ct.c_void_p]),
    "sbp_partition_trace": (ct.c_int, [ct.c_int64, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_double), ct.c_int32]),
    "sbp_engine_graph_bytes": (ct.c_size_t, [ct.c_int32, ct.c_int32]),
    "sbp_engine_workspace_bytes": (ct.c_size_t, [ct.c_int64, ct.c_int64, ct.c_int32]),
    "sbp_engine_create": (ct.c_int, [ct.c_void_p, ct.c_size_t, ct.c_int64, ct.c_int64, ct.c_int32, ct.c_void_p,
                                     ct.POINTER(ct.c_void_p)]),
    "sbp_engine_admit": (ct.c_int, [ct.c_void_p, ct.POINTER(Graph), ct.POINTER(PartitionParams), ct.c_void_p,
                                    ct.c_int32, ct.c_int64]),
    "sbp_engine_step": (ct.c_int, [ct.c_void_p, ct.POINTER(ct.c_int32)]),
    "sbp_engine_poll": (ct.c_int, [ct.c_void_p, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int32),
                                   ct.POINTER(ct.c_double)]),
    "sbp_engine_destroy": (ct.c_int, [ct.c_void_p]),
    "sbp_tune": (ct.c_int, [ct.c_char_p, ct.c_int64]),
    "sbp_profile_enable": (ct.c_int, [ct.c_int32]),
    "sbp_profile_read": (ct.c_int, [ct.c_char_p, ct.POINTER(ct.c_double), ct.POINTER(ct.c_int64), ct.c_int32]),
}

_lib = None


def lib():
    """Load libsbp.so; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_2305_18663_amd/build.py (hipcc, gfx950)")
        L = ct.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise SbpError(rc, lib().sbp_last_error().decode())


def _stream():
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ct.c_void_p(t.data_ptr()) if t is not None else None


def _buffer(nbytes, device):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


class DeviceGraph:
    """CSR/CSC of a graph resident in device memory."""

    def __init__(self, g, device="cuda"):
        self.n, self.e = int(g.n), int(g.e)
        self.device = torch.device(device)
        self.out_ptr = torch.from_numpy(np.ascontiguousarray(g.out_ptr, np.int32)).to(self.device)
        self.out_idx = torch.from_numpy(np.ascontiguousarray(g.out_idx, np.int32)).to(self.device)
        self.in_ptr = torch.from_numpy(np.ascontiguousarray(g.in_ptr, np.int32)).to(self.device)
        self.in_idx = torch.from_numpy(np.ascontiguousarray(g.in_idx, np.int32)).to(self.device)
        if self.e == 0:  # keep valid pointers for empty edge arrays
            self.out_idx = torch.zeros(1, dtype=torch.int32, device=self.device)
            self.in_idx = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.struct = Graph(self.n, self.e, self.out_ptr.data_ptr(), self.out_idx.data_ptr(),
                            self.in_ptr.data_ptr(), self.in_idx.data_ptr())
        self._ws = None

    def workspace(self):
        if self._ws is None:
            self._ws = _buffer(lib().sbp_workspace_bytes(0, self.n, self.e, 1), self.device)
        return self._ws


def labels(x, device="cuda"):
    return torch.from_numpy(np.ascontiguousarray(x, np.int32)).to(device)


# ------------------------------------------------------------------ graph / labels
def sbp_graph_from_edges(n, src, dst, device="cuda"):
    """Device CSR/CSC from an edge list; returns a DeviceGraph built on the GPU."""
    s = torch.as_tensor(np.ascontiguousarray(src, np.int32)).to(device)
    d = torch.as_tensor(np.ascontiguousarray(dst, np.int32)).to(device)
    e = s.numel()
    out_ptr = torch.empty(n + 1, dtype=torch.int32, device=device)
    in_ptr = torch.empty_like(out_ptr)
    out_idx = torch.empty(max(e, 1), dtype=torch.int32, device=device)
    in_idx = torch.empty_like(out_idx)
    ws = _buffer(lib().sbp_graph_workspace_bytes(n, e), device)
    _check(lib().sbp_graph_from_edges(n, e, _ptr(s), _ptr(d), _ptr(out_ptr), _ptr(out_idx), _ptr(in_ptr),
                                      _ptr(in_idx), _ptr(ws), ws.numel(), _stream()))
    dg = DeviceGraph.__new__(DeviceGraph)
    dg.n, dg.e, dg.device = n, e, torch.device(device)
    dg.out_ptr, dg.out_idx, dg.in_ptr, dg.in_idx = out_ptr, out_idx, in_ptr, in_idx
    dg.struct = Graph(n, e, out_ptr.data_ptr(), out_idx.data_ptr(), in_ptr.data_ptr(), in_idx.data_ptr())
    dg._ws = None
    return dg


def sbp_validate_graph(dg: DeviceGraph):
    ws = dg.workspace()
    _check(lib().sbp_validate_graph(ct.byref(dg.struct), _ptr(ws), ws.numel(), _stream()))


def sbp_check_labels(dg: DeviceGraph, assign, C):
    ws = dg.workspace()
    _check(lib().sbp_check_labels(dg.n, _ptr(assign), C, _ptr(ws), ws.numel(), _stream()))


# ------------------------------------------------------------------ blockmodel / DL
def sbp_blockmodel_bytes(n, e, C):
    return lib().sbp_blockmodel_bytes(n, e, C)


def sbp_build_blockmodel(dg: DeviceGraph, assign, C, bm=None):
    nb = lib().sbp_blockmodel_bytes(dg.n, dg.e, C)
    if bm is None:
        bm = _buffer(nb, dg.device)
    ws = dg.workspace()
    _check(lib().sbp_build_blockmodel(ct.byref(dg.struct), _ptr(assign), C, _ptr(bm), bm.numel(), _ptr(ws),
                                      ws.numel(), _stream()))
    return bm


def sbp_blockmodel_coo(dg: DeviceGraph, C, bm):
    cap = max(dg.e, C * C, 1)
    rows = torch.empty(cap, dtype=torch.int32, device=dg.device)
    cols = torch.empty_like(rows)
    vals = torch.empty_like(rows)
    dout = torch.empty(C, dtype=torch.int32, device=dg.device)
    din = torch.empty_like(dout)
    nnz = ct.c_int64()
    _check(lib().sbp_blockmodel_coo(ct.byref(dg.struct), C, _ptr(bm), _ptr(rows), _ptr(cols), _ptr(vals),
                                    _ptr(dout), _ptr(din), ct.byref(nnz), _stream()))
    k = nnz.value
    return dict(rows=rows[:k].cpu().numpy(), cols=cols[:k].cpu().numpy(), vals=vals[:k].cpu().numpy(),
                dout=dout.cpu().numpy(), din=din.cpu().numpy())


def sbp_description_length(dg: DeviceGraph, C, bm):
    out = torch.empty(1, dtype=torch.float64, device=dg.device)
    _check(lib().sbp_description_length(ct.byref(dg.struct), C, _ptr(bm), _ptr(out), _stream()))
    return float(out.item())


# ------------------------------------------------------------------ sweeps
def sbp_nodal_sweep(dg: DeviceGraph, assign, C, bm, seed, sweep, beta=3.0, eps=1, n_batches=1, trace=True,
                    stats=True, n_hubs=0, static=False):
    """One sweep; assign and bm are updated in place.  Returns trace/stats dicts.
    n_hubs > 0: the hybrid sweep (the highest-degree vertices one at a time
    first; dense tier only).  static: the allocation-free entry point
    (sbp_nodal_sweep_static; no workspace)."""
    p = SweepParams(seed, sweep, n_batches, beta, eps, n_hubs)
    tr = None
    out = {}
    if trace:
        out["prop"] = torch.empty(dg.n, dtype=torch.int32, device=dg.device)
        out["dS"] = torch.empty(dg.n, dtype=torch.float64, device=dg.device)
        out["lnH"] = torch.empty(dg.n, dtype=torch.float64, device=dg.device)
        out["margin"] = torch.empty(dg.n, dtype=torch.float64, device=dg.device)
        out["accept"] = torch.empty(dg.n, dtype=torch.int8, device=dg.device)
        tr = SweepTrace(*(out[k].data_ptr() for k in ("prop", "dS", "lnH", "margin", "accept")))
    st = torch.zeros(6, dtype=torch.float64, device=dg.device) if stats else None
    if static:
        _check(lib().sbp_nodal_sweep_static(ct.byref(dg.struct), _ptr(assign), C, _ptr(bm), bm.numel(), ct.byref(p),
                                            _ptr(st), ct.byref(tr) if tr is not None else None, _stream()))
    else:
        ws = dg.workspace()
        _check(lib().sbp_nodal_sweep(ct.byref(dg.struct), _ptr(assign), C, _ptr(bm), bm.numel(), ct.byref(p),
                                     _ptr(st), ct.byref(tr) if tr is not None else None, _ptr(ws), ws.numel(),
                                     _stream()))
    res = {}
    if trace:
        res = {k: v.cpu().numpy() for k, v in out.items()}
        res["accept"] = res["accept"].astype(bool)
    if stats:
        res.update(_stats_dict(st))
    return res


def _stats_dict(st):
    raw = st.cpu().numpy()
    ints = raw[:4].view(np.int64)
    return dict(proposals=int(ints[0]), self_proposals=int(ints[1]), accepted=int(ints[2]),
                near_ties=int(ints[3]), sum_dS=float(raw[4]), dl_after=float(raw[5]))


class SweepGraph:
    """One sweep captured as a HIP graph (sbp_sweep_graph_create); every
    launch() runs the next sweep: it reads the sweep index from device
    memory and advances it.  assign, bm and the graph must stay alive and
    unmoved while this object lives (it keeps references to them)."""

    def __init__(self, dg: DeviceGraph, assign, C, bm, seed, sweep, beta=3.0, eps=1, n_batches=1, n_hubs=0):
        self.dg, self.assign, self.bm = dg, assign, bm
        self.ws = _buffer(lib().sbp_workspace_bytes(0, dg.n, dg.e, 1), dg.device)
        self.index = torch.full((1,), int(sweep), dtype=torch.int32, device=dg.device)
        self.st = torch.zeros(6, dtype=torch.float64, device=dg.device)
        p = SweepParams(seed, sweep, n_batches, beta, eps, n_hubs)
        h = ct.c_void_p()
        _check(lib().sbp_sweep_graph_create(ct.byref(dg.struct), _ptr(assign), C, _ptr(bm), bm.numel(), ct.byref(p),
                                            _ptr(self.index), _ptr(self.st), _ptr(self.ws), self.ws.numel(),
                                            ct.byref(h)))
        self.h = h

    def launch(self):
        _check(lib().sbp_sweep_graph_launch(self.h, _stream()))

    def sweep_index(self):
        return int(self.index.cpu()[0])

    def stats(self):
        return _stats_dict(self.st)

    def close(self):
        if self.h:
            torch.cuda.current_stream().synchronize()
            _check(lib().sbp_sweep_graph_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ merges
def sbp_merge_scores(dg: DeviceGraph, assign, C, bm, seed, phase, proposals=10, eps=1):
    partner = torch.empty(C, dtype=torch.int32, device=dg.device)
    dS = torch.empty(C, dtype=torch.float64, device=dg.device)
    dSl = torch.empty(C, dtype=torch.float64, device=dg.device)
    p = MergeParams(seed, phase, proposals, eps, 0)
    ws = dg.workspace()
    _check(lib().sbp_merge_scores(ct.byref(dg.struct), _ptr(assign), C, _ptr(bm), ct.byref(p), _ptr(partner),
                                  _ptr(dS), _ptr(dSl), _ptr(ws), ws.numel(), _stream()))
    return partner.cpu().numpy(), dS.cpu().numpy(), dSl.cpu().numpy()


def sbp_merge_apply(partner, dS_local, n_merges, device="cuda"):
    C = len(partner)
    p = labels(partner, device)
    d = torch.from_numpy(np.ascontiguousarray(dS_local, np.float64)).to(device)
    m = torch.empty(C, dtype=torch.int32, device=device)
    newC = ct.c_int32()
    ws = _buffer(lib().sbp_workspace_bytes(3, C, 1, C), device)
    _check(lib().sbp_merge_apply(C, _ptr(p), _ptr(d), n_merges, _ptr(m), ct.byref(newC), _ptr(ws), ws.numel(),
                                 _stream()))
    return newC.value, m.cpu().numpy()


def sbp_relabel(assign, mapping):
    _check(lib().sbp_relabel(assign.numel(), _ptr(assign), _ptr(mapping), _stream()))


def sbp_compact(assign, C):
    n = assign.numel()
    newC = ct.c_int32()
    ws = _buffer(lib().sbp_workspace_bytes(3, max(n, C), 1, C), assign.device)
    _check(lib().sbp_compact(n, _ptr(assign), C, ct.byref(newC), _ptr(ws), ws.numel(), _stream()))
    return newC.value


# ------------------------------------------------------------------ whole method
def params(**kw):
    p = dict(PARTITION_DEFAULTS)
    p.update(kw)
    return PartitionParams(p["seed"], p["beta"], p["eps"], p["merge_proposals"], p["max_sweeps"], p["n_batches"],
                           p["t_pre"], p["t_post"], p["merge_rate"], p["max_iters"], p["n_hubs"])


def sbp_partition_trace(tag, cap=512):
    rows = (ct.c_int64 * (5 * cap))()
    dl = (ct.c_double * cap)()
    k = lib().sbp_partition_trace(tag, rows, dl, cap)
    return np.array(rows[: 5 * k], dtype=np.int64).reshape(k, 5), np.array(dl[:k])


def sbp_partition(dg: DeviceGraph, assign_in=None, C_in=0, **kw):
    p = params(**kw)
    n = (ct.c_int32 * 1)(dg.n)
    e = (ct.c_int32 * 1)(dg.e)
    ws = _buffer(lib().sbp_partition_workspace_bytes(1, n, e), dg.device)
    out = torch.empty(dg.n, dtype=torch.int32, device=dg.device)
    C = ct.c_int32()
    dl = ct.c_double()
    _check(lib().sbp_partition(ct.byref(dg.struct), _ptr(assign_in), C_in, ct.byref(p), _ptr(out), ct.byref(C),
                               ct.byref(dl), _ptr(ws), ws.numel(), _stream()))
    trace, trace_dl = sbp_partition_trace(-1)
    return dict(lab=out.cpu().numpy(), C=C.value, dl=dl.value, trace=trace, trace_dl=trace_dl)


def sbp_partition_batch(dgs, param_list=None, **kw):
    G = len(dgs)
    plist = param_list or [dict(kw) for _ in range(G)]
    P = (PartitionParams * G)(*[params(**p) for p in plist])
    graphs = (Graph * G)(*[d.struct for d in dgs])
    n = (ct.c_int32 * G)(*[d.n for d in dgs])
    e = (ct.c_int32 * G)(*[d.e for d in dgs])
    dev = dgs[0].device
    ws = _buffer(lib().sbp_partition_workspace_bytes(G, n, e), dev)
    outs = [torch.empty(d.n, dtype=torch.int32, device=dev) for d in dgs]
    optrs = (ct.c_void_p * G)(*[o.data_ptr() for o in outs])
    C = (ct.c_int32 * G)()
    dl = (ct.c_double * G)()
    _check(lib().sbp_partition_batch(G, graphs, P, optrs, C, dl, _ptr(ws), ws.numel(), _stream()))
    res = []
    for i in range(G):
        tr, trdl = sbp_partition_trace(i)
        res.append(dict(lab=outs[i].cpu().numpy(), C=C[i], dl=dl[i], trace=tr, trace_dl=trdl))
    return res


def sbp_dcsbp(dg: DeviceGraph, n_sub, **kw):
    """Divide-and-conquer SBP (Alg. 3) over n_sub round-robin subgraphs."""
    p = params(**kw)
    ws = _buffer(lib().sbp_dcsbp_workspace_bytes(dg.n, dg.e, n_sub), dg.device)
    out = torch.empty(dg.n, dtype=torch.int32, device=dg.device)
    C = ct.c_int32()
    dl = ct.c_double()
    sub_C = (ct.c_int32 * max(int(n_sub), 1))()
    _check(lib().sbp_dcsbp(ct.byref(dg.struct), int(n_sub), ct.byref(p), _ptr(out), ct.byref(C), ct.byref(dl),
                           ct.cast(sub_C, ct.c_void_p), _ptr(ws), ws.numel(), _stream()))
    trace, trace_dl = sbp_partition_trace(-1)  # the final whole-graph run
    return dict(lab=out.cpu().numpy(), C=C.value, dl=dl.value, sub_C=np.array(sub_C[:n_sub], np.int32),
                trace=trace, trace_dl=trace_dl)


def sbp_tune(key, value):
    """Set a launch-shape tuning knob (results do not depend on it)."""
    _check(lib().sbp_tune(key.encode(), int(value)))


def sbp_profile_enable(on=True, stride=1):
    """Time every `stride`-th sweep-evaluation launch with HIP events (off: on=False)."""
    _check(lib().sbp_profile_enable(int(stride) if on else 0))


def sbp_profile_read(kernel="sweep_eval", reset=True):
    """(total milliseconds, launches) of the named kernel since the last reset."""
    ms = ct.c_double()
    n = ct.c_int64()
    _check(lib().sbp_profile_read(kernel.encode(), ct.byref(ms), ct.byref(n), 1 if reset else 0))
    return ms.value, n.value


class Engine:
    """Continuous-batching partition engine over a fixed device workspace."""

    def __init__(self, max_vertices, max_edges, max_graphs, device="cuda"):
        self.device = torch.device(device)
        nbytes = lib().sbp_engine_workspace_bytes(max_vertices, max_edges, max_graphs)
        if nbytes == 0:
            raise SbpError(-1, "bad engine capacity")
        self.ws = _buffer(nbytes, self.device)
        h = ct.c_void_p()
        _check(lib().sbp_engine_create(_ptr(self.ws), self.ws.numel(), max_vertices, max_edges, max_graphs,
                                       _stream(), ct.byref(h)))
        self.h = h
        self.outputs = {}
        self.graphs = {}

    @staticmethod
    def graph_bytes(n, e):
        return lib().sbp_engine_graph_bytes(n, e)

    def admit(self, dg: DeviceGraph, tag, **kw):
        """True if admitted, False if it does not fit right now."""
        p = params(**kw)
        out = torch.empty(dg.n, dtype=torch.int32, device=dg.device)
        rc = lib().sbp_engine_admit(self.h, ct.byref(dg.struct), ct.byref(p), _ptr(out), 0, tag)
        if rc == -4:
            return False
        _check(rc)
        self.outputs[tag] = out
        self.graphs[tag] = dg
        return True

    def step(self):
        active = ct.c_int32()
        _check(lib().sbp_engine_step(self.h, ct.byref(active)))
        return active.value

    def poll(self):
        tag = ct.c_int64()
        C = ct.c_int32()
        dl = ct.c_double()
        done = []
        while lib().sbp_engine_poll(self.h, ct.byref(tag), ct.byref(C), ct.byref(dl)):
            out = self.outputs.pop(tag.value)
            self.graphs.pop(tag.value, None)
            trace, _ = sbp_partition_trace(tag.value)  # read (and so released) with the result
            done.append((tag.value, C.value, dl.value, out, trace))
        return done

    def close(self):
        if self.h:
            lib().sbp_engine_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
