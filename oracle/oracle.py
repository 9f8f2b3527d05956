"""ctypes wrapper of the plain C oracle (sbp_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the HIP implementation.  Every call maps one-to-one onto a function of
sbp_oracle.c, which cites the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sbp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

I32P = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
I64P = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
F64P = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
I8P = np.ctypeslib.ndpointer(dtype=np.int8, flags="C_CONTIGUOUS")
U64P = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
U32P = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 (no fast-math, no threads)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-fPIC", "-shared", "-fno-fast-math",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ct.Structure):
    _fields_ = [("seed", ct.c_uint64), ("beta", ct.c_double), ("eps", ct.c_int64),
                ("merge_proposals", ct.c_int), ("max_sweeps", ct.c_int),
                ("t_pre", ct.c_double), ("t_post", ct.c_double), ("merge_rate", ct.c_double),
                ("n_batches", ct.c_int), ("max_iters", ct.c_int), ("n_hubs", ct.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ct.CDLL(build())
        L = _lib
        L.orc_philox4x32_10.argtypes = [U32P, U32P, U32P]
        L.orc_words.argtypes = [ct.c_uint64, ct.c_uint32, ct.c_uint32, ct.c_uint32, ct.c_uint32, U64P]
        L.orc_build_blockmodel.argtypes = [ct.c_int, I32P, I32P, I32P, ct.c_int, ct.POINTER(ct.c_int64),
                                           I32P, I32P, I64P, I64P, I64P, ct.POINTER(ct.c_double)]
        L.orc_description_length.argtypes = [ct.c_int, I32P, I32P, I32P, ct.c_int]
        L.orc_description_length.restype = ct.c_double
        L.orc_eval_move.argtypes = [ct.c_int, I32P, I32P, I32P, I32P, I32P, ct.c_int, ct.c_int, U64P,
                                    ct.c_double, ct.c_int64, ct.POINTER(ct.c_int), ct.POINTER(ct.c_double),
                                    ct.POINTER(ct.c_double), ct.POINTER(ct.c_double), ct.POINTER(ct.c_int)]
        L.orc_nodal_sweep.argtypes = [ct.c_int, I32P, I32P, I32P, I32P, I32P, ct.c_int, ct.c_uint64,
                                      ct.c_uint32, ct.c_double, ct.c_int64, ct.c_int, I32P, F64P, F64P,
                                      F64P, F64P, I8P, ct.c_void_p, I64P, ct.POINTER(ct.c_double)]
        L.orc_nodal_sweep_h.argtypes = [ct.c_int, I32P, I32P, I32P, I32P, I32P, ct.c_int, ct.c_uint64,
                                        ct.c_uint32, ct.c_double, ct.c_int64, ct.c_int, ct.c_int, I32P, F64P,
                                        F64P, F64P, F64P, I8P, ct.c_void_p, I64P, ct.POINTER(ct.c_double)]
        L.orc_hub_order.argtypes = [ct.c_int, I32P, I32P, ct.c_int, I32P]
        L.orc_merge_scores.argtypes = [ct.c_int, I32P, I32P, I32P, ct.c_int, ct.c_uint64, ct.c_uint32,
                                       ct.c_int, ct.c_int64, I32P, F64P, F64P]
        L.orc_merge_delta.argtypes = [ct.c_int, I32P, I32P, I32P, ct.c_int, ct.c_int, ct.c_int,
                                      ct.POINTER(ct.c_double), ct.POINTER(ct.c_double)]
        L.orc_merge_propose.argtypes = [ct.c_int, I32P, I32P, I32P, ct.c_int, ct.c_int, U64P, ct.c_int64]
        L.orc_merge_apply.argtypes = [ct.c_int, I32P, F64P, ct.c_int, I32P]
        L.orc_golden_insert.argtypes = [I32P, F64P, I32P, ct.c_int, ct.c_double, ct.POINTER(ct.c_int)]
        L.orc_golden_next.argtypes = [I32P, I32P, ct.c_double, ct.POINTER(ct.c_int)]
        L.orc_compact.argtypes = [ct.c_int, I32P, ct.c_int]
        L.orc_partition.argtypes = [ct.c_int, I32P, I32P, I32P, I32P, ct.c_void_p, ct.c_int,
                                    ct.POINTER(_Params), I32P, ct.POINTER(ct.c_int), ct.POINTER(ct.c_double),
                                    I64P, F64P, ct.c_int, ct.POINTER(ct.c_int)]
        U8P = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
        L.orc_induced.argtypes = [ct.c_int, I32P, I32P, I32P, I32P, U8P, I32P, I32P, I32P, I32P, I32P,
                                  ct.POINTER(ct.c_int), ct.POINTER(ct.c_int)]
        L.orc_combine_choice.argtypes = [ct.c_int, I32P, I32P, I32P, ct.c_int, ct.c_int, I32P]
        L.orc_dcsbp.argtypes = [ct.c_int, I32P, I32P, I32P, I32P, ct.c_int, ct.POINTER(_Params), I32P,
                                ct.POINTER(ct.c_int), ct.POINTER(ct.c_double), I32P]
    return _lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# ---------------------------------------------------------------- Philox
def philox(ctr, key):
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def words(seed, a, b, base, tag):
    W = np.zeros(4, np.uint64)
    lib().orc_words(seed, a, b, base, tag, W)
    return W


# ---------------------------------------------------------------- blockmodel / DL
def build_blockmodel(g, lab, C):
    """Sorted COO of M (rows, cols, vals), dout, din and DL (Sec. II-A, Eq. 1-2)."""
    lab = _i32(lab)
    e = max(g.e, 1)
    rows = np.zeros(e, np.int32); cols = np.zeros(e, np.int32); vals = np.zeros(e, np.int64)
    dout = np.zeros(max(C, 1), np.int64); din = np.zeros(max(C, 1), np.int64)
    nnz = ct.c_int64(0); dl = ct.c_double(0)
    rc = lib().orc_build_blockmodel(g.n, g.out_ptr, g.out_idx, lab, C, ct.byref(nnz), rows, cols, vals,
                                    dout, din, ct.byref(dl))
    if rc:
        raise ValueError(f"oracle build failed ({rc})")
    k = nnz.value
    return dict(rows=rows[:k], cols=cols[:k], vals=vals[:k], dout=dout[:C], din=din[:C], dl=dl.value)


def description_length(g, lab, C):
    return lib().orc_description_length(g.n, g.out_ptr, g.out_idx, _i32(lab), C)


# ---------------------------------------------------------------- moves
def eval_move(g, lab, C, v, W, beta=3.0, eps=1):
    s = ct.c_int(); dS = ct.c_double(); lnH = ct.c_double(); lnu = ct.c_double(); acc = ct.c_int()
    rc = lib().orc_eval_move(g.n, g.out_ptr, g.out_idx, g.in_ptr, g.in_idx, _i32(lab), C, v,
                             np.asarray(W, np.uint64), beta, eps, ct.byref(s), ct.byref(dS), ct.byref(lnH),
                             ct.byref(lnu), ct.byref(acc))
    if rc:
        raise ValueError("oracle eval failed")
    return dict(s=s.value, dS=dS.value, lnH=lnH.value, lnu=lnu.value, accept=bool(acc.value))


def hub_order(g, n_hubs):
    """The n_hubs vertices of highest degree (out + in ends), ties by smaller id."""
    order = np.zeros(max(n_hubs, 1), np.int32)
    if lib().orc_hub_order(g.n, g.out_ptr, g.in_ptr, n_hubs, order):
        raise ValueError("bad hub count")
    return order[:n_hubs]


def nodal_sweep(g, lab, C, seed, sweep, beta=3.0, eps=1, n_batches=1, force=None, n_hubs=0):
    """One sweep; returns new labels and per-vertex trace (Alg. 2; the n_hubs
    highest-degree vertices one at a time first, the rest in async batches)."""
    lab = _i32(lab).copy()
    n = g.n
    prop = np.zeros(n, np.int32); dS = np.zeros(n); lnH = np.zeros(n); z = np.zeros(n); lnu = np.zeros(n)
    acc = np.zeros(n, np.int8); stats = np.zeros(4, np.int64); sdS = ct.c_double()
    fptr = None
    if force is not None:
        force = np.ascontiguousarray(force, dtype=np.int8)
        fptr = force.ctypes.data
    rc = lib().orc_nodal_sweep_h(n, g.out_ptr, g.out_idx, g.in_ptr, g.in_idx, lab, C, seed, sweep, beta, eps,
                                 n_batches, n_hubs, prop, dS, lnH, z, lnu, acc, fptr, stats, ct.byref(sdS))
    if rc:
        raise ValueError("oracle sweep failed")
    return dict(lab=lab, prop=prop, dS=dS, lnH=lnH, z=z, lnu=lnu, acc=acc.astype(bool),
                proposals=int(stats[0]), self_proposals=int(stats[1]), accepted=int(stats[2]),
                forced=int(stats[3]), sum_dS=sdS.value)


# ---------------------------------------------------------------- merges
def merge_scores(g, lab, C, seed, phase, x=10, eps=1):
    partner = np.zeros(max(C, 1), np.int32); dS = np.zeros(max(C, 1)); dSl = np.zeros(max(C, 1))
    rc = lib().orc_merge_scores(g.n, g.out_ptr, g.out_idx, _i32(lab), C, seed, phase, x, eps, partner, dS, dSl)
    if rc:
        raise ValueError("oracle merge scoring failed")
    return partner[:C], dS[:C], dSl[:C]


def merge_delta(g, lab, C, c, cp):
    """(full dS, local dS) of merging blocks c and cp (Alg. 1 scoring step)."""
    dS = ct.c_double(); dSl = ct.c_double()
    if lib().orc_merge_delta(g.n, g.out_ptr, g.out_idx, _i32(lab), C, c, cp, ct.byref(dS), ct.byref(dSl)):
        raise ValueError("bad merge pair")
    return dS.value, dSl.value


def merge_propose(g, lab, C, c, W, eps=1):
    """The partner one set of words W0..W3 proposes for block c (Alg. 1 proposal step; may be c)."""
    cp = lib().orc_merge_propose(g.n, g.out_ptr, g.out_idx, _i32(lab), C, c, np.asarray(W, np.uint64), eps)
    if cp < 0:
        raise ValueError("bad merge proposal arguments")
    return cp


def merge_apply(partner, dS_local, n_merges):
    C = len(partner)
    m = np.zeros(max(C, 1), np.int32)
    newC = lib().orc_merge_apply(C, _i32(partner), np.ascontiguousarray(dS_local, np.float64), n_merges, m)
    return newC, m[:C]


def compact(lab, C):
    lab = _i32(lab).copy()
    c = lib().orc_compact(len(lab), lab, C)
    return c, lab


# ---------------------------------------------------------------- golden-ratio search (Sec. II-B)
class Golden:
    """The (hi, mid, lo) triple of the oracle's golden-ratio search over C."""

    def __init__(self):
        self.C = np.zeros(3, np.int32)
        self.dl = np.zeros(3)
        self.used = np.zeros(3, np.int32)

    def insert(self, C, dl):
        """Stores a result; returns (slot written, slot the old mid moved to or -1)."""
        moved = ct.c_int(-1)
        to = lib().orc_golden_insert(self.C, self.dl, self.used, C, dl, ct.byref(moved))
        return to, moved.value

    def next(self, merge_rate=0.5):
        """(start slot, target C), or None when the search is over."""
        t = ct.c_int(0)
        frm = lib().orc_golden_next(self.C, self.used, merge_rate, ct.byref(t))
        return None if frm < 0 else (frm, t.value)

    def slots(self):
        return [(int(self.C[k]), float(self.dl[k])) if self.used[k] else None for k in range(3)]


# ---------------------------------------------------------------- whole method
DEFAULTS = dict(seed=2000, beta=3.0, eps=1, merge_proposals=10, max_sweeps=100, t_pre=5e-4, t_post=1e-4,
                merge_rate=0.5, n_batches=2, max_iters=200, n_hubs=0)


def partition(g, lab_in=None, C_in=0, trace_cap=256, **kw):
    p = dict(DEFAULTS)
    p.update(kw)
    P = _Params(p["seed"], p["beta"], p["eps"], p["merge_proposals"], p["max_sweeps"], p["t_pre"], p["t_post"],
                p["merge_rate"], p["n_batches"], p["max_iters"], p["n_hubs"])
    lab_out = np.zeros(g.n, np.int32)
    C = ct.c_int(); dl = ct.c_double(); iters = ct.c_int()
    tr = np.zeros(5 * trace_cap, np.int64); trdl = np.zeros(trace_cap)
    lp = None
    if lab_in is not None:
        lab_in = _i32(lab_in)
        lp = lab_in.ctypes.data
    rc = lib().orc_partition(g.n, g.out_ptr, g.out_idx, g.in_ptr, g.in_idx, lp, C_in, ct.byref(P), lab_out,
                             ct.byref(C), ct.byref(dl), tr, trdl, trace_cap, ct.byref(iters))
    if rc:
        raise ValueError(f"oracle partition failed ({rc})")
    k = min(iters.value, trace_cap)
    return dict(lab=lab_out, C=C.value, dl=dl.value, trace=tr[: 5 * k].reshape(k, 5), trace_dl=trdl[:k])


def _params(kw):
    p = dict(DEFAULTS)
    p.update(kw)
    return _Params(p["seed"], p["beta"], p["eps"], p["merge_proposals"], p["max_sweeps"], p["t_pre"], p["t_post"],
                   p["merge_rate"], p["n_batches"], p["max_iters"], p["n_hubs"])


def induced(g, keep):
    """Induced subgraph of the vertices with keep[v] (Alg. 3's subgraphs):
    (sub_id [n], -1 for dropped vertices; the subgraph as a Graph)."""
    from paper_2305_18663_amd.gen import Graph
    keep = np.ascontiguousarray(keep, np.uint8)
    n, e = g.n, g.e
    sid = np.zeros(n, np.int32)
    op = np.zeros(n + 1, np.int32); ip = np.zeros(n + 1, np.int32)
    oi = np.zeros(e + 1, np.int32); ii = np.zeros(e + 1, np.int32)
    ns = ct.c_int(); es = ct.c_int()
    if lib().orc_induced(n, g.out_ptr, g.out_idx, g.in_ptr, g.in_idx, keep, sid, op, oi, ip, ii, ct.byref(ns),
                         ct.byref(es)):
        raise ValueError("induced subgraph: CSR and CSC disagree")
    k, m = ns.value, es.value
    return sid, Graph(k, m, op[: k + 1].copy(), oi[:m].copy(), ip[: k + 1].copy(), ii[:m].copy())


def combine_choice(g, lab, C1, C2):
    """For every community C1 + c2 the community of the first result it joins."""
    best = np.zeros(max(C2, 1), np.int32)
    if lib().orc_combine_choice(g.n, g.out_ptr, g.out_idx, _i32(lab), C1, C2, best):
        raise ValueError("combine: bad labels")
    return best[:C2]


def dcsbp(g, n_sub, **kw):
    """Divide-and-conquer SBP (Alg. 3) over n_sub round-robin subgraphs."""
    P = _params(kw)
    lab = np.zeros(g.n, np.int32)
    C = ct.c_int(); dl = ct.c_double()
    sub_C = np.zeros(max(n_sub, 1), np.int32)
    rc = lib().orc_dcsbp(g.n, g.out_ptr, g.out_idx, g.in_ptr, g.in_idx, n_sub, ct.byref(P), lab, ct.byref(C),
                         ct.byref(dl), sub_C)
    if rc:
        raise ValueError(f"oracle dcsbp failed ({rc})")
    return dict(lab=lab, C=C.value, dl=dl.value, sub_C=sub_C[:n_sub])
