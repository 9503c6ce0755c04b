"""Python face of the C ABI (same names, torch tensors for device memory).

Only argument marshalling lives here: tensors are checked for dtype, device
and contiguity and their pointers are passed to libxzzx_sa.so; torch supplies
device allocations and the current HIP stream.
"""
from __future__ import annotations

import contextlib
import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as X
from ._lib import call, lib


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _np_p(a):
    return a.ctypes.data_as(C.c_void_p)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _on(stream):
    """Allocation context for buffers a call on `stream` writes: the caching
    allocator then reuses their memory only in `stream`'s order."""
    return torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()


def _used_on(stream, *tensors):
    """Tensors allocated elsewhere that work on `stream` reads: their memory is
    not reused before that work is done (torch's record_stream)."""
    if stream is None:
        return
    for t in tensors:
        if t is not None and t.is_cuda:
            t.record_stream(stream)


def _dev(t, dtype, name):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA (HIP) tensor")
    return t


# ---------------------------------------------------------------------------
# host-side model calls
# ---------------------------------------------------------------------------
def noise(p, eta, convention=X.BIAS_RATIO):
    out = np.zeros(3, np.float64)
    call("xzzx_noise", p, eta, convention, _np_p(out))
    return out


def weights(p, pxyz):
    pxyz = np.ascontiguousarray(pxyz, np.float64)
    w = np.zeros(4, np.int32)
    wg = np.zeros(2, np.int32)
    call("xzzx_weights", p, _np_p(pxyz), _np_p(w), _np_p(wg))
    return w, wg


def schedule(kind, b0, b1, n):
    beta = np.zeros(max(n, 1), np.float64)
    call("xzzx_schedule", kind, b0, b1, n, _np_p(beta))
    return beta[:n]


def probe_valu(kind, waves_per_simd=8, iters=2000, stream=None):
    """Measured int32 lane-ops/s of one VALU instruction kind (0 xor, 1 add,
    2 bitop3, 3 mad_u64_u32) on every CU."""
    out = C.c_double()
    call("xzzx_probe_valu", kind, waves_per_simd, iters, _stream(stream), C.byref(out))
    return out.value


def probe_lds(bytes_per_read=16, waves_per_simd=8, iters=2000, stream=None):
    """Measured LDS read bytes/s (conflict-free reads of bytes_per_read)."""
    out = C.c_double()
    call("xzzx_probe_lds", bytes_per_read, waves_per_simd, iters, _stream(stream), C.byref(out))
    return out.value


class Lattice:
    def __init__(self, layout, d):
        h = C.c_void_p()
        call("xzzx_lattice_create", layout, d, C.byref(h))
        self.h = h
        self.layout, self.d = layout, d
        nq, ns, pc = C.c_int(), C.c_int(), C.c_int()
        call("xzzx_lattice_info", h, C.byref(nq), C.byref(ns), C.byref(pc))
        self.nq, self.nstab, self.per_class = nq.value, ns.value, pc.value

    def tables(self):
        ns = self.nstab
        fq = np.zeros((ns, 4), np.int32)
        fm = np.zeros((ns, 4), np.uint8)
        fc = np.zeros(ns, np.int32)
        fo = np.zeros(ns, np.int32)
        fr = np.zeros(ns, np.int32)
        call("xzzx_lattice_tables", self.h, _np_p(fq), _np_p(fm), _np_p(fc), _np_p(fo), _np_p(fr))
        return dict(fq=fq, fm=fm, fclass=fc, fcolour=fo, frank=fr)

    def logicals(self):
        lx = np.zeros(self.nq, np.uint8)
        lz = np.zeros(self.nq, np.uint8)
        call("xzzx_lattice_logicals", self.h, _np_p(lx), _np_p(lz))
        return lx, lz

    def cls(self, a, b):
        a = np.ascontiguousarray(a, np.uint8)
        b = np.ascontiguousarray(b, np.uint8)
        out = C.c_int()
        call("xzzx_class_host", self.h, _np_p(a), _np_p(b), C.byref(out))
        return out.value

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and X._lib is not None:
            X._lib.xzzx_lattice_destroy(h)
            self.h = None


class Plan:
    """Device tables for one (lattice, weights, beta schedule)."""

    def __init__(self, lattice: Lattice, w, wg, beta):
        w = np.ascontiguousarray(w, np.int32)
        wg = np.ascontiguousarray(wg, np.int32)
        beta = np.ascontiguousarray(beta, np.float64)
        h = C.c_void_p()
        bp = _np_p(beta) if len(beta) else None
        call("xzzx_plan_create", lattice.h, _np_p(w), _np_p(wg), bp, len(beta), C.byref(h))
        self.h = h
        self.lattice = lattice
        self.nq, self.nstab = lattice.nq, lattice.nstab
        self.n_sweeps = len(beta)

    def info(self):
        vals = [C.c_int() for _ in range(6)]
        call("xzzx_plan_info", self.h, *[C.byref(v) for v in vals])
        keys = ["n_qubits", "n_stabs", "n_sweeps", "n_dE", "lanes_per_chain", "kernel"]
        return {k: v.value for k, v in zip(keys, vals)}

    def set_lanes(self, lanes):
        call("xzzx_plan_set_lanes", self.h, int(lanes))

    def set_kernel(self, kernel):
        call("xzzx_plan_set_kernel", self.h, int(kernel))

    def set_ladder(self, levels, beta_lo=0.0, beta_hi=0.0):
        """Replica exchange on ladders of `levels` fixed inverse temperatures
        from beta_lo to beta_hi (0 levels: back to the annealing schedule);
        n_rep of a decode must then be a multiple of `levels`."""
        call("xzzx_plan_set_ladder", self.h, int(levels), float(beta_lo), float(beta_hi))

    def set_order(self, order):
        """X.ORDER_COLOUR (colour-class sweeps) or X.ORDER_RANDOM_SITE (Alg. 3 as printed)."""
        call("xzzx_plan_set_order", self.h, int(order))

    def autotune(self, n_rep, n_syn=256, probe_sweeps=50, stream=None):
        """Pick the fastest result-invariant launch knobs for this plan."""
        r = X.TuneResult()
        call("xzzx_plan_autotune", self.h, n_rep, n_syn, probe_sweeps, _stream(stream), C.byref(r))
        names = ["rows"] + [f"bytes{1 << i}" for i in range(7)]
        kind = {X.KERNEL_ROWS: "rows", X.KERNEL_ROWS_GENERIC: "rows_generic", X.KERNEL_SITE: "site",
                X.KERNEL_LADDER: "ladder"}.get(r.kernel, "bytes")
        return {"kernel": kind, "lanes_per_chain": r.lanes_per_chain,
                "times_ms": {n: round(t, 3) for n, t in zip(names, r.times_ms) if t >= 0}}

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and X._lib is not None:
            X._lib.xzzx_plan_destroy(h)
            self.h = None


# ---------------------------------------------------------------------------
# device calls
# ---------------------------------------------------------------------------
def syndrome(plan: Plan, cfg: torch.Tensor, stream=None) -> torch.Tensor:
    cfg = _dev(cfg, torch.uint8, "cfg")
    n = cfg.shape[0]
    with _on(stream):
        syn = torch.empty((n, plan.nstab), dtype=torch.uint8, device=cfg.device)
    _used_on(stream, cfg)
    call("xzzx_syndrome", plan.h, _p(cfg), n, _p(syn), _stream(stream))
    return syn


def greedy_init(plan: Plan, syn, uid, n_rep, seed, mode=X.GREEDY_RANDOM, stream=None):
    syn = _dev(syn, torch.uint8, "syn")
    uid = _dev(uid, torch.int32, "uid") if uid.dtype == torch.int32 else _dev(uid, torch.uint32, "uid")
    n = syn.shape[0]
    with _on(stream):
        refs = torch.empty((n, n_rep, plan.nq), dtype=torch.uint8, device=syn.device)
        qcls = torch.empty((n, n_rep), dtype=torch.uint8, device=syn.device)
    _used_on(stream, syn, uid)
    call("xzzx_greedy_init", plan.h, _p(syn), _p(uid), n, n_rep, seed, mode, _p(refs), _p(qcls), _stream(stream))
    return refs, qcls


@dataclass
class GroupOut:
    e_best: torch.Tensor
    cls: torch.Tensor
    recovery: torch.Tensor
    paper_recovery: torch.Tensor | None = None
    e_cls: torch.Tensor | None = None
    best_chain: torch.Tensor | None = None
    refs: torch.Tensor | None = None
    qcls: torch.Tensor | None = None
    chain_emin: torch.Tensor | None = None
    chain_stop: torch.Tensor | None = None
    chain_e: torch.Tensor | None = None
    chain_final: torch.Tensor | None = None
    keep: tuple = ()   # input tensors referenced by the C descriptor (kept alive)


def make_group(plan: Plan, n_rep: int, uid: torch.Tensor, syn=None, refs=None, qcls=None,
               want_chains=False, want_final=False, want_extra=True, stream=None):
    """Allocate the outputs of one group and build its C descriptor.  With a
    stream, the outputs are allocated for work on that stream and the inputs
    are marked as used by it."""
    with _on(stream):
        g, o = _make_group(plan, n_rep, uid, syn, refs, qcls, want_chains, want_final, want_extra)
    _used_on(stream, uid, syn, refs, qcls)
    return g, o


def _make_group(plan, n_rep, uid, syn, refs, qcls, want_chains, want_final, want_extra):
    dev = uid.device
    n = uid.shape[0]
    nc = 4 * n_rep
    o = GroupOut(
        e_best=torch.empty(n, dtype=torch.int32, device=dev),
        cls=torch.empty(n, dtype=torch.uint8, device=dev),
        recovery=torch.empty((n, plan.nq), dtype=torch.uint8, device=dev),
    )
    if want_extra:
        o.paper_recovery = torch.empty((n, plan.nq), dtype=torch.uint8, device=dev)
        o.e_cls = torch.empty((n, 4), dtype=torch.int32, device=dev)
        o.best_chain = torch.empty(n, dtype=torch.int32, device=dev)
        o.refs = refs if refs is not None else torch.empty((n, n_rep, plan.nq), dtype=torch.uint8, device=dev)
        o.qcls = qcls if qcls is not None else torch.empty((n, n_rep), dtype=torch.uint8, device=dev)
    else:
        o.refs, o.qcls = refs, qcls
    if want_chains:
        o.chain_emin = torch.empty((n, nc), dtype=torch.int32, device=dev)
        o.chain_stop = torch.empty((n, nc), dtype=torch.int32, device=dev)
        o.chain_e = torch.empty((n, nc), dtype=torch.int32, device=dev)
    if want_final:
        o.chain_final = torch.empty((n, nc, plan.nq), dtype=torch.uint8, device=dev)
    o.keep = (plan, uid, syn)
    g = X.Group()
    g.plan = plan.h
    g.n_syn = n
    g.n_rep = n_rep
    g.d_uid = _p(uid).value
    g.d_syn = _p(syn).value if syn is not None else None
    for name in ("refs", "qcls", "e_best", "cls", "recovery", "paper_recovery", "e_cls", "best_chain",
                 "chain_emin", "chain_stop", "chain_e", "chain_final"):
        t = getattr(o, name)
        setattr(g, "d_" + name, _p(t).value if t is not None else None)
    return g, o


def _groups_array(groups):
    arr = (X.Group * len(groups))(*groups)
    return arr


def workspace(groups, device="cuda", stream=None):
    arr = _groups_array(groups)
    nb = C.c_size_t()
    call("xzzx_decode_workspace", arr, len(groups), C.byref(nb))
    with _on(stream):
        return torch.empty(nb.value, dtype=torch.uint8, device=device)


def decode_groups(groups, greedy_seed, anneal_seed, greedy_mode=X.GREEDY_RANDOM, flags=0, ws=None, stream=None):
    """xzzx_decode over C group descriptors; returns the workspace, which must
    stay alive until the decode's stream has completed."""
    arr = _groups_array(groups)
    if ws is None:
        ws = workspace(groups, stream=stream)
    else:
        _used_on(stream, ws)
    call("xzzx_decode", arr, len(groups), greedy_seed, anneal_seed, greedy_mode, flags, _p(ws), ws.numel(),
         _stream(stream))
    return ws


def decode_groups_noalloc(groups, greedy_seed, anneal_seed, greedy_mode=X.GREEDY_RANDOM, flags=0, stream=None):
    """xzzx_decode_noalloc: the decode with the library's static per-device
    workspace (no allocation; calls that overlap on one device race)."""
    arr = _groups_array(groups)
    call("xzzx_decode_noalloc", arr, len(groups), greedy_seed, anneal_seed, greedy_mode, flags, _stream(stream))


def anneal_groups(groups, anneal_seed, flags=0, ws=None, stream=None):
    arr = _groups_array(groups)
    if ws is None:
        ws = workspace(groups, stream=stream)
    else:
        _used_on(stream, ws)
    call("xzzx_anneal", arr, len(groups), anneal_seed, flags, _p(ws), ws.numel(), _stream(stream))
    return ws


def decode(plan: Plan, syn: torch.Tensor, uid: torch.Tensor, n_rep: int, greedy_seed: int, anneal_seed: int,
           greedy_mode=X.GREEDY_RANDOM, flags=0, want_chains=False, want_final=False, stream=None) -> GroupOut:
    """Alg. 7 for a batch of syndromes of one plan (on `stream`, default the
    current stream); the outputs are valid once that stream has completed."""
    _dev(syn, torch.uint8, "syn")
    g, o = make_group(plan, n_rep, uid, syn=syn, want_chains=want_chains, want_final=want_final, stream=stream)
    ws = decode_groups([g], greedy_seed, anneal_seed, greedy_mode, flags, stream=stream)
    o.keep = o.keep + (ws,)
    return o


class Graph:
    """One captured decode (hipGraph) over fixed buffers."""

    def __init__(self, groups, greedy_seed, anneal_seed, greedy_mode=X.GREEDY_RANDOM, flags=0, stream=None, ws=None):
        self.groups = groups
        self.arr = _groups_array(groups)
        self.ws = ws if ws is not None else workspace(groups)
        self.stream = stream if stream is not None else torch.cuda.Stream()
        h = C.c_void_p()
        call("xzzx_graph_create", self.arr, len(groups), greedy_seed, anneal_seed, greedy_mode, flags,
             _p(self.ws), self.ws.numel(), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        self.h = h

    def launch(self, stream=None):
        call("xzzx_graph_launch", self.h, _stream(stream if stream is not None else self.stream))

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and X._lib is not None:
            X._lib.xzzx_graph_destroy(h)
            self.h = None


class Server:
    """Serving loop (continuous batching) of the C ABI: submit single-syndrome
    requests, poll results, read latency/throughput statistics."""

    def __init__(self, max_slots=256, max_rep=16, max_qubits=625, sweeps_per_slice=100, max_pending=1 << 20,
                 greedy_seed=0, anneal_seed=0, greedy_mode=X.GREEDY_RANDOM, lds_budget_bytes=0,
                 max_lanes_per_chain=0, max_waves=0):
        cfg = X.ServerCfg(max_slots, max_rep, max_qubits, sweeps_per_slice, max_pending, greedy_mode,
                          lds_budget_bytes, greedy_seed, anneal_seed, max_lanes_per_chain, max_waves)
        h = C.c_void_p()
        call("xzzx_server_create", C.byref(cfg), C.byref(h))
        self.h = h
        self._plans = {}

    def submit(self, plan: Plan, syndrome: np.ndarray, uid: int, n_rep: int) -> int:
        syn = np.ascontiguousarray(syndrome, np.uint8)
        req = X.Request(plan.h, syn.ctypes.data_as(C.c_void_p), int(uid) & 0xFFFFFFFF, n_rep)
        t = C.c_uint64()
        call("xzzx_server_submit", self.h, C.byref(req), C.byref(t))
        self._plans[t.value] = plan
        return t.value

    def submit_many(self, plans, syndromes, uids, n_rep: int):
        """Queue len(plans) requests in one call (xzzx_server_submit_many);
        returns their tickets in order."""
        n = len(plans)
        if n == 0:
            return []
        syns = [np.ascontiguousarray(s, np.uint8) for s in syndromes]
        reqs = (X.Request * n)(*[X.Request(pl.h, sy.ctypes.data_as(C.c_void_p), int(u) & 0xFFFFFFFF, n_rep)
                                 for pl, sy, u in zip(plans, syns, uids)])
        tickets = (C.c_uint64 * n)()
        done = C.c_int(0)
        rc = lib().xzzx_server_submit_many(self.h, reqs, n, tickets, C.byref(done))
        for i in range(done.value):
            self._plans[tickets[i]] = plans[i]
        X.check("xzzx_server_submit_many", rc)
        return [tickets[i] for i in range(n)]

    def try_submit(self, plan, syndrome, uid, n_rep):
        """Like submit, but returns None when the queue is full (EAGAIN)."""
        syn = np.ascontiguousarray(syndrome, np.uint8)
        req = X.Request(plan.h, syn.ctypes.data_as(C.c_void_p), int(uid) & 0xFFFFFFFF, n_rep)
        t = C.c_uint64()
        rc = lib().xzzx_server_submit(self.h, C.byref(req), C.byref(t))
        if rc == X.XZZX_EAGAIN:
            return None
        X.check("xzzx_server_submit", rc)
        self._plans[t.value] = plan
        return t.value

    def poll(self, ticket: int):
        """Result dict, or None while the request is queued or resident."""
        plan = self._plans[ticket]
        rec = np.zeros(plan.nq, np.uint8)
        res = X.Result()
        res.recovery = rec.ctypes.data_as(C.c_void_p)
        rc = lib().xzzx_server_poll(self.h, C.c_uint64(ticket), C.byref(res))
        if rc == X.XZZX_ENOTREADY:
            return None
        X.check("xzzx_server_poll", rc)
        del self._plans[ticket]
        return dict(e_best=res.e_best, cls=res.cls, e_cls=list(res.e_cls), recovery=rec,
                    latency_s=res.latency_s, queue_s=res.queue_s)

    def drain(self):
        call("xzzx_server_drain", self.h)

    def stats(self):
        st = X.ServeStats()
        call("xzzx_server_stats", self.h, C.byref(st))
        return {k: getattr(st, k) for k, _ in X.ServeStats._fields_}

    def close(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and X._lib is not None:
            X._lib.xzzx_server_destroy(h)
            self.h = None

    def __del__(self):
        self.close()
