"""ctypes binding of libxzzx_sa.so (the C ABI in include/xzzx_sa.h).

Argument marshalling only: every computation happens in the library (host
plan setup in C++, per-syndrome work in the gfx950 kernels).  Loading fails
loudly when the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxzzx_sa.so")

XZZX_OK, XZZX_EINVAL, XZZX_ENOMEM, XZZX_EDEVICE, XZZX_ERANGE, XZZX_EAGAIN, XZZX_ENOTREADY = 0, -1, -2, -3, -4, -5, -6
ROTATED, PLANAR = 0, 1
BIAS_RATIO, BIAS_PAPER = 0, 1
SCHED_LINEAR, SCHED_GEOMETRIC, SCHED_PAPER_LOG = 0, 1, 2
GREEDY_RANDOM, GREEDY_SAME, GREEDY_BOUNDARY = 0, 1, 2
FLAG_PLAIN = 1
STAGE_GREEDY, STAGE_ANNEAL, STAGE_FINISH = 2, 4, 8
NOALLOC_SCRATCH_BYTES = 64 << 20   # XZZX_NOALLOC_SCRATCH_BYTES
KERNEL_AUTO, KERNEL_ROWS, KERNEL_BYTES, KERNEL_ROWS_GENERIC, KERNEL_SITE, KERNEL_LADDER = 0, 1, 2, 3, 4, 5
ORDER_COLOUR, ORDER_RANDOM_SITE = 0, 1

_STATUS = {
    XZZX_EINVAL: "EINVAL", XZZX_ENOMEM: "ENOMEM", XZZX_EDEVICE: "EDEVICE",
    XZZX_ERANGE: "ERANGE", XZZX_EAGAIN: "EAGAIN", XZZX_ENOTREADY: "ENOTREADY",
}


class XzzxError(RuntimeError):
    def __init__(self, fn, rc, msg):
        super().__init__(f"{fn} failed: {_STATUS.get(rc, rc)}: {msg}")
        self.rc = rc


class Group(C.Structure):
    _fields_ = [
        ("plan", C.c_void_p),
        ("n_syn", C.c_int64),
        ("n_rep", C.c_int),
        ("d_uid", C.c_void_p),
        ("d_syn", C.c_void_p),
        ("d_refs", C.c_void_p),
        ("d_qcls", C.c_void_p),
        ("d_e_best", C.c_void_p),
        ("d_cls", C.c_void_p),
        ("d_recovery", C.c_void_p),
        ("d_paper_recovery", C.c_void_p),
        ("d_e_cls", C.c_void_p),
        ("d_best_chain", C.c_void_p),
        ("d_chain_emin", C.c_void_p),
        ("d_chain_stop", C.c_void_p),
        ("d_chain_e", C.c_void_p),
        ("d_chain_final", C.c_void_p),
    ]


class TuneResult(C.Structure):
    _fields_ = [("kernel", C.c_int), ("lanes_per_chain", C.c_int), ("times_ms", C.c_float * 8)]


class ServerCfg(C.Structure):
    _fields_ = [
        ("max_slots", C.c_int),
        ("max_rep", C.c_int),
        ("max_qubits", C.c_int),
        ("sweeps_per_slice", C.c_int),
        ("max_pending", C.c_int),
        ("greedy_mode", C.c_int),
        ("lds_budget_bytes", C.c_int64),
        ("greedy_seed", C.c_uint64),
        ("anneal_seed", C.c_uint64),
        ("max_lanes_per_chain", C.c_int),
        ("max_waves", C.c_int),
    ]


class Request(C.Structure):
    _fields_ = [
        ("plan", C.c_void_p),
        ("syndrome", C.c_void_p),
        ("uid", C.c_uint32),
        ("n_rep", C.c_int),
    ]


class Result(C.Structure):
    _fields_ = [
        ("e_best", C.c_int32),
        ("cls", C.c_int32),
        ("e_cls", C.c_int32 * 4),
        ("recovery", C.c_void_p),
        ("latency_s", C.c_double),
        ("queue_s", C.c_double),
    ]


class ServeStats(C.Structure):
    _fields_ = [
        ("submitted", C.c_int64),
        ("completed", C.c_int64),
        ("rejected", C.c_int64),
        ("slices", C.c_int64),
        ("p50_latency_s", C.c_double),
        ("p99_latency_s", C.c_double),
        ("mean_latency_s", C.c_double),
        ("decodes_per_s", C.c_double),
        ("attempts_per_s", C.c_double),
        ("busy_s", C.c_double),
    ]


_lib = None


def lib():
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2509_17837_amd.build` "
            "(there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    V, I, I64, U32, U64, D = C.c_void_p, C.c_int, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
    P = C.POINTER
    sig = {
        "xzzx_last_error": (C.c_char_p, []),
        "xzzx_version": (I, []),
        "xzzx_lattice_create": (I, [I, I, P(V)]),
        "xzzx_lattice_destroy": (None, [V]),
        "xzzx_lattice_info": (I, [V, P(I), P(I), P(I)]),
        "xzzx_lattice_tables": (I, [V, V, V, V, V, V]),
        "xzzx_lattice_logicals": (I, [V, V, V]),
        "xzzx_noise": (I, [D, D, I, V]),
        "xzzx_weights": (I, [D, V, V, V]),
        "xzzx_schedule": (I, [I, D, D, I, V]),
        "xzzx_class_host": (I, [V, V, V, P(I)]),
        "xzzx_plan_create": (I, [V, V, V, V, I, P(V)]),
        "xzzx_plan_destroy": (None, [V]),
        "xzzx_plan_info": (I, [V, P(I), P(I), P(I), P(I), P(I), P(I)]),
        "xzzx_plan_set_lanes": (I, [V, I]),
        "xzzx_plan_set_kernel": (I, [V, I]),
        "xzzx_plan_set_order": (I, [V, I]),
        "xzzx_plan_set_ladder": (I, [V, I, C.c_double, C.c_double]),
        "xzzx_plan_autotune": (I, [V, I, I, I, V, P(TuneResult)]),
        "xzzx_syndrome": (I, [V, V, I64, V, V]),
        "xzzx_greedy_init": (I, [V, V, V, I64, I, U64, I, V, V, V]),
        "xzzx_decode_workspace": (I, [P(Group), I, P(C.c_size_t)]),
        "xzzx_decode": (I, [P(Group), I, U64, U64, I, I, V, C.c_size_t, V]),
        "xzzx_anneal": (I, [P(Group), I, U64, I, V, C.c_size_t, V]),
        "xzzx_decode_noalloc": (I, [P(Group), I, U64, U64, I, I, V]),
        "xzzx_graph_create": (I, [P(Group), I, U64, U64, I, I, V, C.c_size_t, V, P(V)]),
        "xzzx_graph_launch": (I, [V, V]),
        "xzzx_graph_destroy": (None, [V]),
        "xzzx_probe_valu": (I, [I, I, I, V, P(D)]),
        "xzzx_probe_lds": (I, [I, I, I, V, P(D)]),
        "xzzx_server_create": (I, [P(ServerCfg), P(V)]),
        "xzzx_server_submit": (I, [V, P(Request), P(U64)]),
        "xzzx_server_submit_many": (I, [V, P(Request), I, P(U64), P(C.c_int)]),
        "xzzx_server_poll": (I, [V, U64, P(Result)]),
        "xzzx_server_drain": (I, [V]),
        "xzzx_server_stats": (I, [V, P(ServeStats)]),
        "xzzx_server_destroy": (None, [V]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return _lib


def exported_symbols():
    """Names declared in include/xzzx_sa.h that the loaded library exports."""
    L = lib()
    return {n for n in dir(L) if n.startswith("xzzx_")}


def check(fn_name, rc):
    if rc != XZZX_OK:
        msg = lib().xzzx_last_error()
        raise XzzxError(fn_name, rc, msg.decode() if msg else "")
    return rc


def call(fn_name, *args):
    return check(fn_name, getattr(lib(), fn_name)(*args))
